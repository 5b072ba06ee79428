// Batched Runge-Kutta stages over many meshes of mixed order.
//
// A work list holds one item per (mesh, 16-element tile) of every mesh.  Two
// launch modes run the same tile routine a single-mesh launch runs, so a
// mesh's batched result is bitwise its single-mesh result:
//  - mixed: one persistent launch per stage walks the whole list with a
//    static stride and picks each item's order at run time.  Every block
//    first stages the face tables of each order present into LDS (they depend
//    on the order only, not on the mesh); the operator tables are read from
//    memory.  Its register budget is that of the largest order.  With
//    xcd_chunks the list is cut into 8 contiguous parts, part x walked by the
//    blocks of XCD x (blocks are dealt to XCDs round-robin), so a mesh's
//    neighbouring tiles stay in one XCD's L2; otherwise the whole grid
//    strides over the list.
//  - per order: one launch per order present and stage over that order's
//    items (the list is grouped by order), the kernel specialised for the
//    order with the single-mesh kernel's shape, its tile's state staged in
//    LDS.  The chains of different orders touch different meshes, so the
//    host runs them on forked streams.
#include "batch.hpp"
#include "internal.hpp"
#include "lowp_tile.hpp"

namespace dg {
namespace {

using namespace lowp;

constexpr int kXcds = 8;

template <int MODE, int WPB>
__global__ __launch_bounds__(64 * WPB) __attribute__((amdgpu_waves_per_eu(2))) void batch_stage_kernel(
    BatchLaunch L, double a, double b, int odd) {
  extern __shared__ __align__(16) uint8_t lds[];
  for (int p = 1; p <= 4; ++p) {
    uint8_t* nb = lds + L.tabs.nb_off[p];
    for (int i = threadIdx.x; i < L.tabs.nb_bytes[p]; i += blockDim.x) nb[i] = L.tabs.nb[p][i];
    int* fm = reinterpret_cast<int*>(lds + L.tabs.fm_off[p]);
    for (int i = threadIdx.x; i < L.tabs.fm_n[p]; i += blockDim.x) fm[i] = L.tabs.fm[p][i];
  }
  __syncthreads();

  const int wave = __builtin_amdgcn_readfirstlane(threadIdx.x >> 6);  // wave-uniform: tile values in scalar registers
  int64_t begin, end, first, stride;
  if (L.xcd_chunks) {
    const int xcd = blockIdx.x % kXcds;
    const int slot = blockIdx.x / kXcds;
    const int nslots = (static_cast<int>(gridDim.x) - xcd + kXcds - 1) / kXcds;
    begin = L.n_items * xcd / kXcds;
    end = L.n_items * (xcd + 1) / kXcds;
    first = begin + static_cast<int64_t>(slot) * WPB + wave;
    stride = static_cast<int64_t>(nslots) * WPB;
  } else {
    begin = 0;
    end = L.n_items;
    first = static_cast<int64_t>(blockIdx.x) * WPB + wave;
    stride = static_cast<int64_t>(gridDim.x) * WPB;
  }
  for (int64_t i = first; i < end; i += stride) {
    const BatchItem it = L.items[i];
    const BatchMesh& M = L.meshes[it.mesh];
    LowArgs A;
    A.q = odd ? M.tmp : M.q;
    A.qout = odd ? M.q : M.tmp;
    A.res_in = M.res;
    A.res = M.res;
    A.rhs = nullptr;
    A.geo = M.geo;
    A.conn = M.conn;
    A.op32 = nullptr;
    A.opbf = nullptr;
    A.fmask = nullptr;
    A.nbtab = nullptr;
    A.E = M.E;
    A.Epad = M.Epad;
    A.ntiles = static_cast<int>(M.Epad / 16);
    A.xcd_run = 1;
    A.gamma = L.gamma;
    A.a = a;
    A.b = b;
    A.dt = L.dt[it.mesh];
    A.flags = L.flags;
    const int p = M.p;
    const uint32_t* op = L.tabs.op[p];
    const uint8_t* nb = lds + L.tabs.nb_off[p];
    const int* fm = reinterpret_cast<const int*>(lds + L.tabs.fm_off[p]);
    switch (p) {
      case 1: lowp_tile<1, MODE, true>(A, op, nb, fm, it.tile); break;
      case 2: lowp_tile<2, MODE, true>(A, op, nb, fm, it.tile); break;
      case 3: lowp_tile<3, MODE, true>(A, op, nb, fm, it.tile); break;
      default: lowp_tile<4, MODE, true>(A, op, nb, fm, it.tile); break;
    }
  }
}

// Per-order kernel: the items [p_begin[P], p_end[P]) all have order P; one
// wave per item, its tile's state staged in LDS, the register budget of this
// order alone (the single-mesh kernel's launch shape: one-tile blocks and
// face tables read from memory at p = 4).
template <int P>
constexpr int order_waves() { return P >= 4 ? 1 : 4; }

template <int P, int MODE>
__global__ __launch_bounds__(256) __attribute__((amdgpu_waves_per_eu(P < 4 ? 3 : 2))) void batch_order_kernel(
    BatchLaunch L, double a, double b, int odd) {
  using C = LCfg<P>;
  constexpr int W = order_waves<P>();
  __shared__ double s_q[W][5 * 16 * C::NP];
  __shared__ __align__(4) uint8_t s_nbl[lowp_lds_tables<P>() ? 4 * 24 * C::NFP : 4];
  __shared__ int s_fml[lowp_lds_tables<P>() ? 4 * C::NFP : 1];
  if constexpr (lowp_lds_tables<P>()) {
    stage_face_tables<C::NFP, 64 * W>(s_nbl, s_fml, L.tabs.nb[P], L.tabs.fm[P], threadIdx.x);
    __syncthreads();
  }
  const uint8_t* s_nb = lowp_lds_tables<P>() ? s_nbl : L.tabs.nb[P];
  const int* s_fm = lowp_lds_tables<P>() ? s_fml : L.tabs.fm[P];
  const int wave = __builtin_amdgcn_readfirstlane(threadIdx.x >> 6);  // wave-uniform: tile values in scalar registers
  const int64_t i = L.p_begin[P] + static_cast<int64_t>(blockIdx.x) * W + wave;
  if (i >= L.p_end[P]) return;
  const BatchItem it = L.items[i];
  const BatchMesh& M = L.meshes[it.mesh];
  LowArgs A;
  A.q = odd ? M.tmp : M.q;
  A.qout = odd ? M.q : M.tmp;
  A.res_in = M.res;
  A.res = M.res;
  A.rhs = nullptr;
  A.geo = M.geo;
  A.conn = M.conn;
  A.op32 = nullptr;
  A.opbf = nullptr;
  A.fmask = nullptr;
  A.nbtab = nullptr;
  A.E = M.E;
  A.Epad = M.Epad;
  A.ntiles = static_cast<int>(M.Epad / 16);
  A.xcd_run = 1;
  A.gamma = L.gamma;
  A.a = a;
  A.b = b;
  A.dt = L.dt[it.mesh];
  A.flags = L.flags;
  lowp_tile<P, MODE, true, true>(A, L.tabs.op[P], s_nb, s_fm, it.tile, s_q[wave]);
}

template <int P, int MODE>
void launch_order(const BatchLaunch& L, double a, double b, int odd, hipStream_t s) {
  const int64_t count = L.p_end[P] - L.p_begin[P];
  if (count <= 0) return;
  constexpr int W = order_waves<P>();
  batch_order_kernel<P, MODE><<<static_cast<unsigned>((count + W - 1) / W), 64 * W, 0, s>>>(L, a, b, odd);
}

// q <- tmp over the elements of items [begin, end): one wave per item, the
// tile's 16 Np contiguous values of each field.
__global__ __launch_bounds__(256) void batch_copy_kernel(BatchLaunch L, int64_t begin, int64_t end) {
  const int lane = threadIdx.x & 63;
  const int64_t waves = static_cast<int64_t>(gridDim.x) * (blockDim.x >> 6);
  for (int64_t i = begin + static_cast<int64_t>(blockIdx.x) * (blockDim.x >> 6) + (threadIdx.x >> 6); i < end;
       i += waves) {
    const BatchItem it = L.items[i];
    const BatchMesh& M = L.meshes[it.mesh];
    const int np = (M.p + 1) * (M.p + 2) * (M.p + 3) / 6;
    const int64_t e0 = static_cast<int64_t>(it.tile) * 16;
    const int64_t ne = M.E - e0 < 16 ? M.E - e0 : 16;
    const int64_t len = ne * np;
    const int64_t Es = M.E * np;
    for (int f = 0; f < 5; ++f) {
      const int64_t base = f * Es + e0 * np;
      for (int64_t k = lane; k < len; k += 64) M.q[base + k] = M.tmp[base + k];
    }
  }
}

template <int MODE>
const void* stage_kernel(int wpb) {
  switch (wpb) {
    case 2: return reinterpret_cast<const void*>(&batch_stage_kernel<MODE, 2>);
    case 4: return reinterpret_cast<const void*>(&batch_stage_kernel<MODE, 4>);
    case 8: return reinterpret_cast<const void*>(&batch_stage_kernel<MODE, 8>);
    default: return nullptr;
  }
}

const void* stage_kernel(dg_precision prec, int wpb) {
  if (prec == DG_FP32) return stage_kernel<1>(wpb);
  if (prec == DG_SPLIT_BF16) return stage_kernel<2>(wpb);
  return nullptr;
}

template <int MODE>
void launch_order_mode(const BatchLaunch& L, int p, double a, double b, int odd, hipStream_t s) {
  switch (p) {
    case 1: launch_order<1, MODE>(L, a, b, odd, s); break;
    case 2: launch_order<2, MODE>(L, a, b, odd, s); break;
    case 3: launch_order<3, MODE>(L, a, b, odd, s); break;
    default: launch_order<4, MODE>(L, a, b, odd, s); break;
  }
}

template <int MODE>
void launch_mode(const BatchLaunch& L, double a, double b, int odd, hipStream_t s) {
  const dim3 grid(L.blocks), block(64 * L.waves_per_block);
  const size_t lds = L.tabs.lds_bytes;
  switch (L.waves_per_block) {
    case 2: batch_stage_kernel<MODE, 2><<<grid, block, lds, s>>>(L, a, b, odd); break;
    case 4: batch_stage_kernel<MODE, 4><<<grid, block, lds, s>>>(L, a, b, odd); break;
    default: batch_stage_kernel<MODE, 8><<<grid, block, lds, s>>>(L, a, b, odd); break;
  }
}

}  // namespace

int batch_stage_occupancy(dg_precision prec, int waves_per_block, int lds_bytes) {
  const void* k = stage_kernel(prec, waves_per_block);
  if (!k) return 0;
  int nb = 0;
  if (hipOccupancyMaxActiveBlocksPerMultiprocessor(&nb, k, 64 * waves_per_block, lds_bytes) != hipSuccess) return 0;
  return nb;
}

dg_status batch_prepare(dg_precision prec, int waves_per_block, int lds_bytes) {
  const void* k = stage_kernel(prec, waves_per_block);
  if (!k) return fail(DG_ERR_ARG, "batch: waves_per_block must be 2, 4 or 8");
  DG_HIP(hipFuncSetAttribute(k, hipFuncAttributeMaxDynamicSharedMemorySize, lds_bytes));
  return DG_OK;
}

dg_status launch_batch_stage(dg_precision prec, const BatchLaunch& L, double a, double b, int odd, hipStream_t s) {
  if (L.waves_per_block != 2 && L.waves_per_block != 4 && L.waves_per_block != 8)
    return fail(DG_ERR_ARG, "batch: waves_per_block must be 2, 4 or 8");
  if (L.n_items == 0) return DG_OK;
  if (prec == DG_FP32)
    launch_mode<1>(L, a, b, odd, s);
  else if (prec == DG_SPLIT_BF16)
    launch_mode<2>(L, a, b, odd, s);
  else
    return fail(DG_ERR_UNSUPPORTED, "batch: contraction precision must be DG_FP32 or DG_SPLIT_BF16");
  DG_HIP(hipGetLastError());
  return DG_OK;
}

dg_status launch_batch_order_stage(dg_precision prec, const BatchLaunch& L, int p, double a, double b, int odd,
                                   hipStream_t s) {
  if (p < 1 || p > 4) return fail(DG_ERR_ARG, "batch: order must be 1..4");
  if (L.p_end[p] <= L.p_begin[p]) return DG_OK;
  if (prec == DG_FP32)
    launch_order_mode<1>(L, p, a, b, odd, s);
  else if (prec == DG_SPLIT_BF16)
    launch_order_mode<2>(L, p, a, b, odd, s);
  else
    return fail(DG_ERR_UNSUPPORTED, "batch: contraction precision must be DG_FP32 or DG_SPLIT_BF16");
  DG_HIP(hipGetLastError());
  return DG_OK;
}

dg_status launch_batch_copy(const BatchLaunch& L, int64_t begin, int64_t end, hipStream_t s) {
  if (end <= begin) return DG_OK;
  int64_t blocks = (end - begin + 3) / 4;
  if (blocks > 256 * 16) blocks = 256 * 16;
  batch_copy_kernel<<<static_cast<unsigned>(blocks), 256, 0, s>>>(L, begin, end);
  DG_HIP(hipGetLastError());
  return DG_OK;
}

}  // namespace dg
