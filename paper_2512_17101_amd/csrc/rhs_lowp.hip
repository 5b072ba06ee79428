// Euler right-hand side with reduced-precision element contractions, gfx950:
// the single-mesh kernel over the tile routine of lowp_tile.hpp, one wave per
// 16-element tile with the tile's state staged in LDS.
#include "internal.hpp"
#include "lowp_tile.hpp"

namespace dg {
namespace {

using namespace lowp;

// W waves per block (one 16-element tile each; the tile's state is staged in
// LDS, 5 x 16 Np doubles per wave: two or four up to p = 3, as the mesh's
// launch configuration says) and the register target: three waves per SIMD
// up to p = 3, two at p = 4.  At p = 4 the state tile alone is 22.4 KB, so
// LDS bounds the waves per CU: one-tile blocks with the face tables read from
// memory (cache-resident) fit seven per CU against six for two-tile blocks
// with LDS tables (measured 9-10 % faster).
template <int P, int MODE>
constexpr int lowp_wpe() { return P < 4 ? 3 : 2; }

template <int P, int MODE, bool FUSED, int W, bool DMA>
__global__ __launch_bounds__(64 * W) __attribute__((amdgpu_waves_per_eu(lowp_wpe<P, MODE>()))) void rhs_euler_lowp_kernel(
    LowArgs A) {
  using C = LCfg<P>;
  __shared__ __align__(512) double s_q[W][5 * 16 * C::NP];  // 512-byte bases for the LDS DMA path
  __shared__ __align__(4) uint8_t s_nbl[lowp_lds_tables<P>() ? 4 * 24 * C::NFP : 4];
  __shared__ int s_fml[lowp_lds_tables<P>() ? 4 * C::NFP : 1];
  if constexpr (lowp_lds_tables<P>()) {
    stage_face_tables<C::NFP, 64 * W>(s_nbl, s_fml, A.nbtab, A.fmask, threadIdx.x);
    __syncthreads();
  }
  const uint8_t* s_nb = lowp_lds_tables<P>() ? s_nbl : A.nbtab;
  const int* s_fm = lowp_lds_tables<P>() ? s_fml : A.fmask;
  // the operator table is read from memory (cache-resident): LDS holds the states
  const uint32_t* op = MODE == 1 ? reinterpret_cast<const uint32_t*>(A.op32) : reinterpret_cast<const uint32_t*>(A.opbf);
  const int wave = __builtin_amdgcn_readfirstlane(threadIdx.x >> 6);  // wave-uniform: tile values in scalar registers
  const int64_t tile = static_cast<int64_t>(xcd_run_block(blockIdx.x, gridDim.x, A.xcd_run)) * W + wave;
  if (tile < A.ntiles) lowp_tile<P, MODE, FUSED, true, DMA>(A, op, s_nb, s_fm, tile, s_q[wave]);
}

// FP32 contractions: the tile is staged through the LDS DMA path where Np is
// a multiple of 4 (p = 1, 3) and q is 16-byte aligned, as in the FP64
// kernel.  Split BF16 keeps register staging: with the DMA path its kernel
// spills about 500 bytes per lane and runs at half speed.
template <int P, int MODE, int W>
void launch_lowp_pw(const Mesh& m, const LowArgs& args, bool fused, hipStream_t s) {
  const int blocks = static_cast<int>((m.Epad / 16 + W - 1) / W);
  constexpr bool kDma = LCfg<P>::NP % 4 == 0 && MODE == 1;
  const bool dma = kDma && (reinterpret_cast<uintptr_t>(args.q) & 15u) == 0 && m.launch[MODE].lds_stage;
  if (dma) {
    if (fused)
      rhs_euler_lowp_kernel<P, MODE, true, W, kDma><<<blocks, 64 * W, 0, s>>>(args);
    else
      rhs_euler_lowp_kernel<P, MODE, false, W, kDma><<<blocks, 64 * W, 0, s>>>(args);
  } else {
    if (fused)
      rhs_euler_lowp_kernel<P, MODE, true, W, false><<<blocks, 64 * W, 0, s>>>(args);
    else
      rhs_euler_lowp_kernel<P, MODE, false, W, false><<<blocks, 64 * W, 0, s>>>(args);
  }
}

template <int P, int MODE>
dg_status launch_lowp_p(const Mesh& m, const LowArgs& args, bool fused, hipStream_t s) {
  if constexpr (P >= 4)
    launch_lowp_pw<P, MODE, 1>(m, args, fused, s);
  else if (m.launch[MODE].waves_per_block == 4)
    launch_lowp_pw<P, MODE, 4>(m, args, fused, s);
  else
    launch_lowp_pw<P, MODE, 2>(m, args, fused, s);
  DG_HIP(hipGetLastError());
  return DG_OK;
}

template <int MODE>
dg_status launch_mode(const Mesh& m, const LowArgs& A, bool fused, hipStream_t s) {
  switch (m.p) {
    case 1: return launch_lowp_p<1, MODE>(m, A, fused, s);
    case 2: return launch_lowp_p<2, MODE>(m, A, fused, s);
    case 3: return launch_lowp_p<3, MODE>(m, A, fused, s);
    case 4: return launch_lowp_p<4, MODE>(m, A, fused, s);
    default: return fail(DG_ERR_ARG, "rhs: unsupported order");
  }
}

}  // namespace

LowpLayout lowp_layout(int p) {
  LowpLayout L{};
  L.Np = nodes_of(p);
  L.Nfp = face_nodes_of(p);
  L.NPP = (L.Np + 3) / 4 * 4;
  L.KV = L.NPP / 4;
  L.KL = L.Nfp;
  L.NR = (L.Np + 15) / 16;
  L.REM4 = L.Np % 16 != 0 && L.Np % 16 <= 4 && L.NR <= 2;
  L.KS32 = 3 * L.KV + L.KL;
  L.VKS = (3 * L.KV + 7) / 8;
  L.FKS = (L.KL + 7) / 8;
  return L;
}

dg_status launch_rhs_euler_lowp(const Mesh& m, dg_precision prec, double gamma, const double* q, double* rhs,
                                const double* res_in, double* res, double* q_out, double a, double b, double dt,
                                bool fused, hipStream_t s) {
  LowArgs A;
  A.q = q;
  A.rhs = rhs;
  A.res_in = res_in;
  A.res = res;
  A.qout = q_out;
  A.geo = m.d_geo;
  A.conn = m.d_conn;
  A.op32 = m.d_op32;
  A.opbf = m.d_opbf;
  A.fmask = m.d_fmask;
  A.nbtab = m.d_nbtab;
  A.E = m.E;
  A.Epad = m.Epad;
  A.ntiles = static_cast<int>(m.Epad / 16);
  A.xcd_run = m.launch[prec == DG_SPLIT_BF16 ? DG_SPLIT_BF16 : DG_FP32].xcd_run;
  A.gamma = gamma;
  A.a = a;
  A.b = b;
  A.dt = dt;
  A.flags = device_flags();
  if (prec == DG_FP32) return launch_mode<1>(m, A, fused, s);
  if (prec == DG_SPLIT_BF16) return launch_mode<2>(m, A, fused, s);
  return fail(DG_ERR_ARG, "rhs: unknown precision");
}

}  // namespace dg
