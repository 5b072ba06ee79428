// Euler right-hand side with reduced-precision element contractions, gfx950:
// the single-mesh persistent kernel over the tile routine of lowp_tile.hpp.
#include "internal.hpp"
#include "lowp_tile.hpp"

namespace dg {
namespace {

using namespace lowp;

constexpr int kWaves = 4;
constexpr int kXcds = 8;

template <int P, int MODE, bool FUSED>
__global__ __launch_bounds__(256) __attribute__((amdgpu_waves_per_eu(2))) void rhs_euler_lowp_kernel(LowArgs A) {
  using C = LCfg<P>;
  constexpr int OPN = MODE == 1 ? C::OP32 : C::OPBF / 2;  // 32-bit words
  __shared__ uint32_t s_op[OPN];
  __shared__ uint8_t s_nb[4 * 24 * C::NFP];
  __shared__ int s_fm[4 * C::NFP];
  {
    const uint32_t* src = MODE == 1 ? reinterpret_cast<const uint32_t*>(A.op32)
                                    : reinterpret_cast<const uint32_t*>(A.opbf);
    for (int i = threadIdx.x; i < OPN; i += blockDim.x) s_op[i] = src[i];
    for (int i = threadIdx.x; i < 4 * 24 * C::NFP; i += blockDim.x) s_nb[i] = A.nbtab[i];
    for (int i = threadIdx.x; i < 4 * C::NFP; i += blockDim.x) s_fm[i] = A.fmask[i];
  }
  __syncthreads();
  const int wave = threadIdx.x >> 6;
  const int xcd = blockIdx.x % kXcds;
  const int slot = blockIdx.x / kXcds;
  const int nslots = (static_cast<int>(gridDim.x) - xcd + kXcds - 1) / kXcds;
  const int64_t T = A.ntiles;
  const int64_t t_begin = T * xcd / kXcds, t_end = T * (xcd + 1) / kXcds;
  for (int64_t tile = t_begin + slot * kWaves + wave; tile < t_end; tile += static_cast<int64_t>(nslots) * kWaves)
    lowp_tile<P, MODE, FUSED>(A, s_op, s_nb, s_fm, tile);
}

template <int P, int MODE, bool FUSED>
int lowp_grid(const Mesh& m) {
  static int blocks_per_cu = -1;
  static int cus = 0;
  if (blocks_per_cu < 0) {
    int nb = 0;
    if (hipOccupancyMaxActiveBlocksPerMultiprocessor(&nb, rhs_euler_lowp_kernel<P, MODE, FUSED>, 64 * kWaves, 0) !=
            hipSuccess || nb < 1)
      nb = 1;
    hipDeviceProp_t prop;
    cus = hipGetDeviceProperties(&prop, m.device) == hipSuccess ? prop.multiProcessorCount : 256;
    blocks_per_cu = nb;
  }
  const int64_t tiles = m.Epad / 16;
  const int64_t needed = (tiles + kWaves - 1) / kWaves;
  int64_t grid = static_cast<int64_t>(blocks_per_cu) * cus;
  if (grid > needed) grid = (needed + kXcds - 1) / kXcds * kXcds;
  return static_cast<int>(grid < 1 ? 1 : grid);
}

template <int P, int MODE>
dg_status launch_lowp_p(const Mesh& m, const LowArgs& args, bool fused, hipStream_t s) {
  if (fused)
    rhs_euler_lowp_kernel<P, MODE, true><<<lowp_grid<P, MODE, true>(m), 64 * kWaves, 0, s>>>(args);
  else
    rhs_euler_lowp_kernel<P, MODE, false><<<lowp_grid<P, MODE, false>(m), 64 * kWaves, 0, s>>>(args);
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
  L.KS32 = 3 * L.KV + L.KL;
  L.VKS = (3 * L.KV + 7) / 8;
  L.FKS = (L.KL + 7) / 8;
  return L;
}

dg_status launch_rhs_euler_lowp(const Mesh& m, dg_precision prec, double gamma, const double* q, double* rhs,
                                double* res, double* q_out, double a, double b, double dt, bool fused,
                                hipStream_t s) {
  LowArgs A;
  A.q = q;
  A.rhs = rhs;
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
  A.gamma = gamma;
  A.a = a;
  A.b = b;
  A.dt = dt;
  if (prec == DG_FP32) return launch_mode<1>(m, A, fused, s);
  if (prec == DG_SPLIT_BF16) return launch_mode<2>(m, A, fused, s);
  return fail(DG_ERR_ARG, "rhs: unknown precision");
}

}  // namespace dg
