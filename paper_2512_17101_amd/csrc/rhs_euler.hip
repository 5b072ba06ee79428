// Strong-form nodal DG right-hand side of the Euler equations on affine
// tetrahedra, FP64, for gfx950.
//
// One wave owns a tile of 16 elements.  Lane l works for element n = l % 16 of
// the tile and node/face-node residue g = l / 16 (mod 4).  The element-local
// contraction
//     rhs = [-Dr | -Ds | -Dt | LIFT] * [G_r; G_s; G_t; Delta]
// runs on the FP64 matrix cores: the K axis is stepped 4 at a time, lane
// (n, g) supplying the B-operand entry k = 4 ks + g of element n, which is the
// contravariant flux G_a of node j = 4 s + g (volume part) or the scaled
// Lax-Friedrichs jump Delta of face node 4 s + g (lift part).  Rows 0..15 use
// the 16x16x4 tile, the remaining rows 4x4x4 tiles fed from the same B
// register, so no row padding beyond a multiple of 4 is multiplied.
//
// Volume (pointwise, FP64):  u = m / rho,  p = (gamma - 1)(E - m.u / 2),
//   U_a = grad a . u,  G_a = (rho U_a, m U_a + p grad a, (E + p) U_a).
// Surface, with N = Fscale n taken from the metric (f0: -grad t, f1: -grad s,
//   f2: grad r + grad s + grad t, f3: -grad r), U_n = N . u:
//   Delta = 1/2 (N.F(q-) - N.F(q+)) - 1/2 max(|U_n-| + c- |N|, |U_n+| + c+ |N|) (q- - q+).
// Fused Runge-Kutta epilogue (stage of the 2N-storage scheme):
//   res <- a res + dt rhs;  q_out <- q + b res   (q_out is a second buffer,
//   because neighbouring tiles still read q; the tile's q comes from its
//   LDS copy, not from memory).
#include "euler_point.hpp"
#include "internal.hpp"

typedef double v4d __attribute__((ext_vector_type(4)));

namespace dg {
namespace {

template <int P>
struct Cfg {
  static constexpr int NP = (P + 1) * (P + 2) * (P + 3) / 6;
  static constexpr int NFP = (P + 1) * (P + 2) / 2;
  static constexpr int NPP = (NP + 3) / 4 * 4;
  static constexpr int NB16 = NP / 16;
  static constexpr int NB4 = (NP - 16 * NB16 + 3) / 4;
  static constexpr int NRB = NB16 + NB4;
  static constexpr int KV = NPP / 4;
  static constexpr int KL = NFP;
};

struct RhsArgs {
  const double* __restrict__ q;
  double* __restrict__ rhs;
  const double* res_in;  // residual read by the fused stage (may alias res or qout)
  double* res;           // residual written by the fused stage (null: not stored)
  double* qout;
  const double* __restrict__ geo;
  const int2* __restrict__ conn;
  const double* __restrict__ op;
  const int* __restrict__ fmask;
  const uint8_t* __restrict__ nbtab;
  int64_t E, Epad;
  int ntiles;
  int dma;  // q is 16-byte aligned and the launch configuration asks for the LDS DMA staging
  int xcd_run;  // blocks per XCD run (1: plain order)
  double gamma, a, b, dt;
  unsigned* flags;  // device failure flags (non-finite output)
};

// Waves (tiles) per block W: the per-wave state tile lives in LDS (5 fields
// x 16 elements x Np doubles), so order 4 runs two-wave blocks only; up to
// p = 3 the mesh's launch configuration picks two or four.  The operator
// table is read from memory (it stays in the L1/L2 caches): keeping it in LDS
// as well would cap the kernel at two waves per SIMD (measured slower at p = 3
// than the three waves per SIMD this layout allows).
template <int P, int W>
struct Tiling {
  using C = Cfg<P>;
  static constexpr int WAVES = W;
  static constexpr int TQ = 16 * C::NP;  // doubles of one field of one tile
};

// Register budget for three waves per SIMD (two at p = 4, whose tile would
// spill): measured at p = 3, the scheduling
// this target produces runs 28 % faster than the unconstrained default.
template <int P, bool FUSED, int W, bool DMA>
__global__ __launch_bounds__(64 * W) __attribute__((amdgpu_waves_per_eu(P >= 4 ? 2 : 3))) void rhs_euler_fp64_kernel(RhsArgs A) {
  using C = Cfg<P>;
  using TL = Tiling<P, W>;
  constexpr int NB16 = C::NB16 > 0 ? C::NB16 : 1;
  constexpr int NB4 = C::NB4 > 0 ? C::NB4 : 1;
  __shared__ __align__(512) double s_q[TL::WAVES][5 * TL::TQ];  // 512-byte bases for the LDS DMA path
  __shared__ __align__(4) uint8_t s_nb[4 * 24 * C::NFP];
  __shared__ int s_fm[4 * C::NFP];
  stage_face_tables<C::NFP, 64 * W>(s_nb, s_fm, A.nbtab, A.fmask, threadIdx.x);
  __syncthreads();
  const double* __restrict__ op = A.op;

  const int lane = threadIdx.x & 63;
  const int wave = __builtin_amdgcn_readfirstlane(threadIdx.x >> 6);  // wave-uniform: tile values in scalar registers
  const int tile = xcd_run_block(blockIdx.x, gridDim.x, A.xcd_run) * TL::WAVES + wave;
  if (tile >= A.ntiles) return;  // uniform per wave; no block barrier follows
  const int n = lane & 15, g = lane >> 4;
  const int64_t e0 = static_cast<int64_t>(tile) * 16;
  const int64_t e = e0 + n;
  const bool valid = e < A.E;
  const int64_t ec = valid ? e : A.E - 1;
  const int64_t Es = A.E * C::NP;
  const double* __restrict__ q = A.q;
  const double gm1 = A.gamma - 1.0;
  double* sq = s_q[wave];

  // metric and connectivity requested first, then this tile's state staged
  // (coalesced: each field's tile block is contiguous), straight into LDS in
  // the DMA instantiation (measured at p = 3: 2 % faster for the RHS, 4 % for
  // the fused Runge-Kutta stages; selecting the path with a run-time flag
  // inside one kernel was 7 % slower than either).  The DMA path exists only
  // where every destination base is a multiple of 512 bytes (Np a multiple
  // of 4: p = 1, 3): at p = 2 (1,280-byte field blocks) it gave wrong values.
  const int nval = static_cast<int>(A.E - e0 < 16 ? A.E - e0 : 16) * C::NP;
  double gm[9];
#pragma unroll
  for (int c = 0; c < 9; ++c) gm[c] = A.geo[c * A.Epad + ec];
  int2 cn[4];
#pragma unroll
  for (int f = 0; f < 4; ++f) cn[f] = A.conn[f * A.Epad + ec];
  if constexpr (DMA)
    stage_tile_dma<TL::TQ>(sq, q, Es, e0 * C::NP, nval, lane);
  else
    stage_tile<TL::TQ>(sq, q, Es, e0 * C::NP, nval, lane);
  __builtin_amdgcn_wave_barrier();
  const int nl = valid ? n : static_cast<int>(ec - e0);  // element row in the tile

  v4d acc16[5][NB16];
  double acc4[5][NB4];
#pragma unroll
  for (int f = 0; f < 5; ++f) {
#pragma unroll
    for (int r = 0; r < NB16; ++r) acc16[f][r] = v4d{0.0, 0.0, 0.0, 0.0};
#pragma unroll
    for (int r = 0; r < NB4; ++r) acc4[f][r] = 0.0;
  }

  // ---- volume: contravariant fluxes of node j = 4 s + g, contracted with -D_a
#pragma unroll
  for (int s = 0; s < C::KV; ++s) {
    const int j = 4 * s + g;
    double G[3][5];
    if (j < C::NP) {
      double qq[5];
#pragma unroll
      for (int f = 0; f < 5; ++f) qq[f] = sq[f * TL::TQ + nl * C::NP + j];
      contravariant_flux(qq, gm, gm1, G);
    } else {
#pragma unroll
      for (int r = 0; r < 3; ++r)
#pragma unroll
        for (int f = 0; f < 5; ++f) G[r][f] = 0.0;
    }
#pragma unroll
    for (int r = 0; r < 3; ++r) {
#pragma unroll
      for (int rb = 0; rb < C::NRB; ++rb) {
        const double a = op[((r * C::KV + s) * C::NRB + rb) * 64 + lane];
        if (rb < C::NB16) {
#pragma unroll
          for (int f = 0; f < 5; ++f)
            acc16[f][rb] = __builtin_amdgcn_mfma_f64_16x16x4f64(a, G[r][f], acc16[f][rb], 0, 0, 0);
        } else {
#pragma unroll
          for (int f = 0; f < 5; ++f)
            acc4[f][rb - C::NB16] = __builtin_amdgcn_mfma_f64_4x4x4f64(a, G[r][f], acc4[f][rb - C::NB16], 0, 0, 0);
        }
      }
    }
  }

  // ---- surface: Lax-Friedrichs jump at face node fm = 4 s + g, contracted with LIFT;
  // own traces from the staged tile, neighbour traces from it when the
  // neighbour is in the tile, else from memory
#pragma unroll
  for (int s = 0; s < C::KL; ++s) {
    const int fm = 4 * s + g;
    const int face = fm / C::NFP;
    const int mm = fm - face * C::NFP;
    const int own = s_fm[fm];
    const int2 c = face == 0 ? cn[0] : face == 1 ? cn[1] : face == 2 ? cn[2] : cn[3];
    const int jp = s_nb[(face * 24 + c.y) * C::NFP + mm];
    const int64_t nloc = static_cast<int64_t>(c.x) - e0;
    const bool in_tile = nloc >= 0 && nloc < 16;
    double qm[5], qp[5];
#pragma unroll
    for (int f = 0; f < 5; ++f) {
      qm[f] = sq[f * TL::TQ + nl * C::NP + own];
      qp[f] = in_tile ? sq[f * TL::TQ + static_cast<int>(nloc) * C::NP + jp]
                      : q[f * Es + static_cast<int64_t>(c.x) * C::NP + jp];
    }
    double Nx, Ny, Nz, D[5];
    step_normal<C::NFP>(s, face, gm, Nx, Ny, Nz);
    lf_jump(qm, qp, Nx, Ny, Nz, A.gamma, D);
#pragma unroll
    for (int rb = 0; rb < C::NRB; ++rb) {
      const double a = op[((3 * C::KV + s) * C::NRB + rb) * 64 + lane];
      if (rb < C::NB16) {
#pragma unroll
        for (int f = 0; f < 5; ++f)
          acc16[f][rb] = __builtin_amdgcn_mfma_f64_16x16x4f64(a, D[f], acc16[f][rb], 0, 0, 0);
      } else {
#pragma unroll
        for (int f = 0; f < 5; ++f)
          acc4[f][rb - C::NB16] = __builtin_amdgcn_mfma_f64_4x4x4f64(a, D[f], acc4[f][rb - C::NB16], 0, 0, 0);
      }
    }
  }

  // ---- store through this wave's LDS tile buffer (the state is no longer
  // needed there; the fused stage first takes its share of it into
  // registers): lane (n, g) holds rows 16 rb + 4 v + g and 16 NB16 + 4 rb4 + g
  // of element n; the tile's outputs of one field are contiguous in memory,
  // so they leave with coalesced stores.
  constexpr int KN = (TL::TQ + 63) / 64;
  double qv[FUSED ? 5 : 1][FUSED ? KN : 1];
  if constexpr (FUSED) tile_from_lds<TL::TQ>(sq, nval, lane, qv);
  __builtin_amdgcn_wave_barrier();
  if (valid) {
#pragma unroll
    for (int f = 0; f < 5; ++f) {
#pragma unroll
      for (int rb = 0; rb < C::NB16; ++rb)
#pragma unroll
        for (int v = 0; v < 4; ++v) sq[f * TL::TQ + n * C::NP + 16 * rb + 4 * v + g] = acc16[f][rb][v];
#pragma unroll
      for (int rb = 0; rb < C::NB4; ++rb) {
        const int row = 16 * C::NB16 + 4 * rb + g;
        if (row < C::NP) sq[f * TL::TQ + n * C::NP + row] = acc4[f][rb];
      }
    }
  }
  __builtin_amdgcn_wave_barrier();
  if constexpr (FUSED)
    store_tile_stage<TL::TQ>(sq, qv, nval, e0 * C::NP, Es, lane, A.res_in, A.res, A.qout, A.a, A.b, A.dt, A.flags);
  else
    store_tile<false, TL::TQ>(sq, nval, e0 * C::NP, Es, lane, A.rhs, A.res_in, A.res, A.qout, q, A.a, A.b, A.dt,
                              A.flags);
}

template <int P, int W>
void launch_pw(const RhsArgs& args, bool fused, hipStream_t s) {
  const int blocks = (args.ntiles + W - 1) / W;
  constexpr bool kDma = Cfg<P>::NP % 4 == 0;  // the DMA path exists where Np is a multiple of 4
  if (kDma && args.dma) {
    if (fused)
      rhs_euler_fp64_kernel<P, true, W, kDma><<<blocks, 64 * W, 0, s>>>(args);
    else
      rhs_euler_fp64_kernel<P, false, W, kDma><<<blocks, 64 * W, 0, s>>>(args);
  } else {
    if (fused)
      rhs_euler_fp64_kernel<P, true, W, false><<<blocks, 64 * W, 0, s>>>(args);
    else
      rhs_euler_fp64_kernel<P, false, W, false><<<blocks, 64 * W, 0, s>>>(args);
  }
}

template <int P>
dg_status launch_p(const Mesh& m, const RhsArgs& args, bool fused, hipStream_t s) {
  if (P < 4 && m.launch[DG_FP64].waves_per_block == 4)
    launch_pw<P, P < 4 ? 4 : 2>(args, fused, s);
  else
    launch_pw<P, 2>(args, fused, s);
  DG_HIP(hipGetLastError());
  return DG_OK;
}

}  // namespace

dg_status launch_rhs_euler_fp64(const Mesh& m, double gamma, const double* q, double* rhs, const double* res_in,
                                double* res, double* q_out, double a, double b, double dt, bool fused, hipStream_t s) {
  RhsArgs A;
  A.q = q;
  A.rhs = rhs;
  A.res_in = res_in;
  A.res = res;
  A.qout = q_out;
  A.geo = m.d_geo;
  A.conn = m.d_conn;
  A.op = m.d_op64;
  A.fmask = m.d_fmask;
  A.nbtab = m.d_nbtab;
  A.E = m.E;
  A.Epad = m.Epad;
  A.ntiles = static_cast<int>(m.Epad / 16);
  A.dma = (reinterpret_cast<uintptr_t>(q) & 15u) == 0 && m.launch[DG_FP64].lds_stage ? 1 : 0;
  A.xcd_run = m.launch[DG_FP64].xcd_run;
  A.gamma = gamma;
  A.a = a;
  A.b = b;
  A.dt = dt;
  A.flags = device_flags();
  switch (m.p) {
    case 1: return launch_p<1>(m, A, fused, s);
    case 2: return launch_p<2>(m, A, fused, s);
    case 3: return launch_p<3>(m, A, fused, s);
    case 4: return launch_p<4>(m, A, fused, s);
    default: return fail(DG_ERR_ARG, "rhs: unsupported order");
  }
}

}  // namespace dg
