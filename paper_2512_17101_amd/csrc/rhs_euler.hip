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
//   because neighbouring tiles still read q).
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
  double* __restrict__ res;
  double* __restrict__ qout;
  const double* __restrict__ geo;
  const int2* __restrict__ conn;
  const double* __restrict__ op;
  const int* __restrict__ fmask;
  const uint8_t* __restrict__ nbtab;
  int64_t E, Epad;
  int ntiles;
  double gamma, a, b, dt;
};

template <int P, bool FUSED>
__global__ __launch_bounds__(256) void rhs_euler_fp64_kernel(RhsArgs A) {
  using C = Cfg<P>;
  constexpr int NB16 = C::NB16 > 0 ? C::NB16 : 1;
  constexpr int NB4 = C::NB4 > 0 ? C::NB4 : 1;
  const int lane = threadIdx.x & 63;
  const int tile = blockIdx.x * (blockDim.x >> 6) + (threadIdx.x >> 6);
  if (tile >= A.ntiles) return;  // uniform per wave
  const int n = lane & 15, g = lane >> 4;
  const int64_t e = static_cast<int64_t>(tile) * 16 + n;
  const bool valid = e < A.E;
  const int64_t ec = valid ? e : A.E - 1;
  const int64_t Es = A.E * C::NP;
  const double* __restrict__ q = A.q;
  const double gm1 = A.gamma - 1.0;

  double gm[9];
#pragma unroll
  for (int c = 0; c < 9; ++c) gm[c] = A.geo[c * A.Epad + ec];

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
      for (int f = 0; f < 5; ++f) qq[f] = q[f * Es + ec * C::NP + j];
      const double ir = 1.0 / qq[0];
      const double u = qq[1] * ir, v = qq[2] * ir, w = qq[3] * ir;
      const double p = gm1 * (qq[4] - 0.5 * (qq[1] * u + qq[2] * v + qq[3] * w));
#pragma unroll
      for (int r = 0; r < 3; ++r) {
        const double U = gm[3 * r] * u + gm[3 * r + 1] * v + gm[3 * r + 2] * w;
        G[r][0] = qq[0] * U;
        G[r][1] = qq[1] * U + p * gm[3 * r];
        G[r][2] = qq[2] * U + p * gm[3 * r + 1];
        G[r][3] = qq[3] * U + p * gm[3 * r + 2];
        G[r][4] = (qq[4] + p) * U;
      }
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
        const double a = A.op[((r * C::KV + s) * C::NRB + rb) * 64 + lane];
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

  // ---- surface: Lax-Friedrichs jump at face node fm = 4 s + g, contracted with LIFT
#pragma unroll
  for (int s = 0; s < C::KL; ++s) {
    const int fm = 4 * s + g;
    const int face = fm / C::NFP;
    const int mm = fm - face * C::NFP;
    const int own = A.fmask[fm];
    const int2 cn = A.conn[face * A.Epad + ec];
    const int jp = A.nbtab[(face * 24 + cn.y) * C::NFP + mm];
    double qm[5], qp[5];
#pragma unroll
    for (int f = 0; f < 5; ++f) {
      qm[f] = q[f * Es + ec * C::NP + own];
      qp[f] = q[f * Es + static_cast<int64_t>(cn.x) * C::NP + jp];
    }
    double Nx, Ny, Nz;
    if (face == 0) { Nx = -gm[6]; Ny = -gm[7]; Nz = -gm[8]; }
    else if (face == 1) { Nx = -gm[3]; Ny = -gm[4]; Nz = -gm[5]; }
    else if (face == 2) { Nx = gm[0] + gm[3] + gm[6]; Ny = gm[1] + gm[4] + gm[7]; Nz = gm[2] + gm[5] + gm[8]; }
    else { Nx = -gm[0]; Ny = -gm[1]; Nz = -gm[2]; }
    const double Fs = sqrt(Nx * Nx + Ny * Ny + Nz * Nz);
    const double irm = 1.0 / qm[0], irp = 1.0 / qp[0];
    const double um = qm[1] * irm, vm = qm[2] * irm, wm = qm[3] * irm;
    const double up = qp[1] * irp, vp = qp[2] * irp, wp = qp[3] * irp;
    const double pm = gm1 * (qm[4] - 0.5 * (qm[1] * um + qm[2] * vm + qm[3] * wm));
    const double pp = gm1 * (qp[4] - 0.5 * (qp[1] * up + qp[2] * vp + qp[3] * wp));
    const double Unm = Nx * um + Ny * vm + Nz * wm;
    const double Unp = Nx * up + Ny * vp + Nz * wp;
    const double cm = sqrt(A.gamma * pm * irm), cp = sqrt(A.gamma * pp * irp);
    const double lamFs = fmax(fabs(Unm) + cm * Fs, fabs(Unp) + cp * Fs);
    double D[5];
    D[0] = 0.5 * (qm[0] * Unm - qp[0] * Unp) - 0.5 * lamFs * (qm[0] - qp[0]);
    D[1] = 0.5 * (qm[1] * Unm + pm * Nx - qp[1] * Unp - pp * Nx) - 0.5 * lamFs * (qm[1] - qp[1]);
    D[2] = 0.5 * (qm[2] * Unm + pm * Ny - qp[2] * Unp - pp * Ny) - 0.5 * lamFs * (qm[2] - qp[2]);
    D[3] = 0.5 * (qm[3] * Unm + pm * Nz - qp[3] * Unp - pp * Nz) - 0.5 * lamFs * (qm[3] - qp[3]);
    D[4] = 0.5 * ((qm[4] + pm) * Unm - (qp[4] + pp) * Unp) - 0.5 * lamFs * (qm[4] - qp[4]);
#pragma unroll
    for (int rb = 0; rb < C::NRB; ++rb) {
      const double a = A.op[((3 * C::KV + s) * C::NRB + rb) * 64 + lane];
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

  // ---- store: lane (n, g) holds rows 16 rb + 4 v + g and 16 NB16 + 4 rb4 + g
  if (!valid) return;
  auto put = [&](int f, int row, double val) {
    const int64_t idx = f * Es + e * C::NP + row;
    if (!FUSED) {
      A.rhs[idx] = val;
    } else {
      const double r = (A.a == 0.0 ? 0.0 : A.a * A.res[idx]) + A.dt * val;
      A.res[idx] = r;
      A.qout[idx] = q[idx] + A.b * r;
    }
  };
#pragma unroll
  for (int f = 0; f < 5; ++f) {
#pragma unroll
    for (int rb = 0; rb < C::NB16; ++rb)
#pragma unroll
      for (int v = 0; v < 4; ++v) put(f, 16 * rb + 4 * v + g, acc16[f][rb][v]);
#pragma unroll
    for (int rb = 0; rb < C::NB4; ++rb) {
      const int row = 16 * C::NB16 + 4 * rb + g;
      if (row < C::NP) put(f, row, acc4[f][rb]);
    }
  }
}

template <int P>
dg_status launch_p(const Mesh& m, const RhsArgs& args, bool fused, hipStream_t s) {
  const int waves = 4;
  const int blocks = (args.ntiles + waves - 1) / waves;
  if (fused)
    rhs_euler_fp64_kernel<P, true><<<blocks, 64 * waves, 0, s>>>(args);
  else
    rhs_euler_fp64_kernel<P, false><<<blocks, 64 * waves, 0, s>>>(args);
  DG_HIP(hipGetLastError());
  return DG_OK;
}

}  // namespace

dg_status launch_rhs_euler_fp64(const Mesh& m, double gamma, const double* q, double* rhs, double* res, double* q_out,
                                double a, double b, double dt, bool fused, hipStream_t s) {
  RhsArgs A;
  A.q = q;
  A.rhs = rhs;
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
  A.gamma = gamma;
  A.a = a;
  A.b = b;
  A.dt = dt;
  switch (m.p) {
    case 1: return launch_p<1>(m, A, fused, s);
    case 2: return launch_p<2>(m, A, fused, s);
    case 3: return launch_p<3>(m, A, fused, s);
    case 4: return launch_p<4>(m, A, fused, s);
    default: return fail(DG_ERR_ARG, "rhs: unsupported order");
  }
}

}  // namespace dg
