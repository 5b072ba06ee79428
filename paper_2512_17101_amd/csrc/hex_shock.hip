// Shock capturing on the tensor-product hexahedra: the modal smoothness
// indicator with the per-element artificial viscosity and its BR1 viscous
// flux, and the positivity-preserving limiter.
//
//  hex_av_flux_kernel   per element: rho's orthonormal tensor Legendre
//                       coefficients (three 1-D passes with the inverse
//                       modal Vandermonde), s = log10(top-mode energy /
//                       energy), eps = c_eps h / p max(|u| + c) ramp(s); then
//                       per field and direction the lifted gradient
//                       sigma_d = (2/h_d)(D_d q + sum_side l_side n_d (q+ - q-)/2)
//                       and G_d = eps sigma_d, stored [d][f][E][Np].
//  hex_limit_kernel     per element, in place: density then pressure
//                       positivity by scaling towards the cell average
//                       (Zhang & Shu), with delta; elements that need no
//                       limiting are not written.
// The element reductions (energies, wave speed, averages, minima) run in a
// fixed order (the indicator's at p >= 3 as eight strided partial sums and
// their sum), so results do not depend on the launch.
#include <cmath>

#include "hex.hpp"

namespace dg {
namespace {

template <int P>
struct ShCfg {
  static constexpr int N1 = P + 1;
  static constexpr int NP = N1 * N1 * N1;
  static constexpr int NFP = N1 * N1;
  static constexpr int EPB = 256 / NP;
  static constexpr int NT = EPB * NP;
  static constexpr int NS = EPB * 6 * NFP;
  static constexpr int KF = (NS + 255) / 256;
};

struct ShArgs {
  const double* __restrict__ q;
  double* __restrict__ qio;       // limiter: state in place
  double* __restrict__ G;         // [3][5][E][Np]
  double* __restrict__ s_out;     // [E] indicator (may be null)
  double* __restrict__ eps_out;   // [E] viscosity (may be null)
  const double* __restrict__ ih;  // [nx | ny | nz] 2 / h
  const double* __restrict__ op;  // [D1 | lift]
  const double* __restrict__ sh;  // [Vinv (N1 x N1) | w1 (N1)]
  int nx, ny, nz, E;
  double gamma, s0, kappa, c_eps, delta;
  unsigned* flags;
};

template <int N1>
__device__ inline int nidx(int a, int b, int c) { return a + N1 * (b + N1 * c); }

template <int P>
__global__ __launch_bounds__(256) __attribute__((amdgpu_waves_per_eu(P == 1 || P == 3 ? 3 : 4))) void hex_av_flux_kernel(
    ShArgs A) {
  using C = ShCfg<P>;
  constexpr int N1 = C::N1, NP = C::NP, NFP = C::NFP, EPB = C::EPB;
  constexpr int RW = NP >= 64 ? 8 : 1;  // partial sums per element in the reductions
  static_assert(EPB * RW <= 256, "reduction threads");
  __shared__ double s_q[EPB][5][NP];
  __shared__ double s_J[EPB][6][5][NFP];
  __shared__ double s_t[2][EPB * NP];  // modal passes
  __shared__ double s_r[3][EPB * NP];  // per-node energies and wave speeds
  __shared__ double s_p[3][EPB * RW];  // their partial sums
  __shared__ double s_eps[EPB];
  const int tid = threadIdx.x;
  const int E = A.E;
  const int e0 = blockIdx.x * EPB;
  const int el = tid / NP, i = tid - (tid / NP) * NP;
  const bool own = tid < C::NT;
  const int elc = own ? el : 0, ic = own ? i : 0;
  const int e = e0 + elc < E ? e0 + elc : E - 1;
  const bool valid = own && e0 + el < E;
  const int idx = e * NP + ic;
  const size_t Es = static_cast<size_t>(E) * NP;

  // (1) the indicator and the viscosity need only the element's own nodes.
  // At p <= 2 (8 or 27 nodes, 32 or 9 elements per block) most blocks on a
  // shock front hold a viscous element, and the neighbour traces are
  // requested here already, so that their latency overlaps the indicator;
  // at p >= 3 they are gathered only by blocks that need them.
  constexpr bool kPrefetch = P <= 2;
  double qv[5];
#pragma unroll
  for (int f = 0; f < 5; ++f) qv[f] = A.q[f * Es + idx];
  double qp[C::KF][5];
  int nbi[C::KF], ownn[C::KF];
#pragma unroll
  for (int u = 0; u < C::KF; ++u) {
    const int s = tid + 256 * u < C::NS ? tid + 256 * u : C::NS - 1;
    const int fl = s / (6 * NFP), rem = s - fl * (6 * NFP);
    const int face = rem / NFP, m = rem - face * NFP;
    const int d = face >> 1, side = face & 1;
    const int ef = e0 + fl < E ? e0 + fl : E - 1;
    const int fx = ef % A.nx, fxy = ef / A.nx, fy = fxy % A.ny, fz = fxy / A.ny;
    const int cd = d == 0 ? fx : d == 1 ? fy : fz;
    const int nd = d == 0 ? A.nx : d == 1 ? A.ny : A.nz;
    const int stride = d == 0 ? 1 : d == 1 ? A.nx : A.nx * A.ny;
    const int en = side ? (cd == nd - 1 ? ef - (nd - 1) * stride : ef + stride)
                        : (cd == 0 ? ef + (nd - 1) * stride : ef - stride);
    const int uu = m % N1, vv = m / N1;
    const int fo = side ? P : 0, fn = side ? 0 : P;
    ownn[u] = d == 0 ? nidx<N1>(fo, uu, vv) : d == 1 ? nidx<N1>(uu, fo, vv) : nidx<N1>(uu, vv, fo);
    nbi[u] = en * NP + (d == 0 ? nidx<N1>(fn, uu, vv) : d == 1 ? nidx<N1>(uu, fn, vv) : nidx<N1>(uu, vv, fn));
    if constexpr (kPrefetch) {
#pragma unroll
      for (int f = 0; f < 5; ++f) qp[u][f] = A.q[f * Es + nbi[u]];
    }
  }
  const int cx = e % A.nx, cxy = e / A.nx;
  const double ihx = A.ih[cx], ihy = A.ih[A.nx + cxy % A.ny], ihz = A.ih[A.nx + A.ny + cxy / A.ny];
  if (own) {
#pragma unroll
    for (int f = 0; f < 5; ++f) s_q[el][f][i] = qv[f];
  }
  __syncthreads();

  // modal coefficients of rho, three passes (a, b, c)
  const int a = ic % N1, bb = (ic / N1) % N1, c = ic / (N1 * N1);
  const double* Vi = A.sh;
  const int base = elc * NP;
  {
    double t = 0.0;
#pragma unroll
    for (int m = 0; m < N1; ++m) t = fma(Vi[a * N1 + m], s_q[elc][0][nidx<N1>(m, bb, c)], t);
    if (own) s_t[0][tid] = t;
  }
  __syncthreads();
  {
    double t = 0.0;
#pragma unroll
    for (int m = 0; m < N1; ++m) t = fma(Vi[bb * N1 + m], s_t[0][base + nidx<N1>(a, m, c)], t);
    if (own) s_t[1][tid] = t;
  }
  __syncthreads();
  {
    double t = 0.0;
#pragma unroll
    for (int m = 0; m < N1; ++m) t = fma(Vi[c * N1 + m], s_t[1][base + nidx<N1>(a, bb, m)], t);
    const bool top = a == P || bb == P || c == P;
    const double ir = 1.0 / qv[0];
    const double u = qv[1] * ir, v = qv[2] * ir, w = qv[3] * ir;
    const double pr = (A.gamma - 1.0) * (qv[4] - 0.5 * (qv[1] * u + qv[2] * v + qv[3] * w));
    if (own) {
      s_r[0][tid] = t * t;
      s_r[1][tid] = top ? t * t : 0.0;
      s_r[2][tid] = sqrt(u * u + v * v + w * w) + sqrt(A.gamma * pr * ir);
    }
  }
  __syncthreads();
  // energies and the largest wave speed per element, in a fixed order:
  // RW strided partial sums (RW = 1 below 64 nodes), then their sum
  if (tid < EPB * RW) {
    const int re = tid / RW, rk = tid - re * RW;
    double num = 0.0, den = 0.0, lam = 0.0;
    for (int k = rk; k < NP; k += RW) {
      den += s_r[0][re * NP + k];
      num += s_r[1][re * NP + k];
      lam = fmax(lam, s_r[2][re * NP + k]);
    }
    s_p[0][tid] = den;
    s_p[1][tid] = num;
    s_p[2][tid] = lam;
  }
  __syncthreads();
  if (tid < EPB) {
    double num = 0.0, den = 0.0, lam = 0.0;
#pragma unroll
    for (int k = 0; k < RW; ++k) {
      den += s_p[0][tid * RW + k];
      num += s_p[1][tid * RW + k];
      lam = fmax(lam, s_p[2][tid * RW + k]);
    }
    const int ee = e0 + tid < E ? e0 + tid : E - 1;
    const int ex = ee % A.nx, exy = ee / A.nx;
    const double h = fmin(fmin(2.0 / A.ih[ex], 2.0 / A.ih[A.nx + exy % A.ny]), 2.0 / A.ih[A.nx + A.ny + exy / A.ny]);
    const double sv = num > 0.0 ? log10(num / den) : -INFINITY;
    double ramp;
    if (sv < A.s0 - A.kappa) ramp = 0.0;
    else if (sv > A.s0 + A.kappa) ramp = 1.0;
    else ramp = 0.5 * (1.0 + sin(3.14159265358979323846 * (sv - A.s0) / (2.0 * A.kappa)));
    const double eps = A.c_eps * h / P * lam * ramp;
    s_eps[tid] = eps;
    if (e0 + tid < E) {
      if (A.s_out) A.s_out[e0 + tid] = sv;
      if (A.eps_out) A.eps_out[e0 + tid] = eps;
    }
  }
  __syncthreads();

  // (2) lifted gradients and the viscous flux, per field, only in blocks
  // with a viscous element: an inviscid element (eps = 0, most of them) has
  // G = 0, which is neither formed nor stored (the right-hand side reads G
  // only where eps > 0), so most blocks end here without gathering any
  // neighbour trace
  bool any = false;
#pragma unroll
  for (int k = 0; k < EPB; ++k) any |= s_eps[k] > 0.0;
  if (!any) return;
  const double epsv = s_eps[elc];
  // central jumps n_d (q+ - q-) / 2 of the block's face slots
  if constexpr (!kPrefetch) {
#pragma unroll
    for (int u = 0; u < C::KF; ++u)
#pragma unroll
      for (int f = 0; f < 5; ++f) qp[u][f] = A.q[f * Es + nbi[u]];
  }
#pragma unroll
  for (int u = 0; u < C::KF; ++u) {
    const int s = tid + 256 * u;
    if (s < C::NS) {
      const int fl = s / (6 * NFP), rem = s - fl * (6 * NFP);
      const int face = rem / NFP, m = rem - face * NFP;
      const double hn = (face & 1) ? 0.5 : -0.5;
#pragma unroll
      for (int f = 0; f < 5; ++f) s_J[fl][face][f][m] = hn * (qp[u][f] - s_q[fl][f][ownn[u]]);
    }
  }
  __syncthreads();
  const double* D1 = A.op;
  const double* lift = A.op + N1 * N1;
#pragma unroll 1
  for (int f = 0; f < 5; ++f) {
    double gx = 0.0, gy = 0.0, gz = 0.0;
#pragma unroll
    for (int m = 0; m < N1; ++m) {
      gx = fma(D1[a * N1 + m], s_q[elc][f][nidx<N1>(m, bb, c)], gx);
      gy = fma(D1[bb * N1 + m], s_q[elc][f][nidx<N1>(a, m, c)], gy);
      gz = fma(D1[c * N1 + m], s_q[elc][f][nidx<N1>(a, bb, m)], gz);
    }
    gx += lift[a * 2] * s_J[elc][0][f][bb + N1 * c] + lift[a * 2 + 1] * s_J[elc][1][f][bb + N1 * c];
    gy += lift[bb * 2] * s_J[elc][2][f][a + N1 * c] + lift[bb * 2 + 1] * s_J[elc][3][f][a + N1 * c];
    gz += lift[c * 2] * s_J[elc][4][f][a + N1 * bb] + lift[c * 2 + 1] * s_J[elc][5][f][a + N1 * bb];
    if (valid && epsv > 0.0) {
      A.G[(0 * 5 + f) * Es + idx] = epsv * (ihx * gx);
      A.G[(1 * 5 + f) * Es + idx] = epsv * (ihy * gy);
      A.G[(2 * 5 + f) * Es + idx] = epsv * (ihz * gz);
    }
  }
}

template <int P>
__global__ __launch_bounds__(256) void hex_limit_kernel(ShArgs A) {
  using C = ShCfg<P>;
  constexpr int N1 = C::N1, NP = C::NP, EPB = C::EPB;
  __shared__ double s_q[EPB][5][NP];
  __shared__ double s_w[EPB][NP];     // per-node work values for the reductions
  __shared__ double s_bar[EPB][6];    // averages (5) and the pressure of the average
  __shared__ double s_th[EPB][2];     // theta1, theta2
  const int tid = threadIdx.x;
  const int E = A.E;
  const int e0 = blockIdx.x * EPB;
  const int el = tid / NP, i = tid - (tid / NP) * NP;
  const bool own = tid < C::NT;
  const int elc = own ? el : 0, ic = own ? i : 0;
  const int e = e0 + elc < E ? e0 + elc : E - 1;
  const bool valid = own && e0 + el < E;
  const int idx = e * NP + ic;
  const size_t Es = static_cast<size_t>(E) * NP;
  const double g1 = A.gamma - 1.0;
  const double* w1 = A.sh + N1 * N1;
  __shared__ int s_any;
  double qv[5];
#pragma unroll
  for (int f = 0; f < 5; ++f) qv[f] = A.qio[f * Es + idx];
  if (tid == 0) s_any = 0;
  __syncthreads();
  {
    // only a block with an inadmissible node does anything more (an element
    // whose nodes are all admissible is left as it is in any case)
    const double p0 = g1 * (qv[4] - 0.5 * (qv[1] * qv[1] + qv[2] * qv[2] + qv[3] * qv[3]) / qv[0]);
    if (valid && !(qv[0] >= A.delta && p0 >= A.delta)) s_any = 1;
  }
  __syncthreads();
  if (!s_any) return;
  if (own) {
#pragma unroll
    for (int f = 0; f < 5; ++f) s_q[el][f][i] = qv[f];
  }
  __syncthreads();
  // averages with the weights int l_i (thread f of each element sums field
  // f; thread 5 the minimum density)
  if (tid < EPB * 6) {
    const int ee = tid / 6, f = tid - ee * 6;
    if (f < 5) {
      double sw = 0.0, sq = 0.0;
      for (int k = 0; k < NP; ++k) {
        const double w = w1[k % N1] * w1[(k / N1) % N1] * w1[k / (N1 * N1)];
        sw += w;
        sq += w * s_q[ee][f][k];
      }
      s_bar[ee][f] = sq / sw;
    } else {
      double mn = s_q[ee][0][0];
      for (int k = 1; k < NP; ++k) mn = fmin(mn, s_q[ee][0][k]);
      s_w[ee][0] = mn;  // read back below before s_w is reused
    }
  }
  __syncthreads();
  if (tid < EPB) {
    const double* qb = s_bar[tid];
    const double pb = g1 * (qb[4] - 0.5 * (qb[1] * qb[1] + qb[2] * qb[2] + qb[3] * qb[3]) / qb[0]);
    s_bar[tid][5] = pb;
    const double rmin = s_w[tid][0];
    const bool adm = qb[0] > A.delta && pb > A.delta;
    // theta1 < 1: the density step applies; -1: the element is left as it is
    s_th[tid][0] = !adm ? -1.0 : rmin < A.delta ? (qb[0] - A.delta) / (qb[0] - rmin) : 1.0;
  }
  __syncthreads();
  // density step, then each node's limit for the pressure step (2 = none)
  const double* qb = s_bar[elc];
  const double th1 = s_th[elc][0];
  double q1[5];
#pragma unroll
  for (int f = 0; f < 5; ++f) q1[f] = th1 >= 0.0 && th1 < 1.0 ? qb[f] + th1 * (qv[f] - qb[f]) : qv[f];
  const double pn = g1 * (q1[4] - 0.5 * (q1[1] * q1[1] + q1[2] * q1[2] + q1[3] * q1[3]) / q1[0]);
  if (own) s_w[el][i] = pn < A.delta ? (qb[5] - A.delta) / (qb[5] - pn) : 2.0;
  __syncthreads();
  if (tid < EPB) {
    double th = 2.0;
    for (int k = 0; k < NP; ++k) th = fmin(th, s_w[tid][k]);
    s_th[tid][1] = th;
  }
  __syncthreads();
  const double th2 = s_th[elc][1];
  if (valid && th1 >= 0.0 && (th1 < 1.0 || th2 < 2.0)) {
#pragma unroll
    for (int f = 0; f < 5; ++f) A.qio[f * Es + idx] = th2 < 2.0 ? qb[f] + th2 * (q1[f] - qb[f]) : q1[f];
  }
}

// p = 1 on the boxes of TX x TY x TZ cells of the p = 1 right-hand side: a
// cell's 8 nodes are 8 consecutive lanes (node i = a + 2 b + 4 c), so the
// three modal passes, the cell's reductions and the line derivatives take the
// other node of a line from lane i ^ 1, i ^ 2 or i ^ 4 instead of LDS (the
// reductions as a butterfly over the cell's lanes: every lane gets the same
// bits); each face node's central jump 1/2 (q_R - q_L), the same for both
// sides, is formed once, in-tile sides from the tile's LDS copy.
template <int TX, int TY, int TZ>
__global__ __launch_bounds__(256) __attribute__((amdgpu_waves_per_eu(4))) void hex_av_flux_tile_kernel(ShArgs A) {
  constexpr int P = 1;
  using C = HexTileCfg<P, TX, TY, TZ>;
  constexpr int NP = C::NP, NFP = C::NFP, NC = C::NC;
  static_assert(C::NT == 256, "one thread per node, every thread");
  __shared__ double s_q[NC][5][NP];
  __shared__ double s_J[NC][6][5][NFP];
  const int tid = threadIdx.x;
  const int nx = A.nx, ny = A.ny, nz = A.nz;
  const int ntx = (nx + TX - 1) / TX, nty = (ny + TY - 1) / TY;
  const int X0 = (blockIdx.x % ntx) * TX, Y0 = ((blockIdx.x / ntx) % nty) * TY, Z0 = (blockIdx.x / (ntx * nty)) * TZ;
  const size_t Es = static_cast<size_t>(A.E) * NP;
  const int cl = tid / NP, ic = tid - cl * NP;
  const int lx = cl % TX, ly = (cl / TX) % TY, lz = cl / (TX * TY);
  const bool valid = X0 + lx < nx && Y0 + ly < ny && Z0 + lz < nz;
  const int gx = valid ? X0 + lx : 0, gy = valid ? Y0 + ly : 0, gz = valid ? Z0 + lz : 0;
  const int e = gx + nx * (gy + ny * gz);
  const int idx = e * NP + ic;

  // own node, and the out-of-tile sides of this thread's face nodes
  double qv[5];
#pragma unroll
  for (int f = 0; f < 5; ++f) qv[f] = A.q[f * Es + idx];
  int fdir[C::KF], fm[C::KF], fcell[C::KF][2], fnn[C::KF][2];
  bool fin[C::KF][2], fuse[C::KF];
  double gq[C::KF][2][5];
#pragma unroll
  for (int u = 0; u < C::KF; ++u) {
    const int s = tid + 256 * u < C::NS ? tid + 256 * u : C::NS - 1;
    const TileFaceNode fn = tile_face_node<P, TX, TY, TZ>(s, s == tid + 256 * u, X0, Y0, Z0, nx, ny, nz);
    fdir[u] = fn.d;
    fm[u] = fn.m;
#pragma unroll
    for (int side = 0; side < 2; ++side) {
      fin[u][side] = fn.in[side];
      fcell[u][side] = fn.cell[side];
      fnn[u][side] = fn.gi[side] - fn.ge[side] * NP;
#pragma unroll
      for (int f = 0; f < 5; ++f) gq[u][side][f] = fn.in[side] ? 0.0 : A.q[f * Es + fn.gi[side]];
    }
    fuse[u] = fn.in[0] || fn.in[1];
  }
#pragma unroll
  for (int f = 0; f < 5; ++f) s_q[cl][f][ic] = qv[f];

  // rho's modal coefficients: the inverse modal Vandermonde along a, b, c
  const int a = ic & 1, bb = (ic >> 1) & 1, c = ic >> 2;
  const double* Vi = A.sh;
  const double va0 = a ? Vi[2] : Vi[0], va1 = a ? Vi[3] : Vi[1];
  const double vb0 = bb ? Vi[2] : Vi[0], vb1 = bb ? Vi[3] : Vi[1];
  const double vc0 = c ? Vi[2] : Vi[0], vc1 = c ? Vi[3] : Vi[1];
  double t = qv[0];
  {
    const double o = __shfl_xor(t, 1, 64);
    t = fma(va1, a ? t : o, fma(va0, a ? o : t, 0.0));
  }
  {
    const double o = __shfl_xor(t, 2, 64);
    t = fma(vb1, bb ? t : o, fma(vb0, bb ? o : t, 0.0));
  }
  {
    const double o = __shfl_xor(t, 4, 64);
    t = fma(vc1, c ? t : o, fma(vc0, c ? o : t, 0.0));
  }
  const bool top = a == P || bb == P || c == P;
  const double ir = 1.0 / qv[0];
  const double u = qv[1] * ir, v = qv[2] * ir, w = qv[3] * ir;
  const double pr = (A.gamma - 1.0) * (qv[4] - 0.5 * (qv[1] * u + qv[2] * v + qv[3] * w));
  double den = t * t, num = top ? t * t : 0.0;
  double lam = sqrt(u * u + v * v + w * w) + sqrt(A.gamma * pr * ir);
#pragma unroll
  for (int k = 1; k < NP; k <<= 1) {
    den += __shfl_xor(den, k, 64);
    num += __shfl_xor(num, k, 64);
    lam = fmax(lam, __shfl_xor(lam, k, 64));
  }
  const double h = fmin(fmin(2.0 / A.ih[gx], 2.0 / A.ih[nx + gy]), 2.0 / A.ih[nx + ny + gz]);
  const double sv = num > 0.0 ? log10(num / den) : -INFINITY;
  double ramp;
  if (sv < A.s0 - A.kappa) ramp = 0.0;
  else if (sv > A.s0 + A.kappa) ramp = 1.0;
  else ramp = 0.5 * (1.0 + sin(3.14159265358979323846 * (sv - A.s0) / (2.0 * A.kappa)));
  const double eps = A.c_eps * h / P * lam * ramp;
  if (valid && ic == 0) {
    if (A.s_out) A.s_out[e] = sv;
    if (A.eps_out) A.eps_out[e] = eps;
  }

  // lifted gradients and the viscous flux only in tiles holding a viscous
  // element (the block barrier also completes the LDS copy of the state)
  if (!__syncthreads_or(valid && eps > 0.0)) return;
#pragma unroll
  for (int u = 0; u < C::KF; ++u) {
    if (!fuse[u]) continue;
    const int d = fdir[u], m = fm[u];
#pragma unroll
    for (int f = 0; f < 5; ++f) {
      const double qL = fin[u][0] ? s_q[fcell[u][0]][f][fnn[u][0]] : gq[u][0][f];
      const double qR = fin[u][1] ? s_q[fcell[u][1]][f][fnn[u][1]] : gq[u][1][f];
      const double j = 0.5 * (qR - qL);  // n_d (q+ - q-) / 2 on both sides
      if (fin[u][0]) s_J[fcell[u][0]][2 * d + 1][f][m] = j;
      if (fin[u][1]) s_J[fcell[u][1]][2 * d][f][m] = j;
    }
  }
  __syncthreads();
  if (!(valid && eps > 0.0)) return;
  const double* D1 = A.op;
  const double* lift = A.op + 4;
  const double da0 = a ? D1[2] : D1[0], da1 = a ? D1[3] : D1[1];
  const double db0 = bb ? D1[2] : D1[0], db1 = bb ? D1[3] : D1[1];
  const double dc0 = c ? D1[2] : D1[0], dc1 = c ? D1[3] : D1[1];
  const double la0 = a ? lift[2] : lift[0], la1 = a ? lift[3] : lift[1];
  const double lb0 = bb ? lift[2] : lift[0], lb1 = bb ? lift[3] : lift[1];
  const double lc0 = c ? lift[2] : lift[0], lc1 = c ? lift[3] : lift[1];
  const double ihx = A.ih[gx], ihy = A.ih[nx + gy], ihz = A.ih[nx + ny + gz];
#pragma unroll
  for (int f = 0; f < 5; ++f) {
    const double qf = qv[f];
    const double px = __shfl_xor(qf, 1, 64), py = __shfl_xor(qf, 2, 64), pz = __shfl_xor(qf, 4, 64);
    double gxv = fma(da1, a ? qf : px, fma(da0, a ? px : qf, 0.0));
    double gyv = fma(db1, bb ? qf : py, fma(db0, bb ? py : qf, 0.0));
    double gzv = fma(dc1, c ? qf : pz, fma(dc0, c ? pz : qf, 0.0));
    gxv += la0 * s_J[cl][0][f][bb + 2 * c] + la1 * s_J[cl][1][f][bb + 2 * c];
    gyv += lb0 * s_J[cl][2][f][a + 2 * c] + lb1 * s_J[cl][3][f][a + 2 * c];
    gzv += lc0 * s_J[cl][4][f][a + 2 * bb] + lc1 * s_J[cl][5][f][a + 2 * bb];
    A.G[(0 * 5 + f) * Es + idx] = eps * (ihx * gxv);
    A.G[(1 * 5 + f) * Es + idx] = eps * (ihy * gyv);
    A.G[(2 * 5 + f) * Es + idx] = eps * (ihz * gzv);
  }
}

template <int P>
dg_status launch_av_p(const HexMesh& m, const ShArgs& A, hipStream_t s) {
  using C = ShCfg<P>;
  const int64_t blocks = (m.E + C::EPB - 1) / C::EPB;
  if (P == 1) {
    const int64_t tiles = static_cast<int64_t>((m.nx + kTileX1 - 1) / kTileX1) * ((m.ny + kTileY1 - 1) / kTileY1) *
                          ((m.nz + kTileZ1 - 1) / kTileZ1);
    hipLaunchKernelGGL((hex_av_flux_tile_kernel<kTileX1, kTileY1, kTileZ1>), dim3(static_cast<unsigned>(tiles)),
                       dim3(256), 0, s, A);
  } else {
    hipLaunchKernelGGL((hex_av_flux_kernel<P>), dim3(static_cast<unsigned>(blocks)), dim3(256), 0, s, A);
  }
  const hipError_t e = hipGetLastError();
  return e == hipSuccess ? DG_OK : hip_fail(e, "hex viscosity launch");
}

template <int P>
dg_status launch_limit_p(const HexMesh& m, const ShArgs& A, hipStream_t s) {
  using C = ShCfg<P>;
  const int64_t blocks = (m.E + C::EPB - 1) / C::EPB;
  hipLaunchKernelGGL((hex_limit_kernel<P>), dim3(static_cast<unsigned>(blocks)), dim3(256), 0, s, A);
  const hipError_t e = hipGetLastError();
  return e == hipSuccess ? DG_OK : hip_fail(e, "hex limiter launch");
}

ShArgs args_of(const HexMesh& m, const dg_av_params& av, double gamma) {
  ShArgs A{};
  A.ih = m.d_ih;
  A.op = m.d_op;
  A.sh = m.d_sh;
  A.nx = m.nx;
  A.ny = m.ny;
  A.nz = m.nz;
  A.E = static_cast<int>(m.E);
  A.gamma = gamma;
  A.s0 = av.s0;
  A.kappa = av.kappa;
  A.c_eps = av.c_eps;
  A.delta = av.delta;
  A.flags = device_flags();
  return A;
}

}  // namespace

dg_status launch_hex_av_flux(const HexMesh& m, const dg_av_params& av, double gamma, const double* q, double* G,
                             double* s_out, double* eps_out, hipStream_t s) {
  ShArgs A = args_of(m, av, gamma);
  A.q = q;
  A.G = G;
  A.s_out = s_out;
  A.eps_out = eps_out;
  switch (m.p) {
    case 1: return launch_av_p<1>(m, A, s);
    case 2: return launch_av_p<2>(m, A, s);
    case 3: return launch_av_p<3>(m, A, s);
    case 4: return launch_av_p<4>(m, A, s);
    default: return fail(DG_ERR_ARG, "hex viscosity: unsupported order");
  }
}

dg_status launch_hex_limit(const HexMesh& m, const dg_av_params& av, double gamma, double* q, hipStream_t s) {
  ShArgs A = args_of(m, av, gamma);
  A.qio = q;
  switch (m.p) {
    case 1: return launch_limit_p<1>(m, A, s);
    case 2: return launch_limit_p<2>(m, A, s);
    case 3: return launch_limit_p<3>(m, A, s);
    case 4: return launch_limit_p<4>(m, A, s);
    default: return fail(DG_ERR_ARG, "hex limiter: unsupported order");
  }
}

}  // namespace dg
