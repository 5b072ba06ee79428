// Reacting Navier-Stokes right-hand side with BR1 viscous terms, FP64, gfx950.
//
// Two passes per evaluation, both element-local with the reference operators
// in LDS and one thread per (element, node):
//
//  gradient pass   sigma_d(v)_i = sum_a (da/dx_d) (D_a v)_i
//                                 + sum_f N_{f,d} sum_m LIFT[i, (f, m)] dv_(f,m),
//                  dv = (v+ - v-) / 2, N_f = Fscale_f n_f (from the metric);
//                  the element's primitives and face jumps are staged in LDS,
//                  the thread accumulates D_r v, D_s v, D_t v of all 11
//                  primitives (each operator entry read once for all of them).
//  right-hand side rhs_i = -sum_a sum_j D_a[i, j] G_a,j + sum_m LIFT[i, m] Delta_m
//                  + sources, G_a = total flux along grad a, Delta the face
//                  jump (Lax-Friedrichs on the inviscid flux, central on the
//                  viscous one, no penalty).  The fluxes of every volume node
//                  and the jumps of every face node of the block's elements go
//                  to LDS; the contractions of the 12 fields are then shared
//                  out over all threads.
//
// FP64 matrix cores and FP64 vector FMAs have the same peak on this chip, so
// the contractions run on the vector units; the operator entries come from LDS
// laid out so that consecutive threads (consecutive output rows) read
// consecutive words.
#include "internal.hpp"
#include "ns.hpp"
#include "ns_point.hpp"

namespace dg {
namespace {

// Copies N doubles into LDS, thread t of NT: every load is issued before
// the first write (one memory latency instead of one per loop trip).
template <int N, int NT>
__device__ inline void stage_block_array(double* dst, const double* __restrict__ src, int t) {
  constexpr int K = (N + NT - 1) / NT;
  double v[K];
#pragma unroll
  for (int k = 0; k < K; ++k) {
    const int i = t + k * NT;
    v[k] = src[i < N ? i : N - 1];
  }
#pragma unroll
  for (int k = 0; k < K; ++k) {
    const int i = t + k * NT;
    if (i < N) dst[i] = v[k];
  }
}

template <int P>
struct NsCfg {
  static constexpr int NP = (P + 1) * (P + 2) * (P + 3) / 6;
  static constexpr int NFP = (P + 1) * (P + 2) / 2;
  static constexpr int NFN = 4 * NFP;
  static constexpr int EPB = 256 / NP;      // elements per block
  static constexpr int KOP = 3 * NP + NFN;  // operator rows (D_r, D_s, D_t columns, then LIFT columns)
};

__device__ inline void load_state(const double* __restrict__ q, int64_t Es, int64_t idx, double qq[kNsFields]) {
#pragma unroll
  for (int f = 0; f < kNsFields; ++f) qq[f] = q[f * Es + idx];
}

// sigma is node-major, [E][Np][33]: the 33 gradients of one node are
// contiguous, so a face node gathering its neighbour's node touches about
// three cache lines instead of 33 (one per field array); measured 12 %
// faster for the gradient + right-hand-side passes than field-major.
__device__ inline void load_sigma(const double* __restrict__ sg, int64_t idx, double s[3 * kNsPrims]) {
#pragma unroll
  for (int f = 0; f < 3 * kNsPrims; ++f) s[f] = sg[idx * (3 * kNsPrims) + f];
}

// LDS of the gradient pass: the block's primitives [EPB][11][Np] and face
// half-jumps [EPB][11][4 Nfp]; after the contraction the same memory holds
// the block's gradients node-major, [EPB Np][33], for one coalesced copy out.
template <int P>
struct NsGradLds {
  using C = NsCfg<P>;
  static constexpr int V = C::EPB * kNsPrims * C::NP;
  static constexpr int D = C::EPB * kNsPrims * C::NFN;
  static constexpr int S = C::EPB * C::NP * 3 * kNsPrims;
  static constexpr int SIZE = V + D > S ? V + D : S;
};

template <int P>
__global__ __launch_bounds__(256) void ns_grad_kernel(NsArgs A) {
  using C = NsCfg<P>;
  using LD = NsGradLds<P>;
  __shared__ double s_op[C::KOP * C::NP];
  __shared__ double s_buf[LD::SIZE];
  auto s_v = reinterpret_cast<double (*)[kNsPrims][C::NP]>(s_buf);
  auto s_d = reinterpret_cast<double (*)[kNsPrims][C::NFN]>(s_buf + LD::V);
  const int tid = threadIdx.x;
  const int64_t e0 = static_cast<int64_t>(blockIdx.x) * C::EPB;
  const int64_t Es = A.E * C::NP;
  const int el = tid / C::NP, i = tid - el * C::NP;
  const bool vol = tid < C::EPB * C::NP;
  const int64_t e = e0 + el;
  const bool valid = vol && e < A.E;
  const int elc = vol ? el : 0, ic = vol ? i : 0;
  const int64_t ecl = e0 + elc < A.E ? e0 + elc : A.E - 1;
  // Every memory read of the first phase is requested before any is used:
  // the operator (for LDS), the metric, this thread's volume node and the
  // neighbour nodes of its face nodes (indices clamped; results of
  // out-of-range slots are discarded below).
  constexpr int NOP = C::KOP * C::NP;
  constexpr int KO = (NOP + 255) / 256;
  constexpr int NS = C::EPB * C::NFN;   // face nodes of the block
  constexpr int KF = (NS + 255) / 256;  // face nodes per thread
  double opv[KO];
#pragma unroll
  for (int k = 0; k < KO; ++k) opv[k] = A.opT[tid + 256 * k < NOP ? tid + 256 * k : NOP - 1];
  double gm[9];
#pragma unroll
  for (int k = 0; k < 9; ++k) gm[k] = A.geo[k * A.Epad + ecl];
  double qv[kNsFields], Tv;
  {
    const int64_t idx = ecl * C::NP + ic;
    load_state(A.q, Es, idx, qv);
    Tv = A.T[idx];
  }
  double qpf[KF][kNsFields], Tpf[KF];
  int ownf[KF];
#pragma unroll
  for (int u = 0; u < KF; ++u) {
    const int s = tid + 256 * u < NS ? tid + 256 * u : NS - 1;
    const int fl = s / C::NFN, fm = s - fl * C::NFN;
    const int64_t ef = e0 + fl < A.E ? e0 + fl : A.E - 1;
    const int face = fm / C::NFP, mm = fm - face * C::NFP;
    const int2 cn = A.conn[face * A.Epad + ef];
    const int jp = A.nbtab[(face * 24 + cn.y) * C::NFP + mm];
    ownf[u] = A.fmask[fm];
    const int64_t ip = static_cast<int64_t>(cn.x) * C::NP + jp;
    load_state(A.q, Es, ip, qpf[u]);
    Tpf[u] = A.T[ip];
  }
#pragma unroll
  for (int k = 0; k < KO; ++k)
    if (tid + 256 * k < NOP) s_op[tid + 256 * k] = opv[k];
  if (vol) {
    double v[kNsPrims];
    if (valid) {
      ns_primitives(qv, Tv, v);
    } else {
#pragma unroll
      for (int c = 0; c < kNsPrims; ++c) v[c] = 0.0;
    }
#pragma unroll
    for (int c = 0; c < kNsPrims; ++c) s_v[el][c][i] = v[c];
  }
  __syncthreads();
#pragma unroll
  for (int u = 0; u < KF; ++u) {
    const int s = tid + 256 * u;
    if (s >= NS) break;
    const int fl = s / C::NFN, fm = s - fl * C::NFN;
    double dv[kNsPrims];
    if (e0 + fl < A.E) {
      double vp[kNsPrims];
      ns_primitives(qpf[u], Tpf[u], vp);
#pragma unroll
      for (int c = 0; c < kNsPrims; ++c) dv[c] = 0.5 * (vp[c] - s_v[fl][c][ownf[u]]);
    } else {
#pragma unroll
      for (int c = 0; c < kNsPrims; ++c) dv[c] = 0.0;
    }
#pragma unroll
    for (int c = 0; c < kNsPrims; ++c) s_d[fl][c][fm] = dv[c];
  }
  __syncthreads();
  // sig[c][d] first holds D_a v (a = r, s, t), then the physical gradient
  // (every thread runs the arithmetic, on clamped indices, so that all reach
  // the barriers below; only valid nodes are stored)
  double sg[kNsPrims][3];
#pragma unroll
  for (int c = 0; c < kNsPrims; ++c) sg[c][0] = sg[c][1] = sg[c][2] = 0.0;
#pragma unroll 2
  for (int j = 0; j < C::NP; ++j) {
    const double dr = s_op[j * C::NP + ic];
    const double ds = s_op[(C::NP + j) * C::NP + ic];
    const double dt = s_op[(2 * C::NP + j) * C::NP + ic];
#pragma unroll
    for (int c = 0; c < kNsPrims; ++c) {
      const double vj = s_v[elc][c][j];
      sg[c][0] = fma(dr, vj, sg[c][0]);
      sg[c][1] = fma(ds, vj, sg[c][1]);
      sg[c][2] = fma(dt, vj, sg[c][2]);
    }
  }
#pragma unroll
  for (int c = 0; c < kNsPrims; ++c) {
    const double wr = sg[c][0], ws = sg[c][1], wt = sg[c][2];
#pragma unroll
    for (int d = 0; d < 3; ++d) sg[c][d] = gm[d] * wr + gm[3 + d] * ws + gm[6 + d] * wt;
  }
#pragma unroll
  for (int f = 0; f < 4; ++f) {
    double N[3];
    scaled_normal(f, gm, N[0], N[1], N[2]);
    double L[kNsPrims];
#pragma unroll
    for (int c = 0; c < kNsPrims; ++c) L[c] = 0.0;
#pragma unroll 2
    for (int m = 0; m < C::NFP; ++m) {
      const double l = s_op[(3 * C::NP + f * C::NFP + m) * C::NP + ic];
#pragma unroll
      for (int c = 0; c < kNsPrims; ++c) L[c] = fma(l, s_d[elc][c][f * C::NFP + m], L[c]);
    }
#pragma unroll
    for (int c = 0; c < kNsPrims; ++c)
#pragma unroll
      for (int d = 0; d < 3; ++d) sg[c][d] = fma(N[d], L[c], sg[c][d]);
  }
  __syncthreads();  // the primitives and jumps are no longer needed
  if (vol) {
#pragma unroll
    for (int c = 0; c < kNsPrims; ++c)
#pragma unroll
      for (int d = 0; d < 3; ++d) s_buf[(el * C::NP + i) * (3 * kNsPrims) + 3 * c + d] = sg[c][d];
  }
  __syncthreads();
  // the block's valid elements are contiguous in sigma: one coalesced copy
  const int64_t ne = A.E - e0 < C::EPB ? A.E - e0 : C::EPB;
  const int nval = static_cast<int>(ne) * C::NP * 3 * kNsPrims;
  double* dst = A.sigma + e0 * C::NP * (3 * kNsPrims);
  for (int k = tid; k < nval; k += blockDim.x) dst[k] = s_buf[k];
}

// Right-hand side: block of EPB = 256 / (4 Nfp) elements.
//  1. Thread t < EPB Np evaluates volume node t once: the contravariant total
//     fluxes G_a (a = r, s, t) of the 12 fields go to LDS, and so does its
//     sound speed.  Thread s < EPB 4 Nfp evaluates the neighbour node of face
//     node s: its total flux along the face's scaled normal N, its normal
//     velocity and sound speed, kept in registers with its state.
//  2. After the block barrier, face node s forms its own side from LDS: with
//     N = sum_a c_a grad a (c_a in {0, +-1}), N . F(-) = sum_a c_a G_a of the
//     own volume node, which is not evaluated again.  Then the jump
//       Delta = 1/2 (N.F(-) - N.F(+)) - 1/2 max(|U_N-| + c- |N|, |U_N+| + c+ |N|) (q- - q+)
//     goes to LDS.
//  3. The contractions of the 12 fields are split over H = 256 / (EPB Np)
//     thread sets of EPB Np threads.
template <int P>
struct NsRhsCfg {
  using C = NsCfg<P>;
  static constexpr int EPB = 256 / C::NFN;
  static constexpr int NV = EPB * C::NP;  // volume threads
  static constexpr int H = 256 / NV;      // field sets (1, 2 or 3: divides 12)
  static constexpr int FH = kNsFields / H;
};

template <int P, bool FUSED>
__global__ __launch_bounds__(256) __attribute__((amdgpu_waves_per_eu(2))) void ns_rhs_kernel(NsArgs A) {
  using C = NsCfg<P>;
  using R = NsRhsCfg<P>;
  static_assert(kNsFields % R::H == 0, "field sets must divide the fields");
  __shared__ double s_op[C::KOP * C::NP];
  __shared__ double s_G[R::EPB][kNsFields][3][C::NP];
  __shared__ double s_D[R::EPB][kNsFields][C::NFN];
  __shared__ double s_c[R::EPB][C::NP];
  const int tid = threadIdx.x;
  const int64_t e0 = static_cast<int64_t>(blockIdx.x) * R::EPB;
  const int64_t Es = A.E * C::NP;
  const Transport tr{A.mu, A.Pr, A.Sc};

  // face node of this thread (clamped indices; results of threads without
  // one, or of elements past the mesh, are discarded)
  const bool fnode = tid < R::EPB * C::NFN;
  const int fs = fnode ? tid : 0;
  const int fl = fs / C::NFN, fm = fs - fl * C::NFN;
  const int face = fm / C::NFP, mm = fm - face * C::NFP;
  const int64_t ef = e0 + fl < A.E ? e0 + fl : A.E - 1;
  const int2 fcn = A.conn[face * A.Epad + ef];
  const int fown = A.fmask[fm];
  const int jp = A.nbtab[(face * 24 + fcn.y) * C::NFP + mm];
  double fgm[9];
#pragma unroll
  for (int k = 0; k < 9; ++k) fgm[k] = A.geo[k * A.Epad + ef];
  stage_block_array<C::KOP * C::NP, 256>(s_op, A.opT, tid);

  if (tid < R::NV) {  // one volume node
    const int el = tid / C::NP, i = tid - el * C::NP;
    const int64_t e = e0 + el;
    double G[kNsFields];
    if (e < A.E) {
      const int64_t idx = e * C::NP + i;
      double qq[kNsFields], sg[3 * kNsPrims], gm[9];
      load_state(A.q, Es, idx, qq);
      load_sigma(A.sigma, idx, sg);
#pragma unroll
      for (int k = 0; k < 9; ++k) gm[k] = A.geo[k * A.Epad + e];
      NsNode nd;
      ns_node(A.th, qq, A.T[idx], sg, nd);
#pragma unroll
      for (int a = 0; a < 3; ++a) {
        ns_flux_along(tr, nd, qq, sg, &gm[3 * a], G);
#pragma unroll
        for (int f = 0; f < kNsFields; ++f) s_G[el][f][a][i] = G[f];
      }
      s_c[el][i] = nd.c;
    } else {
#pragma unroll
      for (int a = 0; a < 3; ++a)
#pragma unroll
        for (int f = 0; f < kNsFields; ++f) s_G[el][f][a][i] = 0.0;
      s_c[el][i] = 0.0;
    }
  }

  // the neighbour side of this thread's face node, and its own state
  double N[3];
  scaled_normal(face, fgm, N[0], N[1], N[2]);
  double qp[kNsFields], Fp[kNsFields], qm[kNsFields];
  double Unp, cp;
  {
    const int64_t ip = static_cast<int64_t>(fcn.x) * C::NP + jp;
    double sg[3 * kNsPrims];
    load_state(A.q, Es, ip, qp);
    load_sigma(A.sigma, ip, sg);
    load_state(A.q, Es, ef * C::NP + fown, qm);
    NsNode nd;
    ns_node(A.th, qp, A.T[ip], sg, nd);
    Unp = ns_flux_along(tr, nd, qp, sg, N, Fp);
    cp = nd.c;
  }
  __syncthreads();
  if (fnode) {
    double D[kNsFields];
    if (e0 + fl < A.E) {
      // N = c_r grad r + c_s grad s + c_t grad t for this face (as scaled_normal)
      const int hi = face >> 1, lo = face & 1;
      const double cr = static_cast<double>(hi * (1 - 2 * lo));
      const double cs = static_cast<double>((lo ^ hi) * (2 * hi - 1));
      const double ct = static_cast<double>((1 - lo) * (2 * hi - 1));
      const double Fs = sqrt_pos(N[0] * N[0] + N[1] * N[1] + N[2] * N[2]);
      const double ir = recip(qm[0]);
      const double Unm = (N[0] * qm[1] + N[1] * qm[2] + N[2] * qm[3]) * ir;
      const double lamFs = fmax(fabs(Unm) + s_c[fl][fown] * Fs, fabs(Unp) + cp * Fs);
#pragma unroll
      for (int f = 0; f < kNsFields; ++f) {
        const double Fm = cr * s_G[fl][f][0][fown] + cs * s_G[fl][f][1][fown] + ct * s_G[fl][f][2][fown];
        D[f] = 0.5 * (Fm - Fp[f]) - 0.5 * lamFs * (qm[f] - qp[f]);
      }
    } else {
#pragma unroll
      for (int f = 0; f < kNsFields; ++f) D[f] = 0.0;
    }
#pragma unroll
    for (int f = 0; f < kNsFields; ++f) s_D[fl][f][fm] = D[f];
  }
  __syncthreads();
  if (tid >= R::H * R::NV) return;
  const int h = tid / R::NV, t = tid - h * R::NV;
  const int el = t / C::NP, i = t - el * C::NP;
  const int64_t e = e0 + el;
  if (e >= A.E) return;
  const int f0 = h * R::FH;
  double acc[R::FH];
#pragma unroll
  for (int k = 0; k < R::FH; ++k) acc[k] = 0.0;
  // (partial unrolling: full unrolling hoists hundreds of LDS loads and spills)
#pragma unroll 1
  for (int a = 0; a < 3; ++a)
#pragma unroll 2
    for (int j = 0; j < C::NP; ++j) {
      const double d = s_op[(a * C::NP + j) * C::NP + i];
#pragma unroll
      for (int k = 0; k < R::FH; ++k) acc[k] = fma(-d, s_G[el][f0 + k][a][j], acc[k]);
    }
#pragma unroll 2
  for (int m = 0; m < C::NFN; ++m) {
    const double l = s_op[(3 * C::NP + m) * C::NP + i];
#pragma unroll
    for (int k = 0; k < R::FH; ++k) acc[k] = fma(l, s_D[el][f0 + k][m], acc[k]);
  }
  double w[kNsSpecies];
  const int64_t idx = e * C::NP + i;
  if (A.with_sources && f0 + R::FH > 5) {
    double Cc[kMaxSpecies];
#pragma unroll
    for (int k = 0; k < kNsSpecies; ++k) Cc[k] = A.q[(5 + k) * Es + idx] * A.mk.invW[k];
    node_sources(A.mk, Cc, recip(A.T[idx]), w);
  } else {
#pragma unroll
    for (int k = 0; k < kNsSpecies; ++k) w[k] = 0.0;
  }
  if constexpr (!FUSED) {
#pragma unroll
    for (int k = 0; k < R::FH; ++k) {
      const int f = f0 + k;
      A.rhs[f * Es + idx] = f >= 5 ? acc[k] + w[f - 5] : acc[k];
    }
  } else {
    // all res and q loads before the first store, so their latencies overlap
    double rv[R::FH], qv[R::FH];
#pragma unroll
    for (int k = 0; k < R::FH; ++k) {
      const int64_t at = (f0 + k) * Es + idx;
      rv[k] = A.a != 0.0 ? A.res_in[at] : 0.0;
      qv[k] = A.q[at];
    }
#pragma unroll
    for (int k = 0; k < R::FH; ++k) {
      const int f = f0 + k;
      stage_store(f * Es + idx, f >= 5 ? acc[k] + w[f - 5] : acc[k], rv[k], qv[k], A.res, A.qout, A.a, A.b, A.dt);
    }
  }
}

template <int P>
dg_status launch_p(const NsArgs& A, bool grad, bool fused, hipStream_t s) {
  using C = NsCfg<P>;
  using R = NsRhsCfg<P>;
  const dim3 block(256);
  if (grad)
    ns_grad_kernel<P><<<dim3(static_cast<unsigned>((A.E + C::EPB - 1) / C::EPB)), block, 0, s>>>(A);
  else if (fused)
    ns_rhs_kernel<P, true><<<dim3(static_cast<unsigned>((A.E + R::EPB - 1) / R::EPB)), block, 0, s>>>(A);
  else
    ns_rhs_kernel<P, false><<<dim3(static_cast<unsigned>((A.E + R::EPB - 1) / R::EPB)), block, 0, s>>>(A);
  DG_HIP(hipGetLastError());
  return DG_OK;
}

dg_status launch(int p, const NsArgs& A, bool grad, bool fused, hipStream_t s) {
  switch (p) {
    case 1: return launch_p<1>(A, grad, fused, s);
    case 2: return launch_p<2>(A, grad, fused, s);
    case 3: return launch_p<3>(A, grad, fused, s);
    case 4: return launch_p<4>(A, grad, fused, s);
    default: return fail(DG_ERR_ARG, "ns: unsupported order");
  }
}

}  // namespace

dg_status launch_ns_gradients(int p, const NsArgs& A, hipStream_t s) { return launch(p, A, true, false, s); }
dg_status launch_ns_rhs(int p, const NsArgs& A, bool fused, hipStream_t s) { return launch(p, A, false, fused, s); }

}  // namespace dg
