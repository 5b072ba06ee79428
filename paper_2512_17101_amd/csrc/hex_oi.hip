// Overintegrated Euler right-hand side on the tensor-product hexahedra:
// the weak form of the same DG method with the fluxes evaluated at
// nq = ceil(3 (p + 1) / 2) Gauss-Legendre points per direction,
//   (M rhs)_i = int_K grad l_i . F(q_h) - int_dK l_i Fhat,
//   Fhat = 1/2 n.(F(q-) + F(q+)) + 1/2 lam (q- - q+),
// which on the box elements factors into rectangular 1-D contractions:
//   q(quad) = (B x B x B) q,  B[k][j] = l_j(xi_k)                 (nq x (p+1))
//   rhs = sum_d (2 / h_d) [ (S along d, P along the others) F_d(quad)
//                           - sum_side l_side x (P x P) Fhat_face(quad) ],
//   S = M1^{-1} B'^T W,  P = M1^{-1} B^T W                         ((p+1) x nq).
// At p = 4 this is about 220 kflop per element against 10 kB of state: the
// FP64 pipe bounds it, not HBM.  Every contraction pass runs one line per
// thread: the thread loads the line's inputs from LDS into registers and
// forms all outputs of the line, the operator entries being compile-time
// indices into a uniform table (scalar loads, not LDS traffic).  A block of
// 256 threads owns max(1, 256 / nq^3) elements; the passes of a stage are
// separated by barriers.
#include "hex.hpp"

namespace dg {
namespace {

constexpr int oi_nq(int p) { return (3 * (p + 1) + 1) / 2; }
constexpr int cmax(int a, int b) { return a > b ? a : b; }

template <int P>
struct OiCfg {
  static constexpr int N1 = P + 1;
  static constexpr int NQ = oi_nq(P);
  static constexpr int NP = N1 * N1 * N1;
  static constexpr int NF2 = N1 * N1;
  static constexpr int Q3 = NQ * NQ * NQ;
  static constexpr int EPB = Q3 >= 256 ? 1 : 256 / Q3;
  // offsets of the operator table [B (NQ x N1) | S (N1 x NQ) | P (N1 x NQ) | lift (N1 x 2)]
  static constexpr int OB = 0, OS = NQ * N1, OP = 2 * NQ * N1, OL = 3 * NQ * N1;
  // LDS regions per element (doubles)
  static constexpr int R_Q = 5 * NP;                                              // nodal state
  static constexpr int R_OUT = 5 * NP;                                            // accumulated rhs
  static constexpr int R_QQ = 5 * Q3;                                             // state at the quad points
  static constexpr int R1 = cmax(cmax(5 * NF2 * NQ, 3 * NQ * NQ * N1), 10 * N1 * NQ + 5 * NQ * NQ);
  static constexpr int R2 = cmax(cmax(5 * N1 * NQ * NQ, 3 * NQ * NF2), 2 * 5 * NQ * NQ);
  static constexpr int R_F = cmax(3 * Q3, 30 * NF2 + 5 * NQ * N1);
  static constexpr int PER_EL = R_Q + R_OUT + R_QQ + R1 + R2 + R_F;
  static constexpr int KN = (EPB * 6 * 5 * NF2 + 255) / 256;  // neighbour face values per thread
  static constexpr int KR = (EPB * 5 * NP + 255) / 256;       // output entries per thread
};

struct OiArgs {
  const double* __restrict__ q;
  double* __restrict__ rhs;
  double* __restrict__ res;
  double* __restrict__ qout;
  const double* __restrict__ ih;  // [nx | ny | nz] 2 / h
  const double* __restrict__ op;  // [B | S | P | lift]
  int nx, ny, nz;
  int E;
  double gamma, a, b, dt;
  unsigned* flags;
};

// out[o * so] = sum_i A[o * NI + i] in[i * si]: one line, operator entries at
// compile-time offsets of a uniform table
template <int NO, int NI>
__device__ inline void line(const double* __restrict__ A, const double* in, int si, double* out, int so) {
  double x[NI];
#pragma unroll
  for (int i = 0; i < NI; ++i) x[i] = in[i * si];
#pragma unroll
  for (int o = 0; o < NO; ++o) {
    double s = 0.0;
#pragma unroll
    for (int i = 0; i < NI; ++i) s = fma(A[o * NI + i], x[i], s);
    out[o * so] = s;
  }
}

// primitive velocities and pressure of a conserved state
__device__ inline void prim(const double q[5], double g, double& u, double& v, double& w, double& p) {
  const double ir = 1.0 / q[0];
  u = q[1] * ir;
  v = q[2] * ir;
  w = q[3] * ir;
  p = (g - 1.0) * (q[4] - 0.5 * (q[1] * u + q[2] * v + q[3] * w));
}

template <int P, bool FUSED>
__global__ __launch_bounds__(256) void hex_oi_kernel(OiArgs A) {
  using C = OiCfg<P>;
  constexpr int N1 = C::N1, NQ = C::NQ, NP = C::NP, NF2 = C::NF2, Q3 = C::Q3, EPB = C::EPB;
  __shared__ double s_mem[EPB * C::PER_EL];
  double* sQ = s_mem;
  double* sOut = sQ + EPB * C::R_Q;
  double* sQQ = sOut + EPB * C::R_OUT;
  double* sR1 = sQQ + EPB * C::R_QQ;
  double* sR2 = sR1 + EPB * C::R1;
  double* sF = sR2 + EPB * C::R2;
  const int tid = threadIdx.x;
  const int E = A.E;
  const int e0 = blockIdx.x * EPB;
  const size_t Es = static_cast<size_t>(E) * NP;
  const double* B = A.op + C::OB;
  const double* S = A.op + C::OS;
  const double* Pm = A.op + C::OP;
  const double* lift = A.op + C::OL;

  // (0) global reads: own state into LDS; neighbour face nodes and (fused)
  // the residual into registers, written or used later
  for (int t = tid; t < EPB * 5 * NP; t += 256) {
    const int f = t / (EPB * NP), r = t - f * (EPB * NP);
    const int el = r / NP, n = r - el * NP;
    const int e = e0 + el < E ? e0 + el : E - 1;
    sQ[(el * 5 + f) * NP + n] = A.q[f * Es + static_cast<size_t>(e) * NP + n];
  }
  double nb[C::KN];
#pragma unroll
  for (int u = 0; u < C::KN; ++u) {
    const int t0 = tid + 256 * u;
    const int t = t0 < EPB * 6 * 5 * NF2 ? t0 : EPB * 6 * 5 * NF2 - 1;
    const int el = t / (6 * 5 * NF2), r = t - el * (6 * 5 * NF2);
    const int face = r / (5 * NF2), r2 = r - face * (5 * NF2);
    const int f = r2 / NF2, m = r2 - f * NF2;
    const int d = face >> 1, side = face & 1;
    const int ef = e0 + el < E ? e0 + el : E - 1;
    const int cx = ef % A.nx, cxy = ef / A.nx, cy = cxy % A.ny, cz = cxy / A.ny;
    const int cd = d == 0 ? cx : d == 1 ? cy : cz;
    const int nd = d == 0 ? A.nx : d == 1 ? A.ny : A.nz;
    const int stride = d == 0 ? 1 : d == 1 ? A.nx : A.nx * A.ny;
    const int en = side ? (cd == nd - 1 ? ef - (nd - 1) * stride : ef + stride)
                        : (cd == 0 ? ef + (nd - 1) * stride : ef - stride);
    const int fast = m % N1, slow = m / N1, fn = side ? 0 : P;
    const int nn = d == 0 ? fn + N1 * (fast + N1 * slow) : d == 1 ? fast + N1 * (fn + N1 * slow)
                                                                   : fast + N1 * (slow + N1 * fn);
    nb[u] = A.q[f * Es + static_cast<size_t>(en) * NP + nn];
  }
  double rv[C::KR];
  if (FUSED) {
#pragma unroll
    for (int u = 0; u < C::KR; ++u) {
      const int t0 = tid + 256 * u;
      const int t = t0 < EPB * 5 * NP ? t0 : EPB * 5 * NP - 1;
      const int f = t / (EPB * NP), r = t - f * (EPB * NP);
      const int el = r / NP, n = r - el * NP;
      const int e = e0 + el < E ? e0 + el : E - 1;
      rv[u] = A.a == 0.0 ? 0.0 : A.res[f * Es + static_cast<size_t>(e) * NP + n];
    }
  }
  __syncthreads();

  // (1) interpolation to the quad points: along a, b, c
  for (int t = tid; t < EPB * 5 * NF2; t += 256)  // line (el, f, c, b)
    line<NQ, N1>(B, sQ + t * N1, 1, sR1 + t * NQ, 1);
  __syncthreads();
  for (int t = tid; t < EPB * 5 * N1 * NQ; t += 256) {  // line (el, f, c, ka)
    const int ef = t / (N1 * NQ), r = t - ef * (N1 * NQ), c = r / NQ, ka = r - c * NQ;
    line<NQ, N1>(B, sR1 + ef * (NF2 * NQ) + c * N1 * NQ + ka, NQ, sR2 + ef * (N1 * NQ * NQ) + c * NQ * NQ + ka, NQ);
  }
  __syncthreads();
  for (int t = tid; t < EPB * 5 * NQ * NQ; t += 256) {  // line (el, f, kb, ka)
    const int ef = t / (NQ * NQ), r = t - ef * (NQ * NQ);
    line<NQ, N1>(B, sR2 + ef * (N1 * NQ * NQ) + r, NQ * NQ, sQQ + ef * Q3 + r, NQ * NQ);
  }
  __syncthreads();

  // (2) per field: the three fluxes at the quad points, then the projection
  // (S along the flux's direction, P along the others), summed into sOut
#pragma unroll 1
  for (int f = 0; f < 5; ++f) {
    for (int t = tid; t < EPB * Q3; t += 256) {
      const int el = t / Q3, k = t - el * Q3;
      double qq[5];
#pragma unroll
      for (int g = 0; g < 5; ++g) qq[g] = sQQ[(el * 5 + g) * Q3 + k];
      double u, v, w, pr;
      prim(qq, A.gamma, u, v, w, pr);
      const double qe = f == 4 ? qq[4] + pr : (f == 0 ? qq[0] : f == 1 ? qq[1] : f == 2 ? qq[2] : qq[3]);
      sF[(el * 3 + 0) * Q3 + k] = qe * u + (f == 1 ? pr : 0.0);
      sF[(el * 3 + 1) * Q3 + k] = qe * v + (f == 2 ? pr : 0.0);
      sF[(el * 3 + 2) * Q3 + k] = qe * w + (f == 3 ? pr : 0.0);
    }
    __syncthreads();
    // along a: line (el, d, kc, kb), NQ -> N1
    for (int t = tid; t < EPB * NQ * NQ; t += 256) {
      const int el = t / (NQ * NQ), r = t - el * (NQ * NQ);
      line<N1, NQ>(S, sF + (el * 3 + 0) * Q3 + r * NQ, 1, sR1 + (el * 3 + 0) * (NQ * NQ * N1) + r * N1, 1);
      line<N1, NQ>(Pm, sF + (el * 3 + 1) * Q3 + r * NQ, 1, sR1 + (el * 3 + 1) * (NQ * NQ * N1) + r * N1, 1);
      line<N1, NQ>(Pm, sF + (el * 3 + 2) * Q3 + r * NQ, 1, sR1 + (el * 3 + 2) * (NQ * NQ * N1) + r * N1, 1);
    }
    __syncthreads();
    // along b: line (el, d, kc, a), NQ -> N1
    for (int t = tid; t < EPB * NQ * N1; t += 256) {
      const int el = t / (NQ * N1), r = t - el * (NQ * N1), kc = r / N1, a = r - kc * N1;
      const int ib = kc * NQ * N1 + a, ob = kc * NF2 + a;
      line<N1, NQ>(Pm, sR1 + (el * 3 + 0) * (NQ * NQ * N1) + ib, N1, sR2 + (el * 3 + 0) * (NQ * NF2) + ob, N1);
      line<N1, NQ>(S, sR1 + (el * 3 + 1) * (NQ * NQ * N1) + ib, N1, sR2 + (el * 3 + 1) * (NQ * NF2) + ob, N1);
      line<N1, NQ>(Pm, sR1 + (el * 3 + 2) * (NQ * NQ * N1) + ib, N1, sR2 + (el * 3 + 2) * (NQ * NF2) + ob, N1);
    }
    __syncthreads();
    // along c and the sum over directions: line (el, b, a), NQ -> N1
    for (int t = tid; t < EPB * NF2; t += 256) {
      const int el = t / NF2, ba = t - el * NF2;
      const int e = e0 + el < E ? e0 + el : E - 1;
      const int cx = e % A.nx, cxy = e / A.nx;
      const double ihx = A.ih[cx], ihy = A.ih[A.nx + cxy % A.ny], ihz = A.ih[A.nx + A.ny + cxy / A.ny];
      double vx[N1], vy[N1], vz[N1];
      line<N1, NQ>(Pm, sR2 + (el * 3 + 0) * (NQ * NF2) + ba, NF2, vx, 1);
      line<N1, NQ>(Pm, sR2 + (el * 3 + 1) * (NQ * NF2) + ba, NF2, vy, 1);
      line<N1, NQ>(S, sR2 + (el * 3 + 2) * (NQ * NF2) + ba, NF2, vz, 1);
#pragma unroll
      for (int c = 0; c < N1; ++c) sOut[(el * 5 + f) * NP + c * NF2 + ba] = ihx * vx[c] + ihy * vy[c] + ihz * vz[c];
    }
    __syncthreads();
  }

  // (3) faces: the neighbour face nodes into LDS (the flux region is free now)
#pragma unroll
  for (int u = 0; u < C::KN; ++u) {
    const int t = tid + 256 * u;
    if (t < EPB * 6 * 5 * NF2) sF[t] = nb[u];
  }
  __syncthreads();
#pragma unroll 1
  for (int face = 0; face < 6; ++face) {
    const int d = face >> 1, side = face & 1;
    const int fo = side ? P : 0;
    // interpolation along the face's fast axis: line (el, s2, f, slow), own (s2 = 0) and neighbour (1)
    for (int t = tid; t < EPB * 2 * 5 * N1; t += 256) {
      const int el = t / (10 * N1), r = t - el * (10 * N1), s2 = r / (5 * N1), r2 = r - s2 * (5 * N1);
      const int f = r2 / N1, slow = r2 - f * N1;
      double* out = sR1 + ((el * 2 + s2) * 5 + f) * (N1 * NQ) + slow * NQ;
      if (s2 == 0) {
        const double* qe = sQ + (el * 5 + f) * NP;
        if (d == 0) line<NQ, N1>(B, qe + fo + N1 * N1 * slow, N1, out, 1);
        else if (d == 1) line<NQ, N1>(B, qe + N1 * fo + NF2 * slow, 1, out, 1);
        else line<NQ, N1>(B, qe + N1 * slow + NF2 * fo, 1, out, 1);
      } else {
        line<NQ, N1>(B, sF + ((el * 6 + face) * 5 + f) * NF2 + slow * N1, 1, out, 1);
      }
    }
    __syncthreads();
    // along the slow axis: line (el, s2, f, kf)
    for (int t = tid; t < EPB * 2 * 5 * NQ; t += 256) {
      const int g = t / NQ, kf = t - g * NQ;  // g = (el, s2, f)
      line<NQ, N1>(B, sR1 + g * (N1 * NQ) + kf, NQ, sR2 + g * (NQ * NQ) + kf, NQ);
    }
    __syncthreads();
    // Lax-Friedrichs flux at the face quad points
    double* fh = sR1 + EPB * 2 * 5 * N1 * NQ;  // after the face interpolation buffer
    for (int t = tid; t < EPB * NQ * NQ; t += 256) {
      const int el = t / (NQ * NQ), k2 = t - el * (NQ * NQ);
      double qm[5], qp[5];
#pragma unroll
      for (int f = 0; f < 5; ++f) {
        qm[f] = sR2[((el * 2 + 0) * 5 + f) * (NQ * NQ) + k2];
        qp[f] = sR2[((el * 2 + 1) * 5 + f) * (NQ * NQ) + k2];
      }
      double um, vm, wm, pm, up, vp, wp, pp;
      prim(qm, A.gamma, um, vm, wm, pm);
      prim(qp, A.gamma, up, vp, wp, pp);
      const double udm = d == 0 ? um : d == 1 ? vm : wm, udp = d == 0 ? up : d == 1 ? vp : wp;
      const double lam = fmax(fabs(udm) + sqrt(A.gamma * pm / qm[0]), fabs(udp) + sqrt(A.gamma * pp / qp[0]));
      const double sg = side ? 0.5 : -0.5;
#pragma unroll
      for (int f = 0; f < 5; ++f) {
        const double Fm = (f == 4 ? qm[4] + pm : qm[f]) * udm + (f == 1 + d ? pm : 0.0);
        const double Fp = (f == 4 ? qp[4] + pp : qp[f]) * udp + (f == 1 + d ? pp : 0.0);
        fh[(el * 5 + f) * (NQ * NQ) + k2] = sg * (Fm + Fp) + 0.5 * lam * (qm[f] - qp[f]);
      }
    }
    __syncthreads();
    // projection along the fast axis: line (el, f, ks), NQ -> N1
    double* g1 = sF + EPB * 6 * 5 * NF2;  // after the neighbour face nodes
    for (int t = tid; t < EPB * 5 * NQ; t += 256)
      line<N1, NQ>(Pm, fh + t * NQ, 1, g1 + t * N1, 1);
    __syncthreads();
    // along the slow axis and the lift: line (el, f, fast), NQ -> N1; each
    // output (slow, fast) is lifted along the face's normal line
    for (int t = tid; t < EPB * 5 * N1; t += 256) {
      const int ef = t / N1, fast = t - ef * N1, el = ef / 5, f = ef - el * 5;
      double g2[N1];
      line<N1, NQ>(Pm, g1 + ef * (NQ * N1) + fast, N1, g2, 1);
      const int e = e0 + el < E ? e0 + el : E - 1;
      const int cx = e % A.nx, cxy = e / A.nx;
      const double ihd = d == 0 ? A.ih[cx] : d == 1 ? A.ih[A.nx + cxy % A.ny] : A.ih[A.nx + A.ny + cxy / A.ny];
      double* out = sOut + (el * 5 + f) * NP;
#pragma unroll
      for (int slow = 0; slow < N1; ++slow) {
        const double gv = ihd * g2[slow];
#pragma unroll
        for (int i = 0; i < N1; ++i) {
          const int node = d == 0 ? i + N1 * (fast + N1 * slow) : d == 1 ? fast + N1 * (i + N1 * slow)
                                                                         : fast + N1 * (slow + N1 * i);
          out[node] -= lift[i * 2 + side] * gv;
        }
      }
    }
    __syncthreads();
  }

  // (4) store or stage update (coalesced per field)
  bool bad = false;
#pragma unroll
  for (int u = 0; u < C::KR; ++u) {
    const int t = tid + 256 * u;
    if (t < EPB * 5 * NP) {
      const int f = t / (EPB * NP), r = t - f * (EPB * NP);
      const int el = r / NP, n = r - el * NP;
      if (e0 + el < E) {
        const double val = sOut[(el * 5 + f) * NP + n];
        const size_t gi = f * Es + static_cast<size_t>(e0 + el) * NP + n;
        if (FUSED) {
          const double rr = (A.a == 0.0 ? 0.0 : A.a * rv[u]) + A.dt * val;
          const double qn = sQ[(el * 5 + f) * NP + n] + A.b * rr;
          A.res[gi] = rr;
          A.qout[gi] = qn;
          bad |= nonfinite(qn);
        } else {
          A.rhs[gi] = val;
          bad |= nonfinite(val);
        }
      }
    }
  }
  raise_flag(A.flags, bad, kFlagNonFinite);
}

template <int P>
dg_status launch_oi_p(const HexMesh& m, const OiArgs& A, bool fused, hipStream_t s) {
  using C = OiCfg<P>;
  static_assert(C::PER_EL * C::EPB * 8 <= 65536, "LDS budget");
  const int64_t blocks = (m.E + C::EPB - 1) / C::EPB;
  if (fused)
    hipLaunchKernelGGL((hex_oi_kernel<P, true>), dim3(static_cast<unsigned>(blocks)), dim3(256), 0, s, A);
  else
    hipLaunchKernelGGL((hex_oi_kernel<P, false>), dim3(static_cast<unsigned>(blocks)), dim3(256), 0, s, A);
  const hipError_t e = hipGetLastError();
  return e == hipSuccess ? DG_OK : hip_fail(e, "hex overintegrated rhs launch");
}

}  // namespace

int hex_oi_points(int p) { return oi_nq(p); }

dg_status launch_rhs_hex_oi(const HexMesh& m, double gamma, const double* q, double* rhs, double* res, double* q_out,
                            double a, double b, double dt, bool fused, hipStream_t s) {
  OiArgs A;
  A.q = q;
  A.rhs = rhs;
  A.res = res;
  A.qout = q_out;
  A.ih = m.d_ih;
  A.op = m.d_oi;
  A.nx = m.nx;
  A.ny = m.ny;
  A.nz = m.nz;
  A.E = static_cast<int>(m.E);
  A.gamma = gamma;
  A.a = a;
  A.b = b;
  A.dt = dt;
  A.flags = device_flags();
  switch (m.p) {
    case 1: return launch_oi_p<1>(m, A, fused, s);
    case 2: return launch_oi_p<2>(m, A, fused, s);
    case 3: return launch_oi_p<3>(m, A, fused, s);
    case 4: return launch_oi_p<4>(m, A, fused, s);
    default: return fail(DG_ERR_ARG, "hex overintegrated rhs: unsupported order");
  }
}

}  // namespace dg
