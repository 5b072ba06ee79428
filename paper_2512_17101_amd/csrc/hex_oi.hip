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
// At p = 4 this is about 420 kflop per element against 10 kB of state: the
// FP64 pipe bounds it, not HBM.
//
// One wave owns max(1, 64 / nq^2) elements (one at p = 3, 4; two at p = 2;
// seven at p = 1) and is its own workgroup, so the passes are separated by
// single-wave barriers.  Two kinds of pass:
//  - line passes: a lane takes one line of an LDS array, loads its inputs
//    into registers and forms every output of the line; the operator entries
//    are compile-time indices into a uniform table (scalar loads);
//  - column passes: a lane owns one (k1, k2) column of the element's quad
//    grid (or one face quad point) and keeps its values in registers: the
//    last interpolation pass, the fluxes and the first projection pass of
//    the volume term, and the second face interpolation pass plus the
//    Lax-Friedrichs flux, need no LDS round trip.
// Faces come first (own and neighbour traces at the face quad points, the
// flux there, its projection back to the face nodes, kept in LDS), then the
// volume term field by field, to which each node adds the lifted face terms
// of its line before the coalesced store (or the fused Runge-Kutta stage).
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
  static constexpr int QF = NQ * NQ;
  static constexpr int EPW = QF >= 64 ? 1 : 64 / QF;  // elements per wave
  // LDS row strides of arrays whose rows are one lane's line: odd, so that
  // the lanes of a wave spread over the banks (an even stride of 8 doubles
  // puts 16 lanes on one bank)
  static constexpr int NQP = NQ | 1, N1P = N1 | 1;
  // offsets of the operator table [B (NQ x N1) | S (N1 x NQ) | P (N1 x NQ) | lift (N1 x 2)]
  static constexpr int OB = 0, OS = NQ * N1, OP = 2 * NQ * N1, OL = 3 * NQ * N1;
  // LDS per element (doubles): own nodal state, the six face slices (the
  // neighbour's nodes, then the projected face flux), scratch
  static constexpr int L_Q = 5 * NP;
  static constexpr int L_F = 6 * 5 * NF2;
  // scratch layouts (row strides padded to NQP, N1P):
  //   volume interpolation  W1 [NF2][NQP] at 0, W2 [N1][QF] at NF2 NQP
  //   volume projection     Hs [N1][QF] at 0,   Gs [NF2][NQP] at N1 QF
  //   faces                 T1 [2][5][N1][NQP], then Fh [5][NQ][NQP], at 0;
  //                         U [5][NQ][N1P] at X_U
  static constexpr int X_U = cmax(2 * 5 * N1 * NQP, 5 * NQ * NQP);
  static constexpr int L_S = cmax(NF2 * NQP + N1 * QF, X_U + 5 * NQ * N1P);
  static constexpr int PER_EL = L_Q + L_F + L_S;
  static constexpr int KQ = (EPW * 5 * NP + 63) / 64;       // own state loads per lane
  static constexpr int KN = (EPW * 6 * 5 * NF2 + 63) / 64;  // neighbour face loads per lane
  static_assert(EPW * QF <= 64, "one column per lane");
  static_assert(EPW * NF2 <= 64, "one output line per lane");
};

struct OiArgs {
  const double* __restrict__ q;
  double* __restrict__ rhs;
  const double* res_in;  // may alias res or qout (entry-wise)
  double* res;           // null: the new residual is not stored
  double* qout;
  const double* __restrict__ ih;  // [nx | ny | nz] 2 / h
  const double* __restrict__ op;  // [B | S | P | lift]
  int nx, ny, nz;
  int E;
  double gamma, a, b, dt;
  unsigned* flags;
};

typedef const __attribute__((address_space(4))) double cdouble;
// The operator entries of one output of a line, read through the constant
// address space at an offset the compiler cannot see through: scalar loads
// issued at each use.  With plain loads the compiler hoisted every table
// entry out of the loops (about 130 doubles at p = 4), overflowed the
// scalar registers, spilled them to vector-register lanes (some 1,500
// v_readlane / v_writelane per wave) and ran out of vector registers.
// At p = 1 (2 x 3 operators, 22 table entries in all) the hoisted values fit
// and the plain loads are faster.
template <int NO, int NI>
__device__ inline cdouble* op_at(const double* A) {
  int z = 0;
  if constexpr (NO * NI > 8) asm volatile("s_mov_b32 %0, 0" : "=s"(z));
  return (cdouble*)(reinterpret_cast<uintptr_t>(A)) + __builtin_amdgcn_readfirstlane(z);
}

// out[o * so] = sum_i A[o * NI + i] in[i * si]: one line, operator entries at
// compile-time offsets of a uniform table
template <int NO, int NI>
__device__ inline void line(const double* __restrict__ A0, const double* in, int si, double* out, int so) {
  double x[NI];
#pragma unroll
  for (int i = 0; i < NI; ++i) x[i] = in[i * si];
#pragma unroll
  for (int o = 0; o < NO; ++o) {
    cdouble* A = op_at<NO, NI>(A0);
    double s = 0.0;
#pragma unroll
    for (int i = 0; i < NI; ++i) s = fma(A[o * NI + i], x[i], s);
    out[o * so] = s;
  }
}

// the same, with the line's inputs already in registers
template <int NO, int NI>
__device__ inline void line_r(const double* __restrict__ A0, const double (&x)[NI], double (&out)[NO]) {
#pragma unroll
  for (int o = 0; o < NO; ++o) {
    cdouble* A = op_at<NO, NI>(A0);
    double s = 0.0;
#pragma unroll
    for (int i = 0; i < NI; ++i) s = fma(A[o * NI + i], x[i], s);
    out[o] = s;
  }
}

// the element across face (d, side) of element e on the periodic grid
__device__ inline int face_neighbour(int e, int d, int side, int nx, int ny, int nz) {
  const int cx = e % nx, cxy = e / nx, cy = cxy % ny, cz = cxy / ny;
  const int cd = d == 0 ? cx : d == 1 ? cy : cz;
  const int nd = d == 0 ? nx : d == 1 ? ny : nz;
  const int stride = d == 0 ? 1 : d == 1 ? nx : nx * ny;
  return side ? (cd == nd - 1 ? e - (nd - 1) * stride : e + stride) : (cd == 0 ? e + (nd - 1) * stride : e - stride);
}

// the volume node at face coordinates (i1 fast, i2 slow) of face d, fixed
// coordinate fo along d
template <int N1>
__device__ inline int face_node(int d, int fo, int i1, int i2) {
  return d == 0 ? fo + N1 * (i1 + N1 * i2) : d == 1 ? i1 + N1 * (fo + N1 * i2) : i1 + N1 * (i2 + N1 * fo);
}

// Registers: the column state (six values at nq points) plus one line's
// operands; about 185-200 at p = 4 (two waves per SIMD, where the 16 kB of
// LDS per element would allow 2.5), 140-155 at p = 3.
template <int P, bool FUSED>
__global__ __launch_bounds__(64) void hex_oi_kernel(OiArgs A) {
  using C = OiCfg<P>;
  constexpr int N1 = C::N1, NQ = C::NQ, NP = C::NP, NF2 = C::NF2, QF = C::QF, EPW = C::EPW;
  constexpr int NQP = C::NQP, N1P = C::N1P;
  __shared__ double s_mem[EPW * C::PER_EL];
  double* sQ = s_mem;                  // [EPW][5][NP]
  double* sF = sQ + EPW * C::L_Q;      // [EPW][6][5][NF2]
  double* sS = sF + EPW * C::L_F;      // [EPW][L_S]
  const int lane = threadIdx.x;
  const int E = A.E;
  const int e0 = blockIdx.x * EPW;
  const size_t Es = static_cast<size_t>(E) * NP;
  const double* B = A.op + C::OB;
  const double* S = A.op + C::OS;
  const double* Pm = A.op + C::OP;
  const double* lift = A.op + C::OL;
  const double g = A.gamma;

  // (0) own state (coalesced per field) and the neighbours' face nodes, all
  // loads issued before the first LDS write
  {
    double qo[C::KQ], nb[C::KN];
#pragma unroll
    for (int u = 0; u < C::KQ; ++u) {
      const int t0 = lane + 64 * u;
      const int t = t0 < EPW * 5 * NP ? t0 : EPW * 5 * NP - 1;
      const int f = t / (EPW * NP), r = t - f * (EPW * NP);
      const int el = r / NP, n = r - el * NP;
      const int e = e0 + el < E ? e0 + el : E - 1;
      qo[u] = A.q[f * Es + static_cast<size_t>(e) * NP + n];
    }
#pragma unroll
    for (int u = 0; u < C::KN; ++u) {
      const int t0 = lane + 64 * u;
      const int t = t0 < EPW * 6 * 5 * NF2 ? t0 : EPW * 6 * 5 * NF2 - 1;
      const int el = t / (6 * 5 * NF2), r = t - el * (6 * 5 * NF2);
      const int face = r / (5 * NF2), r2 = r - face * (5 * NF2);
      const int f = r2 / NF2, m = r2 - f * NF2;
      const int d = face >> 1, side = face & 1;
      const int e = e0 + el < E ? e0 + el : E - 1;
      const int en = face_neighbour(e, d, side, A.nx, A.ny, A.nz);
      nb[u] = A.q[f * Es + static_cast<size_t>(en) * NP + face_node<N1>(d, side ? 0 : P, m % N1, m / N1)];
    }
#pragma unroll
    for (int u = 0; u < C::KQ; ++u) {
      const int t = lane + 64 * u;
      if (t < EPW * 5 * NP) {
        const int f = t / (EPW * NP), r = t - f * (EPW * NP);
        const int el = r / NP, n = r - el * NP;
        sQ[(el * 5 + f) * NP + n] = qo[u];
      }
    }
#pragma unroll
    for (int u = 0; u < C::KN; ++u) {
      const int t = lane + 64 * u;
      if (t < EPW * 6 * 5 * NF2) sF[t] = nb[u];
    }
  }
  __syncthreads();

  // column-pass identity of this lane: element cel, quad column / face point
  // ck = k2 NQ + k1 (idle lanes read in-bounds scratch and write nothing)
  const bool col = lane < EPW * QF;
  const int cel = col ? lane / QF : 0;
  const int ck = lane - cel * QF;
  const int ck2 = col ? ck / NQ : 0;
  const int ck1 = ck - ck2 * NQ;
  double* cS = sS + cel * C::L_S;

  // (1) faces: Fhat at the face quad points, projected back to the face
  // nodes with P x P, stored over that face's neighbour slice
  {
    double Brow[N1];  // row k2 of B, for this lane's face point
#pragma unroll
    for (int i = 0; i < N1; ++i) Brow[i] = B[ck2 * N1 + i];
#pragma unroll 1
    for (int face = 0; face < 6; ++face) {
      const int d = face >> 1, side = face & 1;
      const int fo = side ? P : 0;
      // own (s2 = 0) and neighbour (1) traces along the face's fast axis:
      // T1[s2][f][i2][k1]
      for (int t = lane; t < EPW * 2 * 5 * N1; t += 64) {
        const int el = t / (10 * N1), r = t - el * (10 * N1), s2 = r / (5 * N1), r2 = r - s2 * (5 * N1);
        const int f = r2 / N1, i2 = r2 - f * N1;
        double* out = sS + el * C::L_S + ((s2 * 5 + f) * N1 + i2) * NQP;
        if (s2 == 0)
          line<NQ, N1>(B, sQ + (el * 5 + f) * NP + face_node<N1>(d, fo, 0, i2), d == 0 ? N1 : 1, out, 1);
        else
          line<NQ, N1>(B, sF + ((el * 6 + face) * 5 + f) * NF2 + i2 * N1, 1, out, 1);
      }
      __syncthreads();
      // along the slow axis in registers, then the Lax-Friedrichs flux
      double fh[5];
      if (col) {
        double qm[5], qp[5];
#pragma unroll
        for (int f = 0; f < 5; ++f) {
          double sm = 0.0, sp = 0.0;
#pragma unroll
          for (int i2 = 0; i2 < N1; ++i2) {
            sm = fma(Brow[i2], cS[((0 * 5 + f) * N1 + i2) * NQP + ck1], sm);
            sp = fma(Brow[i2], cS[((1 * 5 + f) * N1 + i2) * NQP + ck1], sp);
          }
          qm[f] = sm;
          qp[f] = sp;
        }
        const double irm = 1.0 / qm[0], irp = 1.0 / qp[0];
        const double um = qm[1] * irm, vm = qm[2] * irm, wm = qm[3] * irm;
        const double up = qp[1] * irp, vp = qp[2] * irp, wp = qp[3] * irp;
        const double pm = (g - 1.0) * (qm[4] - 0.5 * (qm[1] * um + qm[2] * vm + qm[3] * wm));
        const double pp = (g - 1.0) * (qp[4] - 0.5 * (qp[1] * up + qp[2] * vp + qp[3] * wp));
        const double udm = d == 0 ? um : d == 1 ? vm : wm, udp = d == 0 ? up : d == 1 ? vp : wp;
        const double lam = fmax(fabs(udm) + sqrt(g * pm * irm), fabs(udp) + sqrt(g * pp * irp));
        const double sg = side ? 0.5 : -0.5;
#pragma unroll
        for (int f = 0; f < 5; ++f) {
          const double Fm = (f == 4 ? qm[4] + pm : qm[f]) * udm + (f == 1 + d ? pm : 0.0);
          const double Fp = (f == 4 ? qp[4] + pp : qp[f]) * udp + (f == 1 + d ? pp : 0.0);
          fh[f] = sg * (Fm + Fp) + 0.5 * lam * (qm[f] - qp[f]);
        }
      }
      __syncthreads();  // T1 read: Fh takes its place
      if (col) {
#pragma unroll
        for (int f = 0; f < 5; ++f) cS[(f * NQ + ck2) * NQP + ck1] = fh[f];
      }
      __syncthreads();
      // projection along the fast axis: U[f][k2][i1]
      for (int t = lane; t < EPW * 5 * NQ; t += 64) {
        const int el = t / (5 * NQ), r = t - el * (5 * NQ);  // r = f NQ + k2
        double* base = sS + el * C::L_S;
        line<N1, NQ>(Pm, base + r * NQP, 1, base + C::X_U + r * N1P, 1);
      }
      __syncthreads();
      // along the slow axis, over the neighbour slice: g[f][i2][i1]
      for (int t = lane; t < EPW * 5 * N1; t += 64) {
        const int el = t / (5 * N1), r = t - el * (5 * N1), f = r / N1, i1 = r - f * N1;
        line<N1, NQ>(Pm, sS + el * C::L_S + C::X_U + f * NQ * N1P + i1, N1P,
                     sF + ((el * 6 + face) * 5 + f) * NF2 + i1, N1);
      }
      __syncthreads();
    }
  }

  // (2) the state at the volume quad points, in this lane's column: 1 / rho,
  // the momenta, the pressure and E + p at its NQ points
  double irho[NQ], mx[NQ], my[NQ], mz[NQ], pr[NQ], en[NQ];
#pragma unroll
  for (int f = 0; f < 5; ++f) {
    // along a: W1[cb][ka]
    for (int t = lane; t < EPW * NF2; t += 64) {
      const int el = t / NF2, cb = t - el * NF2;
      line<NQ, N1>(B, sQ + (el * 5 + f) * NP + cb * N1, 1, sS + el * C::L_S + cb * NQP, 1);
    }
    __syncthreads();
    // along b: W2[c][kb][ka]
    for (int t = lane; t < EPW * N1 * NQ; t += 64) {
      const int el = t / (N1 * NQ), r = t - el * (N1 * NQ), c = r / NQ, ka = r - c * NQ;
      double* base = sS + el * C::L_S;
      line<NQ, N1>(B, base + c * N1 * NQP + ka, NQP, base + NF2 * NQP + c * QF + ka, NQ);
    }
    __syncthreads();
    // along c, in registers (the next field's first pass writes W1 only, and
    // W2 is rewritten only after the barrier that follows it)
    double x[N1], z[NQ];
#pragma unroll
    for (int c = 0; c < N1; ++c) x[c] = cS[NF2 * NQP + c * QF + ck];
    line_r<NQ, N1>(B, x, z);
#pragma unroll
    for (int k = 0; k < NQ; ++k) {
      if (f == 0) irho[k] = 1.0 / z[k];
      if (f == 1) mx[k] = z[k];
      if (f == 2) my[k] = z[k];
      if (f == 3) mz[k] = z[k];
      if (f == 4) {
        const double u = mx[k] * irho[k], v = my[k] * irho[k], w = mz[k] * irho[k];
        pr[k] = (g - 1.0) * (z[k] - 0.5 * (mx[k] * u + my[k] * v + mz[k] * w));
        en[k] = z[k] + pr[k];
      }
    }
  }

  // (3) volume term and the lifted face terms, field by field.  Output line
  // of this lane: element lel, nodes (a, b = lb, c = lc), a = 0..p.
  const bool own = lane < EPW * NF2;
  const int lel = own ? lane / NF2 : 0;
  const int lcb = own ? lane - lel * NF2 : 0;  // idle lanes keep in-bounds addresses
  const int lc = lcb / N1, lb = lcb - lc * N1;
  const int le = e0 + lel < E ? e0 + lel : E - 1;
  const bool lvalid = own && e0 + lel < E;
  const int lcx = le % A.nx, lcxy = le / A.nx;
  const double ihx = A.ih[lcx], ihy = A.ih[A.nx + lcxy % A.ny], ihz = A.ih[A.nx + A.ny + lcxy / A.ny];
  const double lb0 = lift[lb * 2], lb1 = lift[lb * 2 + 1], lc0 = lift[lc * 2], lc1 = lift[lc * 2 + 1];
  const double* lS = sS + lel * C::L_S;
  const double* lF = sF + lel * (6 * 5 * NF2);
  bool bad = false;
#pragma unroll
  for (int f = 0; f < 5; ++f) {
    const size_t gbase = f * Es + static_cast<size_t>(le) * NP + lcb * N1;
    double rv[N1];
    if (FUSED) {
#pragma unroll
      for (int a = 0; a < N1; ++a) rv[a] = A.a != 0.0 ? A.res_in[gbase + a] : 0.0;
    }
    double acc[N1];
#pragma unroll
    for (int a = 0; a < N1; ++a) acc[a] = 0.0;
#pragma unroll 1
    for (int d = 0; d < 3; ++d) {
      // flux component d of field f at the column's points, projected along c
      // (S for d = z, P otherwise): Hs[c][kb][ka]
      if (col) {
        double F[NQ], H[N1];
#pragma unroll
        for (int k = 0; k < NQ; ++k) {
          const double md = d == 0 ? mx[k] : d == 1 ? my[k] : mz[k];
          const double ud = md * irho[k];
          F[k] = f == 0 ? md
                 : f == 4 ? en[k] * ud
                          : (f == 1 ? mx[k] : f == 2 ? my[k] : mz[k]) * ud + (f == 1 + d ? pr[k] : 0.0);
        }
        line_r<N1, NQ>(d == 2 ? S : Pm, F, H);
#pragma unroll
        for (int c = 0; c < N1; ++c) cS[c * QF + ck] = H[c];
      }
      __syncthreads();
      // along b (S for d = y): Gs[c][b][ka]
      for (int t = lane; t < EPW * N1 * NQ; t += 64) {
        const int el = t / (N1 * NQ), r = t - el * (N1 * NQ), c = r / NQ, ka = r - c * NQ;
        double* base = sS + el * C::L_S;
        line<N1, NQ>(d == 1 ? S : Pm, base + c * QF + ka, NQ, base + N1 * QF + c * N1 * NQP + ka, NQP);
      }
      __syncthreads();
      // along a (S for d = x), into this lane's output line
      if (own) {
        double x[NQ], y[N1];
#pragma unroll
        for (int k = 0; k < NQ; ++k) x[k] = lS[N1 * QF + lcb * NQP + k];
        line_r<N1, NQ>(d == 0 ? S : Pm, x, y);
        const double ih = d == 0 ? ihx : d == 1 ? ihy : ihz;
#pragma unroll
        for (int a = 0; a < N1; ++a) acc[a] = fma(ih, y[a], acc[a]);
      }
      // the next component's column pass writes Hs only, whose last reads
      // came before the barrier above; Gs is rewritten after the next one
    }
    if (own) {
      // lifted face fluxes: x faces at (i1, i2) = (b, c), y at (a, c), z at (a, b)
      const double* gx0 = lF + (0 * 5 + f) * NF2;
      const double* gx1 = lF + (1 * 5 + f) * NF2;
      const double* gy0 = lF + (2 * 5 + f) * NF2;
      const double* gy1 = lF + (3 * 5 + f) * NF2;
      const double* gz0 = lF + (4 * 5 + f) * NF2;
      const double* gz1 = lF + (5 * 5 + f) * NF2;
      const double sx0 = gx0[lc * N1 + lb], sx1 = gx1[lc * N1 + lb];
#pragma unroll
      for (int a = 0; a < N1; ++a) {
        const double sx = lift[a * 2] * sx0 + lift[a * 2 + 1] * sx1;
        const double sy = lb0 * gy0[lc * N1 + a] + lb1 * gy1[lc * N1 + a];
        const double sz = lc0 * gz0[lb * N1 + a] + lc1 * gz1[lb * N1 + a];
        const double out = acc[a] - (ihx * sx + ihy * sy + ihz * sz);
        if (lvalid) {
          if (FUSED) {
            const double rr = (A.a == 0.0 ? 0.0 : A.a * rv[a]) + A.dt * out;
            const double qn = sQ[(lel * 5 + f) * NP + lcb * N1 + a] + A.b * rr;
            if (A.res) A.res[gbase + a] = rr;
            A.qout[gbase + a] = qn;
            bad |= nonfinite(qn);
          } else {
            A.rhs[gbase + a] = out;
            bad |= nonfinite(out);
          }
        }
      }
    }
  }
  raise_flag(A.flags, bad, kFlagNonFinite);
}

// One face of the p = 1 element: Fhat at the face's 3 x 3 quad points,
// lifted onto the element's nodes (direction and side at compile time, so
// that every register-array index is a constant).
template <int d, int side>
__device__ inline void p1_face(const OiArgs& A, int ec, size_t Es, double ihx, double ihy, double ihz,
                               const double (&q)[5][8], double (&out)[5][8]) {
  constexpr int NQ = 3;
  const double* __restrict__ B = A.op;
  const double* __restrict__ Pm = A.op + 12;
  const double* __restrict__ lift = A.op + 18;
  const double g = A.gamma;
  const int fo = side, fn = 1 - side;  // own / neighbour node coordinate along d
  const double ihd = d == 0 ? ihx : d == 1 ? ihy : ihz;
  const int en = face_neighbour(ec, d, side, A.nx, A.ny, A.nz);
  double qn[5][4];
#pragma unroll
  for (int f = 0; f < 5; ++f)
#pragma unroll
    for (int m = 0; m < 4; ++m)
      qn[f][m] = A.q[f * Es + static_cast<size_t>(en) * 8 + face_node<2>(d, fn, m & 1, m >> 1)];
  const double sg = side ? 0.5 : -0.5;
#pragma unroll 1
  for (int k2 = 0; k2 < NQ; ++k2)
#pragma unroll 1
    for (int k1 = 0; k1 < NQ; ++k1) {
      double wf[4];
#pragma unroll
      for (int m = 0; m < 4; ++m) wf[m] = B[k1 * 2 + (m & 1)] * B[k2 * 2 + (m >> 1)];
      double qm[5], qp[5];
#pragma unroll
      for (int f = 0; f < 5; ++f) {
        double tm = 0.0, tp = 0.0;
#pragma unroll
        for (int m = 0; m < 4; ++m) {
          tm = fma(wf[m], q[f][face_node<2>(d, fo, m & 1, m >> 1)], tm);
          tp = fma(wf[m], qn[f][m], tp);
        }
        qm[f] = tm;
        qp[f] = tp;
      }
      const double irm = 1.0 / qm[0], irp = 1.0 / qp[0];
      const double um = qm[1] * irm, vm = qm[2] * irm, wm = qm[3] * irm;
      const double up = qp[1] * irp, vp = qp[2] * irp, wp = qp[3] * irp;
      const double pm = (g - 1.0) * (qm[4] - 0.5 * (qm[1] * um + qm[2] * vm + qm[3] * wm));
      const double pp = (g - 1.0) * (qp[4] - 0.5 * (qp[1] * up + qp[2] * vp + qp[3] * wp));
      const double udm = d == 0 ? um : d == 1 ? vm : wm, udp = d == 0 ? up : d == 1 ? vp : wp;
      const double lam = fmax(fabs(udm) + sqrt(g * pm * irm), fabs(udp) + sqrt(g * pp * irp));
      double fh[5];
#pragma unroll
      for (int f = 0; f < 5; ++f) {
        const double Fm = (f == 4 ? qm[4] + pm : qm[f]) * udm + (f == 1 + d ? pm : 0.0);
        const double Fp = (f == 4 ? qp[4] + pp : qp[f]) * udp + (f == 1 + d ? pp : 0.0);
        fh[f] = ihd * (sg * (Fm + Fp) + 0.5 * lam * (qm[f] - qp[f]));
      }
#pragma unroll
      for (int m = 0; m < 4; ++m) {
        const double pw = Pm[(m & 1) * 3 + k1] * Pm[(m >> 1) * 3 + k2];
#pragma unroll
        for (int i = 0; i < 2; ++i) {
          const double cf = lift[i * 2 + side] * pw;
          const int node = face_node<2>(d, i, m & 1, m >> 1);
#pragma unroll
          for (int f = 0; f < 5; ++f) out[f][node] = fma(-cf, fh[f], out[f][node]);
        }
      }
    }
}

// p = 1: one lane per element with the element in registers.  A quad line
// has three points and a node line two, so the wave-per-element passes spend
// more on LDS round trips and per-line index arithmetic than on the
// contractions; here each quad point is evaluated directly: the eight
// interpolation weights B_ka,a B_kb,b B_kc,c, the flux there, and its
// projection onto the eight nodes with the coefficients (S x P x P, P x S x P,
// P x P x S)(2 / h).  The table entries are uniform (scalar loads).
template <bool FUSED>
__global__ __launch_bounds__(256) __attribute__((amdgpu_waves_per_eu(2))) void hex_oi_p1_kernel(OiArgs A) {
  constexpr int NQ = 3;
  const double* __restrict__ B = A.op;            // [3][2]
  const double* __restrict__ S = A.op + 6;        // [2][3]
  const double* __restrict__ Pm = A.op + 12;      // [2][3]
  const double* __restrict__ lift = A.op + 18;    // [2][2]
  const int E = A.E;
  const int e = blockIdx.x * 256 + threadIdx.x;
  const bool valid = e < E;
  const int ec = valid ? e : E - 1;
  const size_t Es = static_cast<size_t>(E) * 8;
  const double g = A.gamma;
  double q[5][8];
#pragma unroll
  for (int f = 0; f < 5; ++f)
#pragma unroll
    for (int n = 0; n < 8; ++n) q[f][n] = A.q[f * Es + static_cast<size_t>(ec) * 8 + n];
  const int cx = ec % A.nx, cxy = ec / A.nx;
  const double ihx = A.ih[cx], ihy = A.ih[A.nx + cxy % A.ny], ihz = A.ih[A.nx + A.ny + cxy / A.ny];
  double out[5][8];
#pragma unroll
  for (int f = 0; f < 5; ++f)
#pragma unroll
    for (int n = 0; n < 8; ++n) out[f][n] = 0.0;

  // volume: sum over the quad points of the projected fluxes
#pragma unroll 1
  for (int kc = 0; kc < NQ; ++kc)
#pragma unroll 1
    for (int kb = 0; kb < NQ; ++kb)
#pragma unroll 1
      for (int ka = 0; ka < NQ; ++ka) {
        double z[5];
        {
          double w[8];
#pragma unroll
          for (int n = 0; n < 8; ++n) w[n] = B[ka * 2 + (n & 1)] * B[kb * 2 + ((n >> 1) & 1)] * B[kc * 2 + (n >> 2)];
#pragma unroll
          for (int f = 0; f < 5; ++f) {
            double t = 0.0;
#pragma unroll
            for (int n = 0; n < 8; ++n) t = fma(w[n], q[f][n], t);
            z[f] = t;
          }
        }
        const double ir = 1.0 / z[0];
        const double u = z[1] * ir, v = z[2] * ir, w = z[3] * ir;
        const double pr = (g - 1.0) * (z[4] - 0.5 * (z[1] * u + z[2] * v + z[3] * w));
        const double en = z[4] + pr;
        // (2 / h_d) F_d of the five fields
        const double Fx[5] = {ihx * z[1], ihx * (z[1] * u + pr), ihx * (z[2] * u), ihx * (z[3] * u), ihx * (en * u)};
        const double Fy[5] = {ihy * z[2], ihy * (z[1] * v), ihy * (z[2] * v + pr), ihy * (z[3] * v), ihy * (en * v)};
        const double Fz[5] = {ihz * z[3], ihz * (z[1] * w), ihz * (z[2] * w), ihz * (z[3] * w + pr), ihz * (en * w)};
#pragma unroll
        for (int n = 0; n < 8; ++n) {
          const int a = n & 1, b = (n >> 1) & 1, c = n >> 2;
          const double cxn = S[a * 3 + ka] * Pm[b * 3 + kb] * Pm[c * 3 + kc];
          const double cyn = Pm[a * 3 + ka] * S[b * 3 + kb] * Pm[c * 3 + kc];
          const double czn = Pm[a * 3 + ka] * Pm[b * 3 + kb] * S[c * 3 + kc];
#pragma unroll
          for (int f = 0; f < 5; ++f) out[f][n] = fma(cxn, Fx[f], fma(cyn, Fy[f], fma(czn, Fz[f], out[f][n])));
        }
      }

  // faces
  p1_face<0, 0>(A, ec, Es, ihx, ihy, ihz, q, out);
  p1_face<0, 1>(A, ec, Es, ihx, ihy, ihz, q, out);
  p1_face<1, 0>(A, ec, Es, ihx, ihy, ihz, q, out);
  p1_face<1, 1>(A, ec, Es, ihx, ihy, ihz, q, out);
  p1_face<2, 0>(A, ec, Es, ihx, ihy, ihz, q, out);
  p1_face<2, 1>(A, ec, Es, ihx, ihy, ihz, q, out);

  bool bad = false;
  if (valid) {
#pragma unroll
    for (int f = 0; f < 5; ++f)
#pragma unroll
      for (int n = 0; n < 8; ++n) {
        const size_t gi = f * Es + static_cast<size_t>(e) * 8 + n;
        if (FUSED) {
          const double rr = (A.a == 0.0 ? 0.0 : A.a * A.res_in[gi]) + A.dt * out[f][n];
          const double qn = q[f][n] + A.b * rr;
          if (A.res) A.res[gi] = rr;
          A.qout[gi] = qn;
          bad |= nonfinite(qn);
        } else {
          A.rhs[gi] = out[f][n];
          bad |= nonfinite(out[f][n]);
        }
      }
  }
  raise_flag(A.flags, bad, kFlagNonFinite);
}

template <int P>
dg_status launch_oi_p(const HexMesh& m, const OiArgs& A, bool fused, hipStream_t s) {
  using C = OiCfg<P>;
  static_assert(C::PER_EL * C::EPW * 8 <= 65536, "LDS budget");
  const int64_t blocks = (m.E + C::EPW - 1) / C::EPW;
  if (fused)
    hipLaunchKernelGGL((hex_oi_kernel<P, true>), dim3(static_cast<unsigned>(blocks)), dim3(64), 0, s, A);
  else
    hipLaunchKernelGGL((hex_oi_kernel<P, false>), dim3(static_cast<unsigned>(blocks)), dim3(64), 0, s, A);
  const hipError_t e = hipGetLastError();
  return e == hipSuccess ? DG_OK : hip_fail(e, "hex overintegrated rhs launch");
}

}  // namespace

int hex_oi_points(int p) { return oi_nq(p); }

dg_status launch_rhs_hex_oi(const HexMesh& m, double gamma, const double* q, double* rhs, const double* res_in,
                            double* res, double* q_out, double a, double b, double dt, bool fused, hipStream_t s) {
  OiArgs A;
  A.q = q;
  A.rhs = rhs;
  A.res_in = res_in;
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
    case 1: {
      const unsigned blocks = static_cast<unsigned>((m.E + 255) / 256);
      if (fused)
        hipLaunchKernelGGL((hex_oi_p1_kernel<true>), dim3(blocks), dim3(256), 0, s, A);
      else
        hipLaunchKernelGGL((hex_oi_p1_kernel<false>), dim3(blocks), dim3(256), 0, s, A);
      const hipError_t e = hipGetLastError();
      return e == hipSuccess ? DG_OK : hip_fail(e, "hex overintegrated rhs launch");
    }
    case 2: return launch_oi_p<2>(m, A, fused, s);
    case 3: return launch_oi_p<3>(m, A, fused, s);
    case 4: return launch_oi_p<4>(m, A, fused, s);
    default: return fail(DG_ERR_ARG, "hex overintegrated rhs: unsupported order");
  }
}

}  // namespace dg
