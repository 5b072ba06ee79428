// Strong-form nodal DG right-hand side of the Euler equations on
// tensor-product hexahedra of a periodic rectilinear grid, FP64, gfx950;
// optionally plus the divergence of artificial-viscosity fluxes G (BR1
// central flux: the volume term takes F - G, the face jump adds
// n_d ((G+ + G-)/2 - G-)).
//
// The element is an axis-aligned box, so the volume term is three sums of
// one-dimensional derivatives (sum factorisation: (p + 1) products per node
// and direction instead of (p + 1)^3) and the lift of a face acts along the
// lines normal to it:
//   rhs[a,b,c] = - sum_d (2 / h_d) sum_m D1[i_d, m] F_d(line of d through the node, node m)
//                + sum_d (2 / h_d) (lL[i_d] Delta_{d-} + lR[i_d] Delta_{d+})(the node's face position),
//   Delta = 1/2 n.(F(q-) - F(q+)) - 1/2 max(|u_d-| + c-, |u_d+| + c+) (q- - q+).
// The work is bound by HBM (about 4.5 flop per byte at p = 4), and the 1-D
// operator is at most 5 x 5: matrix cores would multiply zero padding (a
// 16-row block holds 5 rows) for no gain in FP64, whose vector rate equals
// its matrix rate on this chip, so the contractions run as vector FMAs fed
// from LDS.
//
// A 256-thread block owns EPB = 256 / (p + 1)^3 elements (32, 9, 4, 2 for
// p = 1..4), one thread per node.  Phases: (A) every global read is issued
// first: the thread's own node (coalesced: the block's elements are
// contiguous in each field) and the neighbour traces of its face slots;
// (B) the Lax-Friedrichs jumps of the block's 6 (p + 1)^2 face nodes per
// element into LDS; (C) per field, the three fluxes of every node into LDS,
// then each node's three line derivatives and six lift terms, and (D) the
// field's coalesced store, or the fused Runge-Kutta stage update
// res <- a res + dt rhs, q_out <- q + b res.
#include "euler_point.hpp"
#include "hex.hpp"

namespace dg {
namespace {

template <int P>
struct HexCfg {
  static constexpr int N1 = P + 1;
  static constexpr int NP = N1 * N1 * N1;
  static constexpr int NFP = N1 * N1;
  static constexpr int EPB = 256 / NP;      // elements per block
  static constexpr int NT = EPB * NP;       // threads owning a node
  static constexpr int NS = EPB * 6 * NFP;  // face slots of the block
  static constexpr int KF = (NS + 255) / 256;
  static constexpr int NOP = N1 * N1 + 2 * N1;
};

struct HexArgs {
  const double* __restrict__ q;
  const double* __restrict__ G;   // artificial viscosity: viscous fluxes [3][5][E][Np], valid where eps > 0
  const double* __restrict__ eps; // artificial viscosity per element
  double* __restrict__ rhs;
  const double* res_in;  // may alias res or qout (entry-wise)
  double* res;           // null: the new residual is not stored
  double* qout;
  const double* __restrict__ ih;  // [nx | ny | nz] 2 / h
  const double* __restrict__ op;  // [D1 | lift]
  int nx, ny, nz;
  int E;
  double gamma, a, b, dt;
  unsigned* flags;
};

// node index of (a, b, c)
template <int N1>
__device__ inline int nidx(int a, int b, int c) { return a + N1 * (b + N1 * c); }

// flux component along direction d of the five conserved fields, with the
// velocity component u_d and the sound speed.  EXACT: correctly rounded
// division and square root (the artificial-viscosity form, whose limiter,
// viscosity ramp and wave-speed maximum amplify rounding across strong
// jumps); otherwise the hardware reciprocal and reciprocal root refined by
// two Newton steps each (within an ulp or two, at half the instructions).
template <bool EXACT>
__device__ inline void dir_flux(const double q[5], int d, double gamma, double F[5], double& ud, double& c) {
  const double ir = EXACT ? 1.0 / q[0] : recip(q[0]);
  const double u = q[1] * ir, v = q[2] * ir, w = q[3] * ir;
  const double p = (gamma - 1.0) * (q[4] - 0.5 * (q[1] * u + q[2] * v + q[3] * w));
  ud = d == 0 ? u : d == 1 ? v : w;
  F[0] = q[1 + d];
  F[1] = q[1] * ud;
  F[2] = q[2] * ud;
  F[3] = q[3] * ud;
  F[1 + d] += p;
  F[4] = (q[4] + p) * ud;
  const double c2 = gamma * p * ir;
  c = EXACT || !(c2 > 0.0) ? sqrt(c2) : sqrt_pos(c2);  // (c2 <= 0 or NaN: the IEEE root, 0 or NaN)
}

template <int P, bool FUSED, bool AV>
__global__ __launch_bounds__(256) __attribute__((amdgpu_waves_per_eu(P == 1 || (P == 4 && FUSED) || AV ? 3 : 4))) void hex_rhs_kernel(HexArgs A) {
  using C = HexCfg<P>;
  constexpr int N1 = C::N1, NP = C::NP, NFP = C::NFP, EPB = C::EPB;
  __shared__ double s_q[EPB][5][NP];
  __shared__ double s_F[3][EPB * NP];
  __shared__ double s_D[EPB][6][5][NFP];
  __shared__ double s_op[C::NOP];
  const int tid = threadIdx.x;
  const int E = A.E;                 // E Np < 2^31 (checked on the host)
  const int e0 = blockIdx.x * EPB;
  const int el = tid / NP, i = tid - (tid / NP) * NP;
  const bool own = tid < C::NT;
  const int elc = own ? el : 0, ic = own ? i : 0;
  const int e = e0 + elc < E ? e0 + elc : E - 1;
  const bool valid = own && e0 + el < E;
  const int idx = e * NP + ic;
  const size_t Es = static_cast<size_t>(E) * NP;

  // (A) every global read first: the operator, the own node, the
  // neighbour traces of this thread's face slots
  const double opv = A.op[tid < C::NOP ? tid : 0];
  double qv[5];
#pragma unroll
  for (int f = 0; f < 5; ++f) qv[f] = A.q[f * Es + idx];
  double qp[C::KF][5];
  double gp[AV ? C::KF : 1][5], gm[AV ? C::KF : 1][5];
  int ownn[C::KF];
#pragma unroll
  for (int u = 0; u < C::KF; ++u) {
    const int s = tid + 256 * u < C::NS ? tid + 256 * u : C::NS - 1;
    const int fl = s / (6 * NFP), rem = s - fl * (6 * NFP);
    const int face = rem / NFP, m = rem - face * NFP;
    const int d = face >> 1, side = face & 1;
    const int ef = e0 + fl < E ? e0 + fl : E - 1;
    // cell coordinate along d and the neighbour's element id (periodic)
    const int cx = ef % A.nx, cxy = ef / A.nx, cy = cxy % A.ny, cz = cxy / A.ny;
    const int cd = d == 0 ? cx : d == 1 ? cy : cz;
    const int nd = d == 0 ? A.nx : d == 1 ? A.ny : A.nz;
    const int stride = d == 0 ? 1 : d == 1 ? A.nx : A.nx * A.ny;
    const int en = side ? (cd == nd - 1 ? ef - (nd - 1) * stride : ef + stride)
                        : (cd == 0 ? ef + (nd - 1) * stride : ef - stride);
    const int uu = m % N1, vv = m / N1;
    const int fo = side ? P : 0, fn = side ? 0 : P;  // own / neighbour index along d
    ownn[u] = d == 0 ? nidx<N1>(fo, uu, vv) : d == 1 ? nidx<N1>(uu, fo, vv) : nidx<N1>(uu, vv, fo);
    const int nn = d == 0 ? nidx<N1>(fn, uu, vv) : d == 1 ? nidx<N1>(uu, fn, vv) : nidx<N1>(uu, vv, fn);
    const int gi = en * NP + nn;
#pragma unroll
    for (int f = 0; f < 5; ++f) qp[u][f] = A.q[f * Es + gi];
    if (AV) {
      // viscous flux of direction d at both sides of the face node (zero,
      // and not stored, in an inviscid element)
      const int go = ef * NP + ownn[u];
      const bool vp = A.eps[en] > 0.0, vm = A.eps[ef] > 0.0;
#pragma unroll
      for (int f = 0; f < 5; ++f) {
        gp[u][f] = vp ? A.G[(d * 5 + f) * Es + gi] : 0.0;
        gm[u][f] = vm ? A.G[(d * 5 + f) * Es + go] : 0.0;
      }
    }
  }
  if (tid < C::NOP) s_op[tid] = opv;
  if (own) {
#pragma unroll
    for (int f = 0; f < 5; ++f) s_q[el][f][i] = qv[f];
  }
  __syncthreads();

  // (B) Lax-Friedrichs jumps of the face slots
#pragma unroll
  for (int u = 0; u < C::KF; ++u) {
    const int s = tid + 256 * u;
    if (s < C::NS) {
      const int fl = s / (6 * NFP), rem = s - fl * (6 * NFP);
      const int face = rem / NFP, m = rem - face * NFP;
      const int d = face >> 1;
      const double sgn = (face & 1) ? 0.5 : -0.5;
      double qm[5];
#pragma unroll
      for (int f = 0; f < 5; ++f) qm[f] = s_q[fl][f][ownn[u]];
      double FM[5], FP[5], uM, cM, uP, cP;
      dir_flux<AV>(qm, d, A.gamma, FM, uM, cM);
      dir_flux<AV>(qp[u], d, A.gamma, FP, uP, cP);
      const double lam = fmax(fabs(uM) + cM, fabs(uP) + cP);
#pragma unroll
      for (int f = 0; f < 5; ++f) {
        double dj = sgn * (FM[f] - FP[f]) - 0.5 * lam * (qm[f] - qp[u][f]);
        if (AV) dj += sgn * (gp[u][f] - gm[u][f]);  // n_d ((G+ + G-)/2 - G-)
        s_D[fl][face][f][m] = dj;
      }
    }
  }

  // (C) per field: the own node's three fluxes into LDS, then its line
  // derivatives and the lift; (D) the field's store or stage update.  The
  // field loop stays rolled (unrolled, the compiler keeps every field's
  // addresses live and spills); per-field values are picked by selects, not
  // by indexing a register array (which would live in scratch memory).
  const double q0 = qv[0], q1 = qv[1], q2 = qv[2], q3 = qv[3], q4 = qv[4];
  double r0 = 0.0, r1 = 0.0, r2 = 0.0, r3 = 0.0, r4 = 0.0;
  if (FUSED && A.a != 0.0) {
    r0 = A.res_in[idx];
    r1 = A.res_in[Es + idx];
    r2 = A.res_in[2 * Es + idx];
    r3 = A.res_in[3 * Es + idx];
    r4 = A.res_in[4 * Es + idx];
  }
  const int cx = e % A.nx, cxy = e / A.nx;
  const double ihx = A.ih[cx], ihy = A.ih[A.nx + cxy % A.ny], ihz = A.ih[A.nx + A.ny + cxy / A.ny];
  const int a = ic % N1, bb = (ic / N1) % N1, c = ic / (N1 * N1);
  const double ir = AV ? 1.0 / q0 : recip(q0);
  const double vx = q1 * ir, vy = q2 * ir, vz = q3 * ir;
  const double pr = (A.gamma - 1.0) * (q4 - 0.5 * (q1 * vx + q2 * vy + q3 * vz));
  const int base = elc * NP;
  const double* D1 = s_op;
  const double* lift = s_op + N1 * N1;
  bool bad = false;
#pragma unroll 1
  for (int f = 0; f < 5; ++f) {
    const double qf = f == 0 ? q0 : f == 1 ? q1 : f == 2 ? q2 : f == 3 ? q3 : q4;
    __syncthreads();  // previous field's reads done (and, for f = 0, the jumps written)
    if (own) {
      // flux of field f along x, y, z: q_f u_d + p delta(f, 1 + d); energy (E + p) u_d
      const double qe = f == 4 ? qf + pr : qf;
      double fx = qe * vx + (f == 1 ? pr : 0.0);
      double fy = qe * vy + (f == 2 ? pr : 0.0);
      double fz = qe * vz + (f == 3 ? pr : 0.0);
      if (AV && A.eps[e] > 0.0) {  // total flux F - G (the viscous term enters as + div G)
        fx -= A.G[(0 * 5 + f) * Es + idx];
        fy -= A.G[(1 * 5 + f) * Es + idx];
        fz -= A.G[(2 * 5 + f) * Es + idx];
      }
      s_F[0][tid] = fx;
      s_F[1][tid] = fy;
      s_F[2][tid] = fz;
    }
    __syncthreads();
    double dx = 0.0, dy = 0.0, dz = 0.0;
#pragma unroll
    for (int m = 0; m < N1; ++m) {
      dx = fma(D1[a * N1 + m], s_F[0][base + nidx<N1>(m, bb, c)], dx);
      dy = fma(D1[bb * N1 + m], s_F[1][base + nidx<N1>(a, m, c)], dy);
      dz = fma(D1[c * N1 + m], s_F[2][base + nidx<N1>(a, bb, m)], dz);
    }
    const double lx = lift[a * 2] * s_D[elc][0][f][bb + N1 * c] + lift[a * 2 + 1] * s_D[elc][1][f][bb + N1 * c];
    const double ly = lift[bb * 2] * s_D[elc][2][f][a + N1 * c] + lift[bb * 2 + 1] * s_D[elc][3][f][a + N1 * c];
    const double lz = lift[c * 2] * s_D[elc][4][f][a + N1 * bb] + lift[c * 2 + 1] * s_D[elc][5][f][a + N1 * bb];
    const double out = ihx * (lx - dx) + ihy * (ly - dy) + ihz * (lz - dz);
    if (valid) {
      if (FUSED) {
        const double ro = f == 0 ? r0 : f == 1 ? r1 : f == 2 ? r2 : f == 3 ? r3 : r4;
        const double r = (A.a == 0.0 ? 0.0 : A.a * ro) + A.dt * out;
        const double qn = qf + A.b * r;
        if (A.res) A.res[f * Es + idx] = r;
        A.qout[f * Es + idx] = qn;
        bad |= nonfinite(qn);
      } else {
        A.rhs[f * Es + idx] = out;
        bad |= nonfinite(out);
      }
    }
  }
  raise_flag(A.flags, bad, kFlagNonFinite);
}

// Tiled form for p = 1, with or without artificial viscosity: a 256-thread
// block owns a box of TX x TY x TZ cells, one thread per node, so most face neighbours are in
// the block.  Each face node of the tile (every cell face in the box,
// including the planes on its boundary) is evaluated once for both sides:
// with L, R the cells before and after it along d,
//   A = 1/2 (F_d(q_L) - F_d(q_R)),  B = 1/2 max(|u_L| + c_L, |u_R| + c_R) (q_L - q_R),
// L's jump on its +d face is A - B and R's on its -d face is A + B (the
// form above with the signs of n_d worked out; with viscosity both add the
// central viscous term (G_d(R) - G_d(L)) / 2).  A side inside the tile
// (and inside the grid) comes from the tile's LDS copy; the others, on the
// tile's boundary planes or past a ragged grid end, are read from memory
// with the periodic wrap.  Own state and output move in runs of TX cells
// (TX Np consecutive doubles per field).
template <int P, int TX, int TY, int TZ, bool FUSED, bool AV>
__global__ __launch_bounds__(256) __attribute__((amdgpu_waves_per_eu(4))) void hex_rhs_tile_kernel(HexArgs A) {
  static_assert(P == 1, "line partners by lane exchange: a cell's 8 nodes are 8 consecutive lanes");
  using C = HexTileCfg<P, TX, TY, TZ>;
  constexpr int N1 = C::N1, NP = C::NP, NFP = C::NFP, NC = C::NC;
  __shared__ double s_q[NC][5][NP];
  __shared__ double s_D[NC][6][5][NFP];
  const int tid = threadIdx.x;
  const int nx = A.nx, ny = A.ny, nz = A.nz;
  const int ntx = (nx + TX - 1) / TX, nty = (ny + TY - 1) / TY;
  const int X0 = (blockIdx.x % ntx) * TX, Y0 = ((blockIdx.x / ntx) % nty) * TY, Z0 = (blockIdx.x / (ntx * nty)) * TZ;
  const size_t Es = static_cast<size_t>(A.E) * NP;  // E Np < 2^31 (checked on the host)

  // this thread's node: cell (lx, ly, lz) of the tile, node i
  const bool own = tid < C::NT;
  const int cl = own ? tid / NP : 0, ic = own ? tid - (tid / NP) * NP : 0;
  const int lx = cl % TX, ly = (cl / TX) % TY, lz = cl / (TX * TY);
  const bool valid = own && X0 + lx < nx && Y0 + ly < ny && Z0 + lz < nz;
  const int gx = valid ? X0 + lx : 0, gy = valid ? Y0 + ly : 0, gz = valid ? Z0 + lz : 0;
  const int e = gx + nx * (gy + ny * gz);
  const int idx = e * NP + ic;

  // (A) every global read first: the operator, the own node, and the sides
  // of this thread's face nodes that lie outside the tile
  double D1[N1 * N1], lift[2 * N1];  // the 1-D tables (wave-uniform)
#pragma unroll
  for (int j = 0; j < N1 * N1; ++j) D1[j] = A.op[j];
#pragma unroll
  for (int j = 0; j < 2 * N1; ++j) lift[j] = A.op[N1 * N1 + j];
  double qv[5];
#pragma unroll
  for (int f = 0; f < 5; ++f) qv[f] = A.q[f * Es + idx];
  // face node u of this thread: direction, the two cells (tile-local
  // coordinates, -1 / T for outside), node indices, which sides are in the
  // tile, and the out-of-tile sides' states
  int fdir[C::KF], fcell[C::KF][2], fm[C::KF];
  bool fin[C::KF][2], fuse[C::KF];
  double gq[C::KF][2][5];
  // artificial viscosity: whether each side's element is viscous, and the
  // side's node (the G values are loaded after the barrier, rarely)
  bool fvis[AV ? C::KF : 1][2];
  int fgi[AV ? C::KF : 1][2];
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
#pragma unroll
      for (int f = 0; f < 5; ++f) gq[u][side][f] = fn.in[side] ? 0.0 : A.q[f * Es + fn.gi[side]];
      if (AV) {
        fvis[u][side] = A.eps[fn.ge[side]] > 0.0;  // (element 0 where no valid cell touches the face: unused)
        fgi[u][side] = fn.gi[side];
      }
    }
    fuse[u] = fn.in[0] || fn.in[1];
  }
  if (own) {
#pragma unroll
    for (int f = 0; f < 5; ++f) s_q[cl][f][ic] = qv[f];
  }
  __syncthreads();

  // (B) jumps of the tile's face nodes, both sides at once
#pragma unroll
  for (int u = 0; u < C::KF; ++u) {
    if (!fuse[u]) continue;
    const int d = fdir[u], m = fm[u];
    const int uu = m % N1, vv = m / N1;
    double qs[2][5];
#pragma unroll
    for (int side = 0; side < 2; ++side) {
      const int pd = side ? 0 : P;
      const int nn = d == 0 ? nidx<N1>(pd, uu, vv) : d == 1 ? nidx<N1>(uu, pd, vv) : nidx<N1>(uu, vv, pd);
#pragma unroll
      for (int f = 0; f < 5; ++f) qs[side][f] = fin[u][side] ? s_q[fcell[u][side]][f][nn] : gq[u][side][f];
    }
    double FL[5], FR[5], uL, cL, uR, cR;
    dir_flux<false>(qs[0], d, A.gamma, FL, uL, cL);
    dir_flux<false>(qs[1], d, A.gamma, FR, uR, cR);
    const double lam = fmax(fabs(uL) + cL, fabs(uR) + cR);
    // with viscosity both sides add n_d ((G+ + G-)/2 - G-) = (G_R - G_L) / 2,
    // G_d of a side being zero (and not stored) in an inviscid element
    double gv[5] = {0.0, 0.0, 0.0, 0.0, 0.0};
    if (AV && (fvis[u][0] || fvis[u][1])) {
#pragma unroll
      for (int f = 0; f < 5; ++f) {
        const double gL = fvis[u][0] ? A.G[(d * 5 + f) * Es + fgi[u][0]] : 0.0;
        const double gR = fvis[u][1] ? A.G[(d * 5 + f) * Es + fgi[u][1]] : 0.0;
        gv[f] = 0.5 * gR - 0.5 * gL;
      }
    }
#pragma unroll
    for (int f = 0; f < 5; ++f) {
      const double a = 0.5 * (FL[f] - FR[f]);
      const double b = 0.5 * lam * (qs[0][f] - qs[1][f]);
      const double v = gv[f];
      if (fin[u][0]) s_D[fcell[u][0]][2 * d + 1][f][m] = AV ? (a - b) + v : a - b;
      if (fin[u][1]) s_D[fcell[u][1]][2 * d][f][m] = AV ? (a + b) + v : a + b;
    }
  }

  __syncthreads();  // the jumps are written

  // (C) per field: the own node's three fluxes; the line partner's (node
  // i ^ 1, i ^ 2, i ^ 4 along x, y, z: lane tid ^ 1, 2, 4 of the same cell)
  // by lane exchange; the line derivatives and the lift; (D) the field's
  // store or stage update (as in hex_rhs_kernel)
  const double q0 = qv[0], q1 = qv[1], q2 = qv[2], q3 = qv[3], q4 = qv[4];
  double rv[5] = {0.0, 0.0, 0.0, 0.0, 0.0};
  if (FUSED && A.a != 0.0) {
#pragma unroll
    for (int f = 0; f < 5; ++f) rv[f] = A.res_in[f * Es + idx];
  }
  const double ihx = A.ih[gx], ihy = A.ih[nx + gy], ihz = A.ih[nx + ny + gz];
  const int a = ic & 1, bb = (ic >> 1) & 1, c = ic >> 2;
  // this node's rows of D1 and lift along x, y, z (selected, not indexed:
  // an array indexed by a lane value would live in scratch memory)
  const double dxr0 = a ? D1[2] : D1[0], dxr1 = a ? D1[3] : D1[1];
  const double dyr0 = bb ? D1[2] : D1[0], dyr1 = bb ? D1[3] : D1[1];
  const double dzr0 = c ? D1[2] : D1[0], dzr1 = c ? D1[3] : D1[1];
  const double lxr0 = a ? lift[2] : lift[0], lxr1 = a ? lift[3] : lift[1];
  const double lyr0 = bb ? lift[2] : lift[0], lyr1 = bb ? lift[3] : lift[1];
  const double lzr0 = c ? lift[2] : lift[0], lzr1 = c ? lift[3] : lift[1];
  const double ir = recip(q0);
  const double vx = q1 * ir, vy = q2 * ir, vz = q3 * ir;
  const double pr = (A.gamma - 1.0) * (q4 - 0.5 * (q1 * vx + q2 * vy + q3 * vz));
  bool bad = false;
  const bool visc_own = AV && valid && A.eps[e] > 0.0;
#pragma unroll
  for (int f = 0; f < 5; ++f) {
    const double qf = qv[f];
    const double qe = f == 4 ? qf + pr : qf;
    double fx = qe * vx + (f == 1 ? pr : 0.0);
    double fy = qe * vy + (f == 2 ? pr : 0.0);
    double fz = qe * vz + (f == 3 ? pr : 0.0);
    if (AV && visc_own) {  // total flux F - G (the viscous term enters as + div G)
      fx -= A.G[(0 * 5 + f) * Es + idx];
      fy -= A.G[(1 * 5 + f) * Es + idx];
      fz -= A.G[(2 * 5 + f) * Es + idx];
    }
    const double px = __shfl_xor(fx, 1, 64), py = __shfl_xor(fy, 2, 64), pz = __shfl_xor(fz, 4, 64);
    // F at line positions 0 and 1 of this node's x, y, z lines
    const double x0 = a ? px : fx, x1 = a ? fx : px;
    const double y0 = bb ? py : fy, y1 = bb ? fy : py;
    const double z0 = c ? pz : fz, z1 = c ? fz : pz;
    double dx = 0.0, dy = 0.0, dz = 0.0;
    dx = fma(dxr0, x0, dx);
    dy = fma(dyr0, y0, dy);
    dz = fma(dzr0, z0, dz);
    dx = fma(dxr1, x1, dx);
    dy = fma(dyr1, y1, dy);
    dz = fma(dzr1, z1, dz);
    const double lx2 = lxr0 * s_D[cl][0][f][bb + N1 * c] + lxr1 * s_D[cl][1][f][bb + N1 * c];
    const double ly2 = lyr0 * s_D[cl][2][f][a + N1 * c] + lyr1 * s_D[cl][3][f][a + N1 * c];
    const double lz2 = lzr0 * s_D[cl][4][f][a + N1 * bb] + lzr1 * s_D[cl][5][f][a + N1 * bb];
    const double out = ihx * (lx2 - dx) + ihy * (ly2 - dy) + ihz * (lz2 - dz);
    if (valid) {
      if (FUSED) {
        const double rn = (A.a == 0.0 ? 0.0 : A.a * rv[f]) + A.dt * out;
        const double qn = qf + A.b * rn;
        if (A.res) A.res[f * Es + idx] = rn;
        A.qout[f * Es + idx] = qn;
        bad |= nonfinite(qn);
      } else {
        A.rhs[f * Es + idx] = out;
        bad |= nonfinite(out);
      }
    }
  }
  raise_flag(A.flags, bad, kFlagNonFinite);
}

template <int P>
dg_status launch_p(const HexMesh& m, const HexArgs& A, bool fused, hipStream_t s) {
  using C = HexCfg<P>;
  const int64_t blocks = (m.E + C::EPB - 1) / C::EPB;
  if (P == 1) {
    const int64_t tiles = static_cast<int64_t>((m.nx + kTileX1 - 1) / kTileX1) * ((m.ny + kTileY1 - 1) / kTileY1) *
                          ((m.nz + kTileZ1 - 1) / kTileZ1);
    const dim3 grid(static_cast<unsigned>(tiles));
    if (A.G) {
      if (fused)
        hipLaunchKernelGGL((hex_rhs_tile_kernel<1, kTileX1, kTileY1, kTileZ1, true, true>), grid, dim3(256), 0, s, A);
      else
        hipLaunchKernelGGL((hex_rhs_tile_kernel<1, kTileX1, kTileY1, kTileZ1, false, true>), grid, dim3(256), 0, s, A);
    } else if (fused) {
      hipLaunchKernelGGL((hex_rhs_tile_kernel<1, kTileX1, kTileY1, kTileZ1, true, false>), grid, dim3(256), 0, s, A);
    } else {
      hipLaunchKernelGGL((hex_rhs_tile_kernel<1, kTileX1, kTileY1, kTileZ1, false, false>), grid, dim3(256), 0, s, A);
    }
  } else if (A.G) {
    if (fused)
      hipLaunchKernelGGL((hex_rhs_kernel<P, true, true>), dim3(static_cast<unsigned>(blocks)), dim3(256), 0, s, A);
    else
      hipLaunchKernelGGL((hex_rhs_kernel<P, false, true>), dim3(static_cast<unsigned>(blocks)), dim3(256), 0, s, A);
  } else if (fused) {
    hipLaunchKernelGGL((hex_rhs_kernel<P, true, false>), dim3(static_cast<unsigned>(blocks)), dim3(256), 0, s, A);
  } else {
    hipLaunchKernelGGL((hex_rhs_kernel<P, false, false>), dim3(static_cast<unsigned>(blocks)), dim3(256), 0, s, A);
  }
  const hipError_t e = hipGetLastError();
  return e == hipSuccess ? DG_OK : hip_fail(e, "hex rhs launch");
}

}  // namespace

dg_status launch_rhs_hex(const HexMesh& m, double gamma, const double* q, double* rhs, const double* res_in,
                         double* res, double* q_out, double a, double b, double dt, bool fused, hipStream_t s) {
  return launch_rhs_hex_av(m, gamma, q, nullptr, nullptr, rhs, res_in, res, q_out, a, b, dt, fused, s);
}

dg_status launch_rhs_hex_av(const HexMesh& m, double gamma, const double* q, const double* G, const double* eps,
                            double* rhs, const double* res_in, double* res, double* q_out, double a, double b,
                            double dt, bool fused, hipStream_t s) {
  HexArgs A;
  A.q = q;
  A.G = G;
  A.eps = eps;
  A.rhs = rhs;
  A.res_in = res_in;
  A.res = res;
  A.qout = q_out;
  A.ih = m.d_ih;
  A.op = m.d_op;
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
    case 1: return launch_p<1>(m, A, fused, s);
    case 2: return launch_p<2>(m, A, fused, s);
    case 3: return launch_p<3>(m, A, fused, s);
    case 4: return launch_p<4>(m, A, fused, s);
    default: return fail(DG_ERR_ARG, "hex rhs: unsupported order");
  }
}

}  // namespace dg
