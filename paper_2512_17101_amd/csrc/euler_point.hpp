// Pointwise FP64 pieces of the Euler right-hand side shared by the element
// kernels of every contraction precision.
#pragma once
#include <hip/hip_runtime.h>

#include <cstdint>

#include "internal.hpp"

namespace dg {

// Reciprocal and square root from the hardware approximations, refined by
// Newton steps (each squares the relative error; two reach the last bit of a
// double from the hardware's initial accuracy).
__device__ inline double recip(double x) {
  double r = __builtin_amdgcn_rcp(x);
  double e = fma(-x, r, 1.0);
  r = fma(r, e, r);
  e = fma(-x, r, 1.0);
  return fma(r, e, r);
}
__device__ inline double sqrt_pos(double a) {  // a > 0
  double y = __builtin_amdgcn_rsq(a);
  y = y * fma(-0.5 * a * y, y, 1.5);
  y = y * fma(-0.5 * a * y, y, 1.5);
  return a * y;
}

// Contravariant fluxes G_a = sum_d (da/dx_d) F_d(q) of one node for
// a = r, s, t; gm = (grad r, grad s, grad t).  With u = m / rho,
// p = (gamma - 1)(E - m.u / 2) and U_a = grad a . u:
//   G_a = (rho U_a, m U_a + p grad a, (E + p) U_a).
__device__ inline void contravariant_flux(const double qq[5], const double gm[9], double gm1, double G[3][5]) {
  const double ir = recip(qq[0]);
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
}

// Face normal scaled by Fscale = sJ / J, from the metric: f0 {t=-1}: -grad t,
// f1 {s=-1}: -grad s, f2 {r+s+t=-1}: grad r + grad s + grad t, f3 {r=-1}: -grad r,
// i.e. N = c_r grad r + c_s grad s + c_t grad t with (c_r, c_s, c_t) =
// (0,0,-1), (0,-1,0), (1,1,1), (-1,0,0).  The coefficients are formed with
// integer arithmetic on the face index, not a branch chain: hipcc for gfx950
// was measured to return face 1's normal for face 3 when the chain was
// selected by a face index that differs between lanes.  Multiplying by 0 and
// +-1 is exact, so the result is the same vector the chain defines.
__device__ inline void scaled_normal(int face, const double gm[9], double& Nx, double& Ny, double& Nz) {
  const int hi = face >> 1, lo = face & 1;
  const double cr = static_cast<double>(hi * (1 - 2 * lo));             // 0, 0, 1, -1
  const double cs = static_cast<double>((lo ^ hi) * (2 * hi - 1));       // 0, -1, 1, 0
  const double ct = static_cast<double>((1 - lo) * (2 * hi - 1));        // -1, 0, 1, 0
  Nx = cr * gm[0] + cs * gm[3] + ct * gm[6];
  Ny = cr * gm[1] + cs * gm[4] + ct * gm[7];
  Nz = cr * gm[2] + cs * gm[5] + ct * gm[8];
}

// The scaled normal of the face of face-node step s, where lane group g
// takes face node 4 s + g of its element (NFP face nodes per face).  Where
// the four groups sit on one face, which is known once the step loop is
// unrolled, the normal is a metric row negated, or the sum of the three:
// the same values as scaled_normal (up to the sign of a zero component)
// without its multiplications by 0 and 1, which IEEE rules keep in the
// code.  Steps that straddle two faces take scaled_normal.
template <int NFP>
__device__ inline void step_normal(int s, int face, const double gm[9], double& Nx, double& Ny, double& Nz) {
  const int f0 = (4 * s) / NFP;
  if (f0 == (4 * s + 3) / NFP) {
    switch (f0) {
      case 0: Nx = -gm[6]; Ny = -gm[7]; Nz = -gm[8]; break;
      case 1: Nx = -gm[3]; Ny = -gm[4]; Nz = -gm[5]; break;
      case 2:
        Nx = (gm[0] + gm[3]) + gm[6];
        Ny = (gm[1] + gm[4]) + gm[7];
        Nz = (gm[2] + gm[5]) + gm[8];
        break;
      default: Nx = -gm[0]; Ny = -gm[1]; Nz = -gm[2]; break;
    }
  } else {
    scaled_normal(face, gm, Nx, Ny, Nz);
  }
}

// Twice the scaled local Lax-Friedrichs jump at a face node, N = Fscale n,
// U_n = N . u:
//   2 D = N.F(q-) - N.F(q+) - max(|U_n-| + c- |N|, |U_n+| + c+ |N|) (q- - q+).
// The factor 1/2 is folded into the LIFT columns of the operator tables (a
// power-of-two scaling, exact in every precision the tables are kept in, as
// is the doubled jump's rounding to FP32 or BF16), so the contraction gives
// the same products as with D and the unscaled LIFT.  The sound speed and
// |N| enter through one root per side, c |N| = sqrt(gamma p / rho |N|^2).
__device__ inline void lf_jump(const double qm[5], const double qp[5], double Nx, double Ny, double Nz,
                               double gamma, double D[5]) {
  const double gm1 = gamma - 1.0;
  const double N2 = Nx * Nx + Ny * Ny + Nz * Nz;
  const double irm = recip(qm[0]), irp = recip(qp[0]);
  const double um = qm[1] * irm, vm = qm[2] * irm, wm = qm[3] * irm;
  const double up = qp[1] * irp, vp = qp[2] * irp, wp = qp[3] * irp;
  const double pm = gm1 * (qm[4] - 0.5 * (qm[1] * um + qm[2] * vm + qm[3] * wm));
  const double pp = gm1 * (qp[4] - 0.5 * (qp[1] * up + qp[2] * vp + qp[3] * wp));
  const double Unm = Nx * um + Ny * vm + Nz * wm;
  const double Unp = Nx * up + Ny * vp + Nz * wp;
  const double cFm = sqrt_pos(gamma * pm * irm * N2), cFp = sqrt_pos(gamma * pp * irp * N2);
  const double lamFs = fmax(fabs(Unm) + cFm, fabs(Unp) + cFp);
  D[0] = (qm[0] * Unm - qp[0] * Unp) - lamFs * (qm[0] - qp[0]);
  D[1] = (qm[1] * Unm + pm * Nx - qp[1] * Unp - pp * Nx) - lamFs * (qm[1] - qp[1]);
  D[2] = (qm[2] * Unm + pm * Ny - qp[2] * Unp - pp * Ny) - lamFs * (qm[2] - qp[2]);
  D[3] = (qm[3] * Unm + pm * Nz - qp[3] * Unp - pp * Nz) - lamFs * (qm[3] - qp[3]);
  D[4] = ((qm[4] + pm) * Unm - (qp[4] + pp) * Unp) - lamFs * (qm[4] - qp[4]);
}

// Block renumbering for the 8 XCDs, which take workgroups round-robin and
// each have their own L2: with k > 1, XCD x runs the blocks x k .. x k + k - 1
// of each run of 8 k blocks, so that neighbouring tiles (which read each
// other's traces) share an L2 while all XCDs still sweep the mesh together.
// Blocks past the last whole run keep the plain order; a bijection of
// [0, nblocks) for every k >= 1.
__device__ inline int xcd_run_block(int blk, int nblocks, int k) {
  if (k <= 1) return blk;  // also guards the divisions below
  const int full = nblocks / (8 * k) * (8 * k);
  if (blk >= full) return blk;
  const int i = blk >> 3;
  return ((i / k) * 8 + (blk & 7)) * k + i % k;
}

// Copies the face tables of order P's element (neighbour volume node of each
// face node per face and neighbour code, nbtab [4][24][Nfp] bytes; face-node
// mask fmask [4 Nfp]) into LDS, thread t of NT: every load is issued before
// the first write, so a block starts after one memory latency instead of one
// per loop trip.  Indices are clamped, the writes guarded; the caller
// synchronises the block afterwards.
template <int NFP, int NT>
__device__ inline void stage_face_tables(uint8_t* s_nb, int* s_fm, const uint8_t* __restrict__ nbtab,
                                         const int* __restrict__ fmask, int t) {
  constexpr int NBW = 4 * 24 * NFP / 4;  // 32-bit words (96 Nfp bytes)
  constexpr int KW = (NBW + NT - 1) / NT;
  const uint32_t* nb32 = reinterpret_cast<const uint32_t*>(nbtab);
  uint32_t w[KW];
#pragma unroll
  for (int k = 0; k < KW; ++k) {
    const int i = t + k * NT;
    w[k] = nb32[i < NBW ? i : NBW - 1];
  }
  const int fmv = fmask[t < 4 * NFP ? t : 4 * NFP - 1];
  uint32_t* s_nb32 = reinterpret_cast<uint32_t*>(s_nb);
#pragma unroll
  for (int k = 0; k < KW; ++k) {
    const int i = t + k * NT;
    if (i < NBW) s_nb32[i] = w[k];
  }
  if (t < 4 * NFP) s_fm[t] = fmv;
}

// Values per lane in one round of a tile's loads (at most 25 doubles per
// lane in flight: one round up to p = 3, three at p = 4).
template <int TQ>
constexpr int tile_round_fields() {
  constexpr int KN = (TQ + 63) / 64;
  return 25 / KN >= 5 ? 5 : (25 / KN >= 1 ? 25 / KN : 1);
}

// Copies one tile's state (field f's nval valid values at q + f Es + base)
// into this wave's LDS buffer (field f at sq[f TQ]), lane l taking entries
// 64 k + l (coalesced).  The loads are unconditional at indices clamped into
// the tile (nval >= 1), so a round's loads are all in flight together before
// its guarded LDS writes; a guarded load would be waited for one by one.
template <int TQ>
__device__ inline void stage_tile(double* sq, const double* __restrict__ q, int64_t Es, int64_t base, int nval,
                                  int lane) {
  constexpr int KN = (TQ + 63) / 64;
  constexpr int FG = tile_round_fields<TQ>();
#pragma unroll
  for (int f0 = 0; f0 < 5; f0 += FG) {
    double v[FG][KN];
#pragma unroll
    for (int ff = 0; ff < FG; ++ff)
#pragma unroll
      for (int k = 0; k < KN; ++k) {
        const int i = 64 * k + lane;
        v[ff][k] = f0 + ff < 5 ? q[(f0 + ff) * Es + base + (i < nval ? i : nval - 1)] : 0.0;
      }
#pragma unroll
    for (int ff = 0; ff < FG; ++ff)
#pragma unroll
      for (int k = 0; k < KN; ++k) {
        const int i = 64 * k + lane;
        if (f0 + ff < 5 && i < nval) sq[(f0 + ff) * TQ + i] = v[ff][k];
      }
  }
  __builtin_amdgcn_wave_barrier();
}

// The same copy with the LDS DMA path (global_load_lds_dwordx4) for the whole
// 128-double groups of each field: lane l of group k moves entries
// 128 k + 2 l and 128 k + 2 l + 1 straight into LDS, with no registers and no
// LDS write instructions; the rest of the field (fewer than 128 entries) goes
// through registers.  No DMA load sits under a lane-dependent condition:
// with one there, the compiler merged DMA loads of different groups across
// the branch and derived the LDS base (M0) from the first active lane's
// value, which sent one group's data to another group's slots.  Needs TQ and
// nval even, every field block 16-byte aligned in memory (q 16-byte aligned;
// Es and base even) and, as measured, every LDS destination base
// (sq + f TQ + 128 k) a multiple of 512 bytes: Np a multiple of 4.  Entries
// at or past nval re-read the last valid ones (their LDS slots are never
// read).
template <int TQ>
__device__ inline void stage_tile_dma(double* sq, const double* __restrict__ q, int64_t Es, int64_t base, int nval,
                                      int lane) {
  static_assert(TQ % 64 == 0, "512-byte-aligned field blocks");
  constexpr int KG = TQ / 128;        // whole 128-double groups per field
  constexpr int R = TQ - 128 * KG;    // entries left to the register path
  constexpr int KR = (R + 63) / 64;
  const int last = nval / 2 - 1;      // last valid 16-byte chunk
  double v[5][KR > 0 ? KR : 1];
#pragma unroll
  for (int f = 0; f < 5; ++f) {
#pragma unroll
    for (int k = 0; k < KG; ++k) {
      const int c = 64 * k + lane;
      const double* src = q + f * Es + base + 2 * (c <= last ? c : last);
      __builtin_amdgcn_global_load_lds(src, (__attribute__((address_space(3))) void*)(sq + f * TQ + 128 * k), 16, 0,
                                       0);
    }
#pragma unroll
    for (int k = 0; k < KR; ++k) {
      const int i = 128 * KG + 64 * k + lane;
      v[f][k] = q[f * Es + base + (i < nval ? i : nval - 1)];
    }
  }
#pragma unroll
  for (int f = 0; f < 5; ++f)
#pragma unroll
    for (int k = 0; k < KR; ++k) {
      const int i = 128 * KG + 64 * k + lane;
      if (i < R + 128 * KG && i < nval) sq[f * TQ + i] = v[f][k];
    }
  __builtin_amdgcn_s_waitcnt(0x3f70);  // vmcnt(0): every group is in LDS
  __builtin_amdgcn_wave_barrier();
}

// One entry of the fused 2N-storage Runge-Kutta stage
//   res <- a res + dt rhs;  q_out <- q + b res
// from values of res and q loaded beforehand (res_old is not used when
// a == 0: the first stage's residual buffer may hold anything).  The new
// residual goes to res (skipped when res is null: the last stage's is not
// needed); res and qout may be the buffer the old residual came from,
// since every entry is read before it is written by the same thread.
__device__ inline double stage_store(int64_t idx, double val, double res_old, double q_old, double* res, double* qout,
                                     double a, double b, double dt) {
  const double r = (a == 0.0 ? 0.0 : a * res_old) + dt * val;
  const double qn = q_old + b * r;
  if (res) res[idx] = r;
  qout[idx] = qn;
  return qn;
}

// Writes one tile's outputs staged in this wave's LDS buffer (field f's
// nval valid values at sq[f TQ ..], element-major as in memory from entry
// base = e0 Np on) to memory, lane l taking entries 64 k + l of each field,
// so every field leaves with coalesced stores.  In the fused stage every res
// and q value of a round of fields is loaded before the round's first
// store: the compiler cannot rule out that a store to res or qout aliases a
// later load, so entry-by-entry code would wait out one memory latency per
// entry.  A non-finite value among the stored ones (the right-hand side, or
// the new state of a fused stage) raises the device's non-finite flag.
template <bool FUSED, int TQ>
__device__ inline void store_tile(const double* sq, int nval, int64_t base, int64_t Es, int lane,
                                  double* __restrict__ rhs, const double* res_in, double* res, double* qout,
                                  const double* __restrict__ q, double a, double b, double dt, unsigned* flags) {
  constexpr int KN = (TQ + 63) / 64;
  constexpr int FG = tile_round_fields<TQ>();
  // an opaque copy of the tile offset: otherwise the compiler shares these
  // addresses with the staging loads at the kernel start and keeps them
  // live (spilled) across the whole tile
  {
    int lo = static_cast<int>(base), hi = static_cast<int>(base >> 32);
    asm volatile("" : "+v"(lo), "+v"(hi));
    base = (static_cast<int64_t>(hi) << 32) | static_cast<uint32_t>(lo);
  }
  bool bad = false;
  if constexpr (!FUSED) {
#pragma unroll
    for (int f = 0; f < 5; ++f)
#pragma unroll
      for (int k = 0; k < KN; ++k) {
        const int i = 64 * k + lane;
        if (i < nval) {
          const double v = sq[f * TQ + i];
          bad |= nonfinite(v);
          rhs[f * Es + base + i] = v;
        }
      }
  } else {
#pragma unroll
    for (int f0 = 0; f0 < 5; f0 += FG) {
      double rv[FG][KN], qv[FG][KN];
#pragma unroll
      for (int ff = 0; ff < FG; ++ff)
#pragma unroll
        for (int k = 0; k < KN; ++k) {
          const int i = 64 * k + lane;
          const bool ok = f0 + ff < 5;  // known at compile time
          const int64_t idx = (f0 + ff) * Es + base + (i < nval ? i : nval - 1);  // clamped: unconditional loads
          rv[ff][k] = ok && a != 0.0 ? res_in[idx] : 0.0;
          qv[ff][k] = ok ? q[idx] : 0.0;
        }
#pragma unroll
      for (int ff = 0; ff < FG; ++ff)
#pragma unroll
        for (int k = 0; k < KN; ++k) {
          const int i = 64 * k + lane;
          if (f0 + ff < 5 && i < nval)
            bad |= nonfinite(stage_store((f0 + ff) * Es + base + i, sq[(f0 + ff) * TQ + i], rv[ff][k], qv[ff][k], res,
                                         qout, a, b, dt));
        }
    }
  }
  raise_flag(flags, bad, kFlagNonFinite);
}

// This lane's entries (64 k + lane, k < ceil(TQ / 64)) of each field of the
// state tile staged in LDS, read back into registers before the tile buffer is
// reused for the outputs: the fused Runge-Kutta stage takes q from here
// instead of reading it from memory a second time.  Entries at or past nval
// repeat the last valid one (they are never stored).
template <int TQ>
__device__ inline void tile_from_lds(const double* sq, int nval, int lane, double v[5][(TQ + 63) / 64]) {
  constexpr int KN = (TQ + 63) / 64;
#pragma unroll
  for (int f = 0; f < 5; ++f)
#pragma unroll
    for (int k = 0; k < KN; ++k) {
      const int i = 64 * k + lane;
      v[f][k] = sq[f * TQ + (i < nval ? i : nval - 1)];
    }
}

// store_tile's fused stage with the old state already in registers (qv from
// tile_from_lds): only the residual is read from memory, every res value of a
// round of fields before the round's first store.
template <int TQ>
__device__ inline void store_tile_stage(const double* sq, const double qv[5][(TQ + 63) / 64], int nval, int64_t base,
                                        int64_t Es, int lane, const double* res_in, double* res, double* qout, double a,
                                        double b, double dt, unsigned* flags) {
  constexpr int KN = (TQ + 63) / 64;
  constexpr int FG = tile_round_fields<TQ>();
  {
    int lo = static_cast<int>(base), hi = static_cast<int>(base >> 32);
    asm volatile("" : "+v"(lo), "+v"(hi));
    base = (static_cast<int64_t>(hi) << 32) | static_cast<uint32_t>(lo);
  }
  bool bad = false;
#pragma unroll
  for (int f0 = 0; f0 < 5; f0 += FG) {
    double rv[FG][KN];
#pragma unroll
    for (int ff = 0; ff < FG; ++ff)
#pragma unroll
      for (int k = 0; k < KN; ++k) {
        const int i = 64 * k + lane;
        const int64_t idx = (f0 + ff) * Es + base + (i < nval ? i : nval - 1);  // clamped: unconditional loads
        rv[ff][k] = f0 + ff < 5 && a != 0.0 ? res_in[idx] : 0.0;
      }
#pragma unroll
    for (int ff = 0; ff < FG; ++ff)
#pragma unroll
      for (int k = 0; k < KN; ++k) {
        const int i = 64 * k + lane;
        if (f0 + ff < 5 && i < nval)
          bad |= nonfinite(stage_store((f0 + ff) * Es + base + i, sq[(f0 + ff) * TQ + i], rv[ff][k], qv[f0 + ff][k], res,
                                       qout, a, b, dt));
      }
  }
  raise_flag(flags, bad, kFlagNonFinite);
}

}  // namespace dg
