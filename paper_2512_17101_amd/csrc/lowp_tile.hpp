// One 16-element tile of the Euler right-hand side with reduced-precision
// element contractions (FP32 or split BF16 on the matrix cores), shared by the
// single-mesh and the batched multi-mesh kernels.
//
// Only the contraction rhs = [-Dr | -Ds | -Dt | LIFT] [G_r; G_s; G_t; Delta]
// changes precision; fluxes, jumps, the state and the Runge-Kutta stage stay
// FP64.  One wave owns 16 elements, lane (n, g) = (element, residue mod 4) as
// in the FP64 kernel; the FP64 operands are rounded where they enter the
// matrix cores:
//
//  FP32        v_mfma_f32_16x16x4f32, K stepped by 4, lane (n, g) supplying
//              k = 4 ks + g (the same node / face-node mapping as FP64);
//              rows in 16-row blocks, output row 16 rb + 4 g + v in lane (n, g)
//              register v.  When the last block holds at most 4 rows (p = 1
//              and 3) it runs on v_mfma_f32_4x4x1_16b instead: block
//              (g, n / 4) multiplies the 4 rows by the k = 4 ks + g entries of
//              elements 4 (n / 4) .. + 3, so lane (n, g) accumulates the
//              k = g (mod 4) part of each row of element n, and the four lane
//              groups are summed once after the last k-step (a quarter of the
//              matrix-core cycles of a padded 16-row block).
//  split BF16  v_mfma_f32_16x16x32_bf16 with x = hi + lo (hi = bf16(x),
//              lo = bf16(x - hi)) and Op X ~ Op_hi X_hi + Op_hi X_lo +
//              Op_lo X_hi accumulated in FP32; the split is taken in FP32
//              (x = fp32 of the FP64 operand).  Each k-step takes 8 slots from
//              every lane group g; the host permutes the operator's K axis so
//              that lane group g's slots are exactly the values that lane
//              computed: volume slots t = 3 s + a (node 4 s + g, direction
//              a), then face slots t (face node 4 t + g), each padded to a
//              multiple of 8.
//
// Delta form (both modes): the volume operands are G_a(node j) - G_a(node 0)
// of the element.  Every row of D_a sums to zero, so the contraction is
// unchanged in exact arithmetic, while the rounded operands carry the flux
// variation inside the element instead of its level (the pressure part of
// the momentum flux, for instance), and the rounding error shrinks with it.
#pragma once
#include "euler_point.hpp"

namespace dg {
namespace lowp {

typedef float v4f __attribute__((ext_vector_type(4)));
typedef __bf16 v8bf __attribute__((ext_vector_type(8)));
typedef float v2f __attribute__((ext_vector_type(2)));
typedef __bf16 v2bf __attribute__((ext_vector_type(2)));

template <int P>
struct LCfg {
  static constexpr int NP = (P + 1) * (P + 2) * (P + 3) / 6;
  static constexpr int NFP = (P + 1) * (P + 2) / 2;
  static constexpr int NPP = (NP + 3) / 4 * 4;
  static constexpr int KV = NPP / 4;        // node steps per lane
  static constexpr int KL = NFP;            // face-node steps per lane
  static constexpr int NR = (NP + 15) / 16; // 16-row blocks
  // FP32: the last block has at most 4 rows and runs as 4x4 blocks (p = 1
  // and 3; at p = 4 the extra accumulators would spill)
  static constexpr bool REM4 = NP % 16 != 0 && NP % 16 <= 4 && NR <= 2;
  static constexpr int KS32 = 3 * KV + KL;  // FP32 k-steps (4 wide)
  static constexpr int VKS = (3 * KV + 7) / 8;  // BF16 volume k-steps (32 wide)
  static constexpr int FKS = (KL + 7) / 8;      // BF16 face k-steps
  static constexpr int OP32 = KS32 * NR * 64;        // floats
  static constexpr int OPBF = (VKS + FKS) * NR * 2 * 64 * 8;  // bf16 values (hi, lo)
};

// Whether a kernel of order P keeps the face tables in LDS: up to p = 3; at
// p = 4 the 22.4 KB state tile alone bounds the waves per CU, so one-tile
// blocks read the (cache-resident) tables from memory instead.
template <int P>
constexpr bool lowp_lds_tables() { return P < 4; }

struct LowArgs {
  const double* __restrict__ q;
  double* __restrict__ rhs;
  const double* res_in;  // residual read by the fused stage (may alias res or qout)
  double* res;           // residual written by the fused stage (null: not stored)
  double* qout;
  const double* __restrict__ geo;
  const int2* __restrict__ conn;
  const float* __restrict__ op32;
  const uint16_t* __restrict__ opbf;
  const int* __restrict__ fmask;
  const uint8_t* __restrict__ nbtab;
  int64_t E, Epad;
  int ntiles;
  int xcd_run;  // single-mesh kernel: blocks per XCD run (1: plain order)
  double gamma, a, b, dt;
  unsigned* flags;  // device failure flags (non-finite output); may be null
};

// Lane (n, g) holds in register i the k = g (mod 4) part of row i of a 4-row
// block for element n; returns the whole of row g.  Reduce-scatter over the
// four lane groups: rows are halved between lane groups g and g ^ 2, then
// between g and g ^ 1.  Called by the whole wave.
__device__ inline float sum_lane_groups(v4f x, int g) {
  const bool hi = (g & 2) != 0;
  float k0 = hi ? x[2] : x[0], k1 = hi ? x[3] : x[1];
  const float s0 = hi ? x[0] : x[2], s1 = hi ? x[1] : x[3];
  k0 += __shfl_xor(s0, 32);
  k1 += __shfl_xor(s1, 32);
  const bool lo = (g & 1) != 0;
  const float k = lo ? k1 : k0, s = lo ? k0 : k1;
  return k + __shfl_xor(s, 16);
}

// Splits 8 staged FP32 slots per field into hi = bf16(x) and lo = bf16(x - hi)
// (round to nearest even; x - hi is exact in FP32), runs the three products
// Op_hi X_hi + Op_hi X_lo + Op_lo X_hi of k-step k on the matrix cores, and
// clears the slots.
template <int NR>
__device__ inline void split_mma(const v8bf* __restrict__ op, int k, int lane, float (&xf)[5][8], v4f (&acc)[5][NR]) {
#pragma unroll
  for (int f = 0; f < 5; ++f) {
    union { v2bf h[4]; v8bf v; } hi, lo;
#pragma unroll
    for (int w = 0; w < 4; ++w) {
      const v2f x = {xf[f][2 * w], xf[f][2 * w + 1]};
      hi.h[w] = __builtin_convertvector(x, v2bf);
      const v2f h = __builtin_convertvector(hi.h[w], v2f);
      lo.h[w] = __builtin_convertvector(x - h, v2bf);
      xf[f][2 * w] = 0.f;
      xf[f][2 * w + 1] = 0.f;
    }
#pragma unroll
    for (int rb = 0; rb < NR; ++rb) {
      const v8bf ah = op[((k * NR + rb) * 2 + 0) * 64 + lane];
      const v8bf al = op[((k * NR + rb) * 2 + 1) * 64 + lane];
      acc[f][rb] = __builtin_amdgcn_mfma_f32_16x16x32_bf16(ah, hi.v, acc[f][rb], 0, 0, 0);
      acc[f][rb] = __builtin_amdgcn_mfma_f32_16x16x32_bf16(ah, lo.v, acc[f][rb], 0, 0, 0);
      acc[f][rb] = __builtin_amdgcn_mfma_f32_16x16x32_bf16(al, hi.v, acc[f][rb], 0, 0, 0);
    }
  }
}

// One 16-element tile of one mesh: the whole right-hand side (or fused
// Runge-Kutta stage) of elements 16 tile .. 16 tile + 15.  `op` is the
// operator table in the mode's layout, nb / fm the face tables.  With
// STAGED, `sq` is this wave's LDS buffer of 5 x 16 Np doubles: the tile's
// state is first copied there with coalesced loads (with DMA, through the LDS
// DMA path: Np a multiple of 4, q 16-byte aligned, sq 512-byte aligned), and
// own traces and neighbour traces inside the tile are read from it.
template <int P, int MODE, bool FUSED, bool STAGED = false, bool DMA = false>
__device__ inline void lowp_tile(const LowArgs& A, const uint32_t* __restrict__ s_op, const uint8_t* __restrict__ s_nb,
                                 const int* __restrict__ s_fm, int64_t tile, double* __restrict__ sq = nullptr) {
  using C = LCfg<P>;
  constexpr int TQ = 16 * C::NP;
  const int lane = threadIdx.x & 63;
  const int n = lane & 15, g = lane >> 4;
  const int64_t Es = A.E * C::NP;
  const double* __restrict__ q = A.q;
  const double gm1 = A.gamma - 1.0;
  const int64_t e0 = tile * 16;
  const int nval = static_cast<int>(A.E - e0 < 16 ? A.E - e0 : 16) * C::NP;
  if constexpr (STAGED && DMA)
    stage_tile_dma<TQ>(sq, q, Es, e0 * C::NP, nval, lane);
  else if constexpr (STAGED)
    stage_tile<TQ>(sq, q, Es, e0 * C::NP, nval, lane);
  {
    const int64_t e = e0 + n;
    const bool valid = e < A.E;
    const int64_t ec = valid ? e : A.E - 1;
    const int nl = static_cast<int>(ec - e0);  // element row in the tile
    // own-element node value of field f (staged tile or memory)
    auto own_q = [&](int f, int j) -> double {
      if constexpr (STAGED) return sq[f * TQ + nl * C::NP + j];
      else return q[f * Es + ec * C::NP + j];
    };
    double gm[9];
#pragma unroll
    for (int c = 0; c < 9; ++c) gm[c] = A.geo[c * A.Epad + ec];
    int2 cn[4];
#pragma unroll
    for (int f = 0; f < 4; ++f) cn[f] = A.conn[f * A.Epad + ec];

    v4f acc[5][C::NR];
#pragma unroll
    for (int f = 0; f < 5; ++f)
#pragma unroll
      for (int rb = 0; rb < C::NR; ++rb) acc[f][rb] = v4f{0.f, 0.f, 0.f, 0.f};

    // fluxes of the element's node 0: the reference of the delta form
    double G0[3][5];
    {
      double q0[5];
#pragma unroll
      for (int f = 0; f < 5; ++f) q0[f] = own_q(f, 0);
      contravariant_flux(q0, gm, gm1, G0);
    }

    if constexpr (MODE == 1) {
      const float* op = reinterpret_cast<const float*>(s_op);
      // 16-row blocks 0 .. NR16 - 1 in acc, the 4-row remainder (REM4) in acc4
      constexpr int NR16 = C::REM4 ? C::NR - 1 : C::NR;
      v4f acc4[5];
#pragma unroll
      for (int f = 0; f < 5; ++f) acc4[f] = v4f{0.f, 0.f, 0.f, 0.f};
      auto mma = [&](const float a, int rb, const double (&B)[5]) {
#pragma unroll
        for (int f = 0; f < 5; ++f) {
          if (rb < NR16)
            acc[f][rb] = __builtin_amdgcn_mfma_f32_16x16x4f32(a, static_cast<float>(B[f]), acc[f][rb], 0, 0, 0);
          else
            acc4[f] = __builtin_amdgcn_mfma_f32_4x4x1f32(a, static_cast<float>(B[f]), acc4[f], 0, 0, 0);
        }
      };
#pragma unroll
      for (int s = 0; s < C::KV; ++s) {
        const int j = 4 * s + g;
        double G[3][5];
        if (j < C::NP) {
          double qq[5];
#pragma unroll
          for (int f = 0; f < 5; ++f) qq[f] = own_q(f, j);
          contravariant_flux(qq, gm, gm1, G);
#pragma unroll
          for (int r = 0; r < 3; ++r)
#pragma unroll
            for (int f = 0; f < 5; ++f) G[r][f] -= G0[r][f];
        } else {
#pragma unroll
          for (int r = 0; r < 3; ++r)
#pragma unroll
            for (int f = 0; f < 5; ++f) G[r][f] = 0.0;
        }
#pragma unroll
        for (int r = 0; r < 3; ++r)
#pragma unroll
          for (int rb = 0; rb < C::NR; ++rb) mma(op[((r * C::KV + s) * C::NR + rb) * 64 + lane], rb, G[r]);
      }
      // whole face loop unrolled up to p = 3; at p = 4 by two (registers)
      constexpr int FU = P < 4 ? C::KL : 2;
#pragma unroll FU
      for (int s = 0; s < C::KL; ++s) {
        const int fm = 4 * s + g;
        const int face = fm / C::NFP;
        const int mm = fm - face * C::NFP;
        const int2 c = face == 0 ? cn[0] : face == 1 ? cn[1] : face == 2 ? cn[2] : cn[3];
        const int own = s_fm[fm];
        const int jp = s_nb[(face * 24 + c.y) * C::NFP + mm];
        double qm[5], qp[5], D[5];
        const int64_t nloc = static_cast<int64_t>(c.x) - e0;
        const bool in_tile = STAGED && nloc >= 0 && nloc < 16;
#pragma unroll
        for (int f = 0; f < 5; ++f) {
          qm[f] = own_q(f, own);
          if constexpr (STAGED)
            qp[f] = in_tile ? sq[f * TQ + static_cast<int>(nloc) * C::NP + jp]
                            : q[f * Es + static_cast<int64_t>(c.x) * C::NP + jp];
          else
            qp[f] = q[f * Es + static_cast<int64_t>(c.x) * C::NP + jp];
        }
        double Nx, Ny, Nz;
        if constexpr (FU == C::KL)
          step_normal<C::NFP>(s, face, gm, Nx, Ny, Nz);  // s is a constant here
        else
          scaled_normal(face, gm, Nx, Ny, Nz);
        lf_jump(qm, qp, Nx, Ny, Nz, A.gamma, D);
#pragma unroll
        for (int rb = 0; rb < C::NR; ++rb) mma(op[((3 * C::KV + s) * C::NR + rb) * 64 + lane], rb, D);
      }
      // remainder rows: lane (n, g) keeps row 16 NR16 + g of element n in register 0
      if constexpr (C::REM4) {
#pragma unroll
        for (int f = 0; f < 5; ++f) acc[f][NR16] = v4f{sum_lane_groups(acc4[f], g), 0.f, 0.f, 0.f};
      }
    } else {
      const v8bf* op = reinterpret_cast<const v8bf*>(s_op);  // [k][rb][part][64]
      // One k-step's 8 slots per field are staged in FP32, then split and
      // sent to the matrix cores.  Volume slot t = 3 s + a holds direction a of
      // node step s; face slot t holds face-node step t.
      float xf[5][8];
#pragma unroll
      for (int f = 0; f < 5; ++f)
#pragma unroll
        for (int t = 0; t < 8; ++t) xf[f][t] = 0.f;
      double G[3][5];
#pragma unroll
      for (int t = 0; t < 3 * C::KV; ++t) {
        const int s = t / 3, r = t % 3;
        if (r == 0) {
          const int j = 4 * s + g;
          if (j < C::NP) {
            double qq[5];
#pragma unroll
            for (int f = 0; f < 5; ++f) qq[f] = own_q(f, j);
            contravariant_flux(qq, gm, gm1, G);
#pragma unroll
            for (int a = 0; a < 3; ++a)
#pragma unroll
              for (int f = 0; f < 5; ++f) G[a][f] -= G0[a][f];
          } else {
#pragma unroll
            for (int a = 0; a < 3; ++a)
#pragma unroll
              for (int f = 0; f < 5; ++f) G[a][f] = 0.0;
          }
        }
#pragma unroll
        for (int f = 0; f < 5; ++f) xf[f][t % 8] = static_cast<float>(G[r][f]);
        if (t % 8 == 7 || t == 3 * C::KV - 1) split_mma<C::NR>(op, t / 8, lane, xf, acc);
      }
#pragma unroll
      for (int t = 0; t < C::KL; ++t) {
        const int fm = 4 * t + g;
        const int face = fm / C::NFP;
        const int mm = fm - face * C::NFP;
        const int2 c = face == 0 ? cn[0] : face == 1 ? cn[1] : face == 2 ? cn[2] : cn[3];
        const int own = s_fm[fm];
        const int jp = s_nb[(face * 24 + c.y) * C::NFP + mm];
        double qm[5], qp[5], D[5];
        const int64_t nloc = static_cast<int64_t>(c.x) - e0;
        const bool in_tile = STAGED && nloc >= 0 && nloc < 16;
#pragma unroll
        for (int f = 0; f < 5; ++f) {
          qm[f] = own_q(f, own);
          if constexpr (STAGED)
            qp[f] = in_tile ? sq[f * TQ + static_cast<int>(nloc) * C::NP + jp]
                            : q[f * Es + static_cast<int64_t>(c.x) * C::NP + jp];
          else
            qp[f] = q[f * Es + static_cast<int64_t>(c.x) * C::NP + jp];
        }
        double Nx, Ny, Nz;
        step_normal<C::NFP>(t, face, gm, Nx, Ny, Nz);
        lf_jump(qm, qp, Nx, Ny, Nz, A.gamma, D);
#pragma unroll
        for (int f = 0; f < 5; ++f) xf[f][t % 8] = static_cast<float>(D[f]);
        if (t % 8 == 7 || t == C::KL - 1) split_mma<C::NR>(op, C::VKS + t / 8, lane, xf, acc);
      }
    }

    // store: lane (n, g) register v holds row 16 rb + 4 g + v (in FP32 mode
    // the REM4 block holds row 16 rb + g in register 0 only)
    auto out_row = [&](int rb, int v) -> int {
      if (MODE == 1 && C::REM4 && rb == C::NR - 1) return v == 0 ? 16 * rb + g : C::NP;
      return 16 * rb + 4 * g + v;
    };
    if constexpr (STAGED) {
      // through the LDS tile buffer (the state is no longer needed there;
      // the fused stage first takes its share of it into registers):
      // coalesced stores, and in the fused stage all res loads of a round in
      // flight together
      constexpr int KN = (TQ + 63) / 64;
      double qv[FUSED ? 5 : 1][FUSED ? KN : 1];
      if constexpr (FUSED) tile_from_lds<TQ>(sq, nval, lane, qv);
      __builtin_amdgcn_wave_barrier();
      if (valid) {
#pragma unroll
        for (int f = 0; f < 5; ++f)
#pragma unroll
          for (int rb = 0; rb < C::NR; ++rb)
#pragma unroll
            for (int v = 0; v < 4; ++v) {
              const int row = out_row(rb, v);
              if (row < C::NP) sq[f * TQ + n * C::NP + row] = static_cast<double>(acc[f][rb][v]);
            }
      }
      __builtin_amdgcn_wave_barrier();
      if constexpr (FUSED)
        store_tile_stage<TQ>(sq, qv, nval, e0 * C::NP, Es, lane, A.res_in, A.res, A.qout, A.a, A.b, A.dt, A.flags);
      else
        store_tile<false, TQ>(sq, nval, e0 * C::NP, Es, lane, A.rhs, A.res_in, A.res, A.qout, q, A.a, A.b, A.dt,
                              A.flags);
    } else if constexpr (!FUSED) {
      if (valid) {
        bool bad = false;
#pragma unroll
        for (int f = 0; f < 5; ++f)
#pragma unroll
          for (int rb = 0; rb < C::NR; ++rb)
#pragma unroll
            for (int v = 0; v < 4; ++v) {
              const int row = out_row(rb, v);
              if (row < C::NP) {
                const double val = static_cast<double>(acc[f][rb][v]);
                bad |= nonfinite(val);
                A.rhs[f * Es + e * C::NP + row] = val;
              }
            }
        raise_flag(A.flags, bad, kFlagNonFinite);
      }
    } else if (valid) {
      bool bad = false;
      // one field per round: its res and q loads all issued before its stores
#pragma unroll
      for (int f = 0; f < 5; ++f) {
        double rv[C::NR][4], qv[C::NR][4];
#pragma unroll
        for (int rb = 0; rb < C::NR; ++rb)
#pragma unroll
          for (int v = 0; v < 4; ++v) {
            const int row = out_row(rb, v);
            const int64_t idx = f * Es + e * C::NP + (row < C::NP ? row : C::NP - 1);  // clamped: unconditional
            rv[rb][v] = A.a != 0.0 ? A.res_in[idx] : 0.0;
            qv[rb][v] = q[idx];
          }
#pragma unroll
        for (int rb = 0; rb < C::NR; ++rb)
#pragma unroll
          for (int v = 0; v < 4; ++v) {
            const int row = out_row(rb, v);
            if (row < C::NP)
              bad |= nonfinite(stage_store(f * Es + e * C::NP + row, static_cast<double>(acc[f][rb][v]), rv[rb][v],
                                           qv[rb][v], A.res, A.qout, A.a, A.b, A.dt));
          }
      }
      raise_flag(A.flags, bad, kFlagNonFinite);
    }
  }
}

}  // namespace lowp
}  // namespace dg
