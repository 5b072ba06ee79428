// Internal declarations shared by the host runtime and the kernel launchers.
#pragma once
#include <hip/hip_runtime.h>

#include <cstdint>
#include <string>
#include <vector>

#include "../../include/dg.h"
#include "../../include/dg_hex.h"
#include "refelem.hpp"

namespace dg {

// Records a failure for dg_last_error() and returns its status.
dg_status fail(dg_status s, const std::string& msg);
dg_status hip_fail(hipError_t e, const char* what);

// Device-side failure flags: one word per device, OR-ed by kernels and read
// (and cleared) by dg_synchronize.
constexpr unsigned kFlagNoConv = 1u;     // a Newton solve ended without converging
constexpr unsigned kFlagNonFinite = 2u;  // a non-finite value was produced
// Address of the current device's flag word (the device must be current).
unsigned* device_flags();

// True for NaN and +-Inf.
__device__ inline bool nonfinite(double v) { return !(__builtin_fabs(v) <= 1.7976931348623157e308); }
// One atomic OR per lane that saw a failure (none in the normal case).
__device__ inline void raise_flag(unsigned* flags, bool bad, unsigned bit) {
  if (bad && flags) atomicOr(flags, bit);
}

// Low-storage five-stage fourth-order Runge-Kutta coefficients
// (Carpenter & Kennedy 1994): res <- A_s res + dt rhs, q <- q + B_s res.
extern const double kLsrkA[5];
extern const double kLsrkB[5];

// Makes `dev` current for its lifetime and restores the previous device.
struct DeviceGuard {
  int prev = 0;
  bool ok = false;
  explicit DeviceGuard(int dev) {
    hipGetDevice(&prev);
    ok = hipSetDevice(dev) == hipSuccess;
  }
  ~DeviceGuard() { hipSetDevice(prev); }
  DeviceGuard(const DeviceGuard&) = delete;
  DeviceGuard& operator=(const DeviceGuard&) = delete;
};

#define DG_HIP(call)                                     \
  do {                                                   \
    hipError_t _e = (call);                              \
    if (_e != hipSuccess) return ::dg::hip_fail(_e, #call); \
  } while (0)

// Element-local contraction operator in the register layout of the FP64
// matrix-core tiles: for k-step ks and row block rb, lane l of a wave holds
// Op[row(rb, l)][4 ks + l / 16] where Op = [-Dr | -Ds | -Dt | LIFT] with each
// differentiation block padded to a multiple of 4 columns.  Row blocks are
// 16-row blocks (row 16 rb + l % 16) followed by 4-row blocks
// (row 16 NB16 + 4 (rb - NB16) + l % 4); rows >= Np are zero.
struct OpLayout {
  int p, Np, Nfp;
  int NPP;   // differentiation block width padded to a multiple of 4
  int NB16;  // number of 16-row blocks
  int NB4;   // number of 4-row blocks
  int KV;    // k-steps per differentiation block
  int KL;    // k-steps of the lift block (4 Nfp / 4)
  int KS;    // total k-steps
  int NRB;   // NB16 + NB4
};
OpLayout op_layout(int p);

// Layout of the reduced-precision operator tables.
//  FP32:  op32[KS32][NR][64], lane l holding Op[16 rb + l % 16][4 ks + l / 16]
//         (same K order as the FP64 table), 16-row blocks, rows >= Np zero;
//         with REM4 the last block holds 4 rows, lane l Op[16 rb + l % 4][4 ks + l / 16].
//  BF16:  opbf[VKS + FKS][NR][2 (hi, lo)][64][8]: lane l = i + 16 g holds
//         8 consecutive K slots t = 8 k .. 8 k + 7 of lane group g, where the
//         volume slots t = 3 s + a map to column a NPP + 4 s + g and the
//         face slots t map to column 3 NPP + 4 t + g; unused slots are zero.
//         x = fp32(Op), hi = bf16(x), lo = bf16(x - hi), round to nearest even.
struct LowpLayout {
  int Np, Nfp, NPP, KV, KL, NR, KS32, VKS, FKS;
  bool REM4;  // FP32: last of at most two row blocks has at most 4 rows (4x4 blocks)
};
LowpLayout lowp_layout(int p);

struct Mesh {
  int device = 0;
  int p = 0, Np = 0, Nfp = 0;
  int64_t E = 0;
  int64_t Epad = 0;  // E rounded up to a multiple of 16 (SoA stride)
  RefElem ref;
  OpLayout lay{};
  std::vector<double> elem_xyz;   // host copy [E][4][3]
  std::vector<int32_t> conn_host; // [4][Epad][2]: neighbour element, code = 6 nbr_face + perm
  std::vector<uint8_t> nbtab;     // [4][24][Nfp]: neighbour volume node of face node m
  // device
  double* d_geo = nullptr;        // [9][Epad] metric terms rx ry rz sx sy sz tx ty tz
  int2* d_conn = nullptr;         // [4][Epad]
  double* d_op64 = nullptr;       // [KS][NRB][64]
  double* d_opT = nullptr;        // [3 Np + 4 Nfp][Np]: [D_r | D_s | D_t | LIFT] transposed
  float* d_op32 = nullptr;        // FP32 table (LowpLayout)
  uint16_t* d_opbf = nullptr;     // BF16 hi/lo table (LowpLayout)
  int* d_fmask = nullptr;         // [4][Nfp]
  uint8_t* d_nbtab = nullptr;     // [4][24][Nfp]
  // launch configuration per contraction precision (dg_precision index)
  dg_launch_config launch[3] = {{4, 1, 1, 1}, {4, 1, 1, 1}, {4, 1, 1, 1}};
};

// Buffers of stage s of a fused five-stage LSRK step over the caller's state
// q and two state-sized work buffers w1, w2.  A stage reads its state from
// q_in (neighbour traces included) and writes the new state to another
// buffer; the residual is read and written entry by entry, so it may move
// between buffers and share one with the new state.  Rotating the three
// buffers this way leaves the fifth stage's state in q without a copy:
//   stage  q_in  res_in  res_out  q_out
//     1     q     -       w1       w2
//     2     w2    w1      w1       q
//     3     q     w1      w1       w2
//     4     w2    w1      q        w1
//     5     w1    q       -        q
struct LsrkBuffers {
  const double* q_in;
  const double* res_in;
  double* res_out;
  double* q_out;
};
inline LsrkBuffers lsrk_buffers(int s, double* q, double* w1, double* w2) {
  switch (s) {
    case 0: return {q, w1, w1, w2};
    case 1: return {w2, w1, w1, q};
    case 2: return {q, w1, w1, w2};
    case 3: return {w2, w1, q, w1};
    default: return {w1, q, nullptr, q};
  }
}

// kernel launchers (defined in the .hip files)
// RHS of q; with fused_lsrk the result goes through the stage update
// (res <- a res_in + dt rhs; q_out <- q + b res) instead of being stored in
// rhs, res being skipped when null.
dg_status launch_rhs_euler_fp64(const Mesh& m, double gamma, const double* q, double* rhs, const double* res_in,
                                double* res, double* q_out, double a, double b, double dt, bool fused_lsrk,
                                hipStream_t s);
// Same, with the contraction in FP32 or split BF16.
dg_status launch_rhs_euler_lowp(const Mesh& m, dg_precision prec, double gamma, const double* q, double* rhs,
                                const double* res_in, double* res, double* q_out, double a, double b, double dt,
                                bool fused_lsrk, hipStream_t s);
dg_status launch_lsrk_update(int64_t n, double a, double b, double dt, const double* rhs, double* res,
                             double* q, hipStream_t s);
// One LSRK(5,4) Euler step of q in place; work = two state-sized buffers
// (2 x 5 E Np doubles); the mesh's device is current.
dg_status rk_step_euler(const Mesh& m, double gamma, dg_precision prec, double* q, double* work, double dt,
                        hipStream_t stream);
// dg_rhs / dg_rk_step with model 1 (reacting Navier-Stokes), prm->work scratch.
dg_status ns_rhs_model1(const Mesh& m, const dg_params* prm, const double* q, double* rhs, hipStream_t s);
dg_status ns_step_model1(const Mesh& m, const dg_params* prm, double* q, double dt, hipStream_t s);
// q[f][n] <- v[f] for f < 5 (a uniform state).
dg_status launch_fill_state(double* q, int64_t n, const double v[5], hipStream_t s);

}  // namespace dg
