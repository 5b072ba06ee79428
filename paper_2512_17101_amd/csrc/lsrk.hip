// Pointwise stage of the 2N-storage Runge-Kutta scheme, FP64:
//   res <- a res + dt rhs;  q <- q + b res.
// A non-finite new state raises the device's non-finite flag.
// A stage with a = 0 does not read res (it may hold anything).
#include "internal.hpp"

namespace dg {
namespace {

__global__ __launch_bounds__(256) void lsrk_update_kernel(int64_t n, double a, double b, double dt,
                                                          const double* __restrict__ rhs, double* __restrict__ res,
                                                          double* __restrict__ q, unsigned* flags) {
  const int64_t stride = static_cast<int64_t>(gridDim.x) * blockDim.x;
  bool bad = false;
  for (int64_t i = static_cast<int64_t>(blockIdx.x) * blockDim.x + threadIdx.x; i < n; i += stride) {
    const double r = (a == 0.0 ? 0.0 : a * res[i]) + dt * rhs[i];
    const double qn = q[i] + b * r;
    bad |= nonfinite(qn);
    res[i] = r;
    q[i] = qn;
  }
  raise_flag(flags, bad, kFlagNonFinite);
}

struct Five {
  double v[5];
};

__global__ __launch_bounds__(256) void fill_state_kernel(double* __restrict__ q, int64_t n, Five v) {
  const int64_t stride = static_cast<int64_t>(gridDim.x) * blockDim.x;
  for (int64_t i = static_cast<int64_t>(blockIdx.x) * blockDim.x + threadIdx.x; i < n; i += stride)
#pragma unroll
    for (int f = 0; f < 5; ++f) q[f * n + i] = v.v[f];
}

}  // namespace

dg_status launch_fill_state(double* q, int64_t n, const double v[5], hipStream_t s) {
  if (n <= 0) return DG_OK;
  Five f;
  for (int k = 0; k < 5; ++k) f.v[k] = v[k];
  int64_t blocks = (n + 255) / 256;
  if (blocks > 256 * 64) blocks = 256 * 64;
  fill_state_kernel<<<static_cast<unsigned>(blocks), 256, 0, s>>>(q, n, f);
  DG_HIP(hipGetLastError());
  return DG_OK;
}

dg_status launch_lsrk_update(int64_t n, double a, double b, double dt, const double* rhs, double* res, double* q,
                             hipStream_t s) {
  const int64_t threads = 256;
  int64_t blocks = (n + threads - 1) / threads;
  if (blocks > 256 * 64) blocks = 256 * 64;
  lsrk_update_kernel<<<static_cast<unsigned>(blocks), threads, 0, s>>>(n, a, b, dt, rhs, res, q, device_flags());
  DG_HIP(hipGetLastError());
  return DG_OK;
}

}  // namespace dg
