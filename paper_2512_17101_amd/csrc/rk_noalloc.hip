// One LSRK(5,4) Euler step that allocates nothing: dg_rk_step with its
// two state-sized work buffers in a fixed device array instead of a
// caller workspace, for callers that cannot allocate device memory.
//
// The array is a file-scope device variable: the code object reserves it on
// every GPU the library runs on, at its own address there, until the process
// ends.  Host code never passes the variable's name to a kernel (on the host
// it only stands for the symbol): the device address is looked up once per
// device with hipGetSymbolAddress, with that device current, and only that
// address is used.  Calls on one GPU share the array, so calls that overlap
// in time on one GPU race; the step needs no part of it cleared (the first
// stage ignores the old residual, multiplying it by zero is skipped).
#include <mutex>
#include <string>

#include "internal.hpp"

namespace {

// two state arrays of kNoAllocMaxState doubles each (2 x 64 MiB)
constexpr size_t kNoAllocMaxState = DG_NOALLOC_MAX_STATE;
__device__ __align__(256) double scratch[2 * kNoAllocMaxState];

constexpr int kMaxDevices = 64;
std::mutex g_mu;
double* g_scratch[kMaxDevices] = {};

// device address of this GPU's copy of the array (the device is current)
dg_status scratch_address(int dev, double** out) {
  if (dev < 0 || dev >= kMaxDevices) return dg::fail(DG_ERR_ARG, "dg_rk_step_noalloc: device index too large");
  std::lock_guard<std::mutex> lk(g_mu);
  if (!g_scratch[dev]) {
    void* p = nullptr;
    const hipError_t e = hipGetSymbolAddress(&p, HIP_SYMBOL(scratch));
    if (e != hipSuccess || !p) return dg::hip_fail(e, "dg_rk_step_noalloc: hipGetSymbolAddress");
    g_scratch[dev] = static_cast<double*>(p);
  }
  *out = g_scratch[dev];
  return DG_OK;
}

}  // namespace

using namespace dg;

extern "C" dg_status dg_rk_step_noalloc(dg_mesh h, const dg_params* prm, dg_precision prec, double* q, double t,
                                        double dt, hipStream_t stream) {
  (void)t;
  if (!h) return fail(DG_ERR_ARG, "dg_rk_step_noalloc: null mesh");
  if (!prm) return fail(DG_ERR_ARG, "dg_rk_step_noalloc: params is NULL");
  if (prec != DG_FP64 && prec != DG_FP32 && prec != DG_SPLIT_BF16)
    return fail(DG_ERR_ARG, "dg_rk_step_noalloc: unknown precision");
  if (prm->model != 0)
    return fail(DG_ERR_UNSUPPORTED, "dg_rk_step_noalloc: Euler (model 0) only; use dg_rk_step for the reacting model");
  if (!(prm->gamma > 1.0) || !std::isfinite(prm->gamma)) return fail(DG_ERR_ARG, "dg_rk_step_noalloc: gamma must be > 1");
  if (!std::isfinite(dt)) return fail(DG_ERR_ARG, "dg_rk_step_noalloc: dt must be finite");
  if (!q || (reinterpret_cast<uintptr_t>(q) & 7u)) return fail(DG_ERR_ARG, "dg_rk_step_noalloc: null or misaligned q");
  const Mesh& m = *reinterpret_cast<const Mesh*>(h);
  const size_t n = static_cast<size_t>(5) * m.E * m.Np;
  if (n > kNoAllocMaxState)
    return fail(DG_ERR_ARG, "dg_rk_step_noalloc: the state holds " + std::to_string(n) +
                                " doubles, above the limit of " + std::to_string(kNoAllocMaxState) +
                                " (5 E Np); use dg_rk_step with a workspace");
  DeviceGuard g(m.device);
  if (!g.ok) return fail(DG_ERR_HIP, "dg_rk_step_noalloc: hipSetDevice failed");
  double* work = nullptr;
  dg_status st = scratch_address(m.device, &work);
  if (st != DG_OK) return st;
  return rk_step_euler(m, prm->gamma, prec, q, work, dt, stream);
}
