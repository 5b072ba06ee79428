// C-ABI entry points that are not mesh construction: error reporting,
// reference-operator export, right-hand side and Runge-Kutta stepping.
#include <cmath>
#include <cstring>
#include <string>

#include "internal.hpp"

namespace dg {

namespace {
thread_local std::string g_last_error;
}

dg_status fail(dg_status s, const std::string& msg) {
  g_last_error = msg;
  return s;
}

dg_status hip_fail(hipError_t e, const char* what) {
  return fail(DG_ERR_HIP, std::string(what) + ": " + hipGetErrorString(e));
}

// Carpenter & Kennedy (1994) five-stage fourth-order 2N-storage coefficients.
const double kLsrkA[5] = {0.0, -567301805773.0 / 1357537059087.0, -2404267990393.0 / 2016746695238.0,
                          -3550918686646.0 / 2091501179385.0, -1275806237668.0 / 842570457699.0};
const double kLsrkB[5] = {1432997174477.0 / 9575080441755.0, 5161836677717.0 / 13612068292357.0,
                          1720146321549.0 / 2090206949498.0, 3134564353537.0 / 4481467310338.0,
                          2277821191437.0 / 14882151754819.0};

// One LSRK(5,4) Euler step of q in place with work = two state-sized
// buffers (2 n doubles); the device is current.  Allocates nothing.
dg_status rk_step_euler(const Mesh& m, double gamma, dg_precision prec, double* q, double* work, double dt,
                        hipStream_t stream) {
  const size_t n = static_cast<size_t>(5) * m.E * m.Np;
  dg_status st = DG_OK;
  double* res = work;
  if (!m.launch[prec].rk_fused) {
    // RHS into work + n, then the pointwise stage update of q in place
    double* rhs = work + n;
    for (int s = 0; s < 5; ++s) {
      st = prec == DG_FP64
               ? launch_rhs_euler_fp64(m, gamma, q, rhs, nullptr, nullptr, nullptr, 0.0, 0.0, 0.0, false, stream)
               : launch_rhs_euler_lowp(m, prec, gamma, q, rhs, nullptr, nullptr, nullptr, 0.0, 0.0, 0.0, false, stream);
      if (st != DG_OK) return st;
      st = launch_lsrk_update(static_cast<int64_t>(n), kLsrkA[s], kLsrkB[s], dt, rhs, res, q, stream);
      if (st != DG_OK) return st;
    }
    return DG_OK;
  }
  for (int s = 0; s < 5; ++s) {
    const LsrkBuffers B = lsrk_buffers(s, q, work, work + n);
    st = prec == DG_FP64 ? launch_rhs_euler_fp64(m, gamma, B.q_in, nullptr, B.res_in, B.res_out, B.q_out, kLsrkA[s],
                                                 kLsrkB[s], dt, true, stream)
                         : launch_rhs_euler_lowp(m, prec, gamma, B.q_in, nullptr, B.res_in, B.res_out, B.q_out,
                                                 kLsrkA[s], kLsrkB[s], dt, true, stream);
    if (st != DG_OK) return st;
  }
  return DG_OK;
}

}  // namespace dg

using namespace dg;

namespace {

bool aligned8(const void* p) { return (reinterpret_cast<uintptr_t>(p) & 7u) == 0; }

dg_status check_params(const char* who, const dg_params* prm, dg_precision prec) {
  if (!prm) return fail(DG_ERR_ARG, std::string(who) + ": params is NULL");
  if (prec != DG_FP64 && prec != DG_FP32 && prec != DG_SPLIT_BF16)
    return fail(DG_ERR_ARG, std::string(who) + ": unknown precision");
  if (prm->model == 1) {
    if (prec != DG_FP64)
      return fail(DG_ERR_UNSUPPORTED, std::string(who) + ": the reacting model runs FP64 contractions only");
    return DG_OK;
  }
  if (prm->model != 0) return fail(DG_ERR_ARG, std::string(who) + ": model must be 0 (Euler) or 1 (reacting NS)");
  if (!(prm->gamma > 1.0) || !std::isfinite(prm->gamma)) return fail(DG_ERR_ARG, std::string(who) + ": gamma must be > 1");
  return DG_OK;
}

}  // namespace

extern "C" const char* dg_last_error(void) { return g_last_error.c_str(); }

extern "C" dg_status dg_reference_operators(int order, double* rst, double* Dr, double* Ds, double* Dt,
                                            double* LIFT, int32_t* Fmask) {
  RefElem R;
  if (!build_ref_elem(order, R)) return fail(DG_ERR_ARG, "dg_reference_operators: order must be in 1..4");
  if (rst) std::memcpy(rst, R.rst.data(), R.rst.size() * sizeof(double));
  if (Dr) std::memcpy(Dr, R.Dr.data(), R.Dr.size() * sizeof(double));
  if (Ds) std::memcpy(Ds, R.Ds.data(), R.Ds.size() * sizeof(double));
  if (Dt) std::memcpy(Dt, R.Dt.data(), R.Dt.size() * sizeof(double));
  if (LIFT) std::memcpy(LIFT, R.LIFT.data(), R.LIFT.size() * sizeof(double));
  if (Fmask)
    for (size_t i = 0; i < R.Fmask.size(); ++i) Fmask[i] = R.Fmask[i];
  return DG_OK;
}

extern "C" dg_status dg_rhs(dg_mesh h, const dg_params* prm, dg_precision prec, const double* q, double* rhs,
                            hipStream_t stream) {
  if (!h) return fail(DG_ERR_ARG, "dg_rhs: null mesh");
  dg_status st = check_params("dg_rhs", prm, prec);
  if (st != DG_OK) return st;
  if (!q || !rhs || !aligned8(q) || !aligned8(rhs)) return fail(DG_ERR_ARG, "dg_rhs: null or misaligned state pointer");
  const Mesh& m = *reinterpret_cast<const Mesh*>(h);
  if (prm->model == 1) {
    DeviceGuard g(m.device);
    if (!g.ok) return fail(DG_ERR_HIP, "dg_rhs: hipSetDevice failed");
    return ns_rhs_model1(m, prm, q, rhs, stream);
  }
  const size_t n = static_cast<size_t>(5) * m.E * m.Np;
  if (q == rhs || (rhs < q + n && q < rhs + n)) return fail(DG_ERR_ARG, "dg_rhs: q and rhs overlap");
  DeviceGuard g(m.device);
  if (!g.ok) return fail(DG_ERR_HIP, "dg_rhs: hipSetDevice failed");
  if (prec == DG_FP64) return launch_rhs_euler_fp64(m, prm->gamma, q, rhs, nullptr, nullptr, nullptr, 0.0, 0.0, 0.0, false, stream);
  return launch_rhs_euler_lowp(m, prec, prm->gamma, q, rhs, nullptr, nullptr, nullptr, 0.0, 0.0, 0.0, false, stream);
}

extern "C" dg_status dg_rk_step(dg_mesh h, const dg_params* prm, dg_precision prec, double* q, double* work,
                                double t, double dt, hipStream_t stream) {
  (void)t;
  if (!h) return fail(DG_ERR_ARG, "dg_rk_step: null mesh");
  dg_status st = check_params("dg_rk_step", prm, prec);
  if (st != DG_OK) return st;
  if (!std::isfinite(dt)) return fail(DG_ERR_ARG, "dg_rk_step: dt must be finite");
  const Mesh& m = *reinterpret_cast<const Mesh*>(h);
  if (prm->model == 1) {
    if (!q || !aligned8(q)) return fail(DG_ERR_ARG, "dg_rk_step: null or misaligned pointer");
    DeviceGuard g(m.device);
    if (!g.ok) return fail(DG_ERR_HIP, "dg_rk_step: hipSetDevice failed");
    return ns_step_model1(m, prm, q, dt, stream);
  }
  if (!q || !work || !aligned8(q) || !aligned8(work)) return fail(DG_ERR_ARG, "dg_rk_step: null or misaligned pointer");
  const size_t n = static_cast<size_t>(5) * m.E * m.Np;
  if (work < q + n && q < work + 2 * n) return fail(DG_ERR_ARG, "dg_rk_step: work overlaps q");
  DeviceGuard g(m.device);
  if (!g.ok) return fail(DG_ERR_HIP, "dg_rk_step: hipSetDevice failed");
  return dg::rk_step_euler(m, prm->gamma, prec, q, work, dt, stream);
}

extern "C" dg_status dg_lsrk_update(int64_t n, double a, double b, double dt, const double* rhs, double* res,
                                    double* q, hipStream_t stream) {
  if (n < 0) return fail(DG_ERR_ARG, "dg_lsrk_update: negative size");
  if (n == 0) return DG_OK;
  if (!rhs || !res || !q || !aligned8(rhs) || !aligned8(res) || !aligned8(q))
    return fail(DG_ERR_ARG, "dg_lsrk_update: null or misaligned pointer");
  return launch_lsrk_update(n, a, b, dt, rhs, res, q, stream);
}
