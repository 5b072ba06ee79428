// C-ABI of the reacting Navier-Stokes right-hand side and its Runge-Kutta step.
#include <cmath>
#include <string>

#include "internal.hpp"
#include "ns.hpp"

namespace dg {
const ThermoTable& thermo_table(const dg_thermo_s* th);
int thermo_device(const dg_thermo_s* th);
const MechTable& mech_table(const dg_mech_s* mk);
int mech_device(const dg_mech_s* mk);
}  // namespace dg

using namespace dg;

namespace {

constexpr int kFields = 12, kGrad = 33;

bool aligned8(const void* p) { return (reinterpret_cast<uintptr_t>(p) & 7u) == 0; }

bool overlap(const double* a, size_t na, const double* b, size_t nb) { return a < b + nb && b < a + na; }

dg_status check(const char* who, const Mesh& m, const dg_params* prm) {
  const std::string w(who);
  if (!prm) return fail(DG_ERR_ARG, w + ": params is NULL");
  if (prm->model != 1) return fail(DG_ERR_ARG, w + ": model must be 1 (reacting Navier-Stokes)");
  if (!prm->thermo) return fail(DG_ERR_ARG, w + ": params.thermo is NULL");
  if (!(prm->mu >= 0.0) || !std::isfinite(prm->mu) || !(prm->Pr > 0.0) || !std::isfinite(prm->Pr) ||
      !(prm->Sc > 0.0) || !std::isfinite(prm->Sc))
    return fail(DG_ERR_ARG, w + ": need mu >= 0, Pr > 0 and Sc > 0 (finite)");
  if (thermo_table(prm->thermo).ns != 7) return fail(DG_ERR_UNSUPPORTED, w + ": the reacting path needs 7 species");
  if (thermo_device(prm->thermo) != m.device) return fail(DG_ERR_ARG, w + ": thermo table lives on another device");
  if (prm->mech) {
    if (mech_table(prm->mech).ns != 7) return fail(DG_ERR_UNSUPPORTED, w + ": the reacting path needs 7 species");
    if (mech_device(prm->mech) != m.device) return fail(DG_ERR_ARG, w + ": mechanism lives on another device");
  }
  return DG_OK;
}

NsArgs make_args(const Mesh& m, const dg_params* prm) {
  NsArgs A{};
  A.geo = m.d_geo;
  A.conn = m.d_conn;
  A.opT = m.d_opT;
  A.fmask = m.d_fmask;
  A.nbtab = m.d_nbtab;
  A.E = m.E;
  A.Epad = m.Epad;
  A.mu = prm->mu;
  A.Pr = prm->Pr;
  A.Sc = prm->Sc;
  A.th = thermo_table(prm->thermo);
  A.with_sources = prm->mech ? 1 : 0;
  if (prm->mech) A.mk = mech_table(prm->mech);
  return A;
}

}  // namespace

extern "C" dg_status dg_ns_rhs(dg_mesh h, const dg_params* prm, const double* q, const double* T, double* sigma,
                               double* rhs, hipStream_t stream) {
  if (!h) return fail(DG_ERR_ARG, "dg_ns_rhs: null mesh");
  const Mesh& m = *reinterpret_cast<const Mesh*>(h);
  dg_status st = check("dg_ns_rhs", m, prm);
  if (st != DG_OK) return st;
  if (!q || !T || !sigma || !rhs || !aligned8(q) || !aligned8(T) || !aligned8(sigma) || !aligned8(rhs))
    return fail(DG_ERR_ARG, "dg_ns_rhs: null or misaligned pointer");
  const size_t n = static_cast<size_t>(m.E) * m.Np;
  if (overlap(rhs, kFields * n, q, kFields * n) || overlap(rhs, kFields * n, T, n) ||
      overlap(rhs, kFields * n, sigma, kGrad * n) || overlap(sigma, kGrad * n, q, kFields * n) ||
      overlap(sigma, kGrad * n, T, n))
    return fail(DG_ERR_ARG, "dg_ns_rhs: outputs overlap inputs");
  DeviceGuard g(m.device);
  if (!g.ok) return fail(DG_ERR_HIP, "dg_ns_rhs: hipSetDevice failed");
  NsArgs A = make_args(m, prm);
  A.q = q;
  A.T = T;
  A.sigma = sigma;
  A.rhs = rhs;
  st = launch_ns_gradients(m.p, A, stream);
  if (st != DG_OK) return st;
  return launch_ns_rhs(m.p, A, false, stream);
}

namespace {

// One LSRK(5,4) step of the reacting system; T holds the first stage's Newton
// start (T_valid) or is filled from the plain start; work: 58 E Np doubles.
dg_status ns_step(const Mesh& m, const dg_params* prm, double* q, double* T, bool T_valid, double* work, double dt,
                  double tol, int max_iter, hipStream_t stream) {
  const size_t n = static_cast<size_t>(m.E) * m.Np;
  double* sigma = work + 2 * kFields * n;
  int32_t* iters = reinterpret_cast<int32_t*>(work + (2 * kFields + kGrad) * n);
  const ThermoTable& th = thermo_table(prm->thermo);
  NsArgs A = make_args(m, prm);
  A.sigma = sigma;
  A.T = T;
  A.dt = dt;
  for (int s = 0; s < 5; ++s) {
    const LsrkBuffers B = lsrk_buffers(s, q, work, work + kFields * n);
    A.q = B.q_in;
    A.res_in = B.res_in;
    A.res = B.res_out;
    A.qout = B.q_out;
    A.a = kLsrkA[s];
    A.b = kLsrkB[s];
    dg_status st = launch_temperature(th, static_cast<int64_t>(n), A.q, (s > 0 || T_valid) ? T : nullptr, kTdefault, T,
                                      iters, tol, max_iter, stream);
    if (st != DG_OK) return st;
    st = launch_ns_gradients(m.p, A, stream);
    if (st != DG_OK) return st;
    st = launch_ns_rhs(m.p, A, true, stream);
    if (st != DG_OK) return st;
  }
  return DG_OK;
}

double newton_tol(const dg_params* prm) { return prm->tol > 0.0 ? prm->tol : 1e-10; }
int newton_max_iter(const dg_params* prm) { return prm->max_iter > 0 ? prm->max_iter : 50; }

}  // namespace

extern "C" dg_status dg_ns_rk_step(dg_mesh h, const dg_params* prm, double* q, double* T, double* work, double dt,
                                   double tol, int max_iter, hipStream_t stream) {
  if (!h) return fail(DG_ERR_ARG, "dg_ns_rk_step: null mesh");
  const Mesh& m = *reinterpret_cast<const Mesh*>(h);
  dg_status st = check("dg_ns_rk_step", m, prm);
  if (st != DG_OK) return st;
  if (!q || !T || !work || !aligned8(q) || !aligned8(T) || !aligned8(work))
    return fail(DG_ERR_ARG, "dg_ns_rk_step: null or misaligned pointer");
  if (!std::isfinite(dt)) return fail(DG_ERR_ARG, "dg_ns_rk_step: dt must be finite");
  if (!(tol > 0.0) || max_iter < 1) return fail(DG_ERR_ARG, "dg_ns_rk_step: need tol > 0 and max_iter >= 1");
  const size_t n = static_cast<size_t>(m.E) * m.Np;
  if (overlap(work, 58 * n, q, kFields * n) || overlap(work, 58 * n, T, n) || overlap(q, kFields * n, T, n))
    return fail(DG_ERR_ARG, "dg_ns_rk_step: q, T and work must not overlap");
  DeviceGuard g(m.device);
  if (!g.ok) return fail(DG_ERR_HIP, "dg_ns_rk_step: hipSetDevice failed");
  return ns_step(m, prm, q, T, true, work, dt, tol, max_iter, stream);
}

namespace dg {

// dg_rhs with model 1: Newton temperatures from 1000 K, lifted gradients and
// the right-hand side, all scratch in prm->work (DG_NS_RHS_WORK E Np doubles:
// T, Newton counts, gradients).
dg_status ns_rhs_model1(const Mesh& m, const dg_params* prm, const double* q, double* rhs, hipStream_t stream) {
  dg_status st = check("dg_rhs", m, prm);
  if (st != DG_OK) return st;
  const size_t n = static_cast<size_t>(m.E) * m.Np;
  double* w = prm->work;
  if (!w || !aligned8(w)) return fail(DG_ERR_ARG, "dg_rhs: model 1 needs params.work (35 E Np doubles)");
  if (overlap(w, DG_NS_RHS_WORK * n, q, kFields * n) || overlap(w, DG_NS_RHS_WORK * n, rhs, kFields * n) ||
      overlap(q, kFields * n, rhs, kFields * n))
    return fail(DG_ERR_ARG, "dg_rhs: q, rhs and params.work must not overlap");
  double* T = w;
  int32_t* iters = reinterpret_cast<int32_t*>(w + n);
  double* sigma = w + 2 * n;
  st = launch_temperature(thermo_table(prm->thermo), static_cast<int64_t>(n), q, nullptr, kTdefault, T, iters,
                          newton_tol(prm), newton_max_iter(prm), stream);
  if (st != DG_OK) return st;
  NsArgs A = make_args(m, prm);
  A.q = q;
  A.T = T;
  A.sigma = sigma;
  A.rhs = rhs;
  st = launch_ns_gradients(m.p, A, stream);
  if (st != DG_OK) return st;
  return launch_ns_rhs(m.p, A, false, stream);
}

// dg_rk_step with model 1: prm->work holds T (E Np) and the step scratch.
dg_status ns_step_model1(const Mesh& m, const dg_params* prm, double* q, double dt, hipStream_t stream) {
  dg_status st = check("dg_rk_step", m, prm);
  if (st != DG_OK) return st;
  const size_t n = static_cast<size_t>(m.E) * m.Np;
  double* w = prm->work;
  if (!w || !aligned8(w)) return fail(DG_ERR_ARG, "dg_rk_step: model 1 needs params.work (59 E Np doubles)");
  if (overlap(w, DG_NS_STEP_WORK * n, q, kFields * n))
    return fail(DG_ERR_ARG, "dg_rk_step: q and params.work must not overlap");
  return ns_step(m, prm, q, w, false, w + n, dt, newton_tol(prm), newton_max_iter(prm), stream);
}

}  // namespace dg
