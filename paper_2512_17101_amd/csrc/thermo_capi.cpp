// C-ABI of the reacting-flow pointwise kernels: species / mechanism handles,
// temperature Newton solve and Arrhenius sources.
#include <cmath>
#include <new>
#include <string>

#include "internal.hpp"
#include "thermo.hpp"

using namespace dg;

struct dg_thermo_s {
  int device;
  ThermoTable t;
};
struct dg_mech_s {
  int device;
  MechTable m;
};

namespace {
bool aligned8(const void* p) { return (reinterpret_cast<uintptr_t>(p) & 7u) == 0; }
bool aligned4(const void* p) { return (reinterpret_cast<uintptr_t>(p) & 3u) == 0; }
}  // namespace

extern "C" dg_status dg_thermo_create(int n_species, const double* W, const double* coeffs, int device,
                                      dg_thermo* out) {
  if (!out) return fail(DG_ERR_ARG, "dg_thermo_create: out is NULL");
  *out = nullptr;
  if (n_species < 1 || n_species > kMaxSpecies) return fail(DG_ERR_ARG, "dg_thermo_create: n_species must be 1..8");
  if (!W || !coeffs) return fail(DG_ERR_ARG, "dg_thermo_create: null table");
  int ndev = 0;
  if (hipGetDeviceCount(&ndev) != hipSuccess || device < 0 || device >= ndev)
    return fail(DG_ERR_ARG, "dg_thermo_create: invalid device");
  dg_thermo_s* h = new (std::nothrow) dg_thermo_s();
  if (!h) return fail(DG_ERR_ALLOC, "dg_thermo_create: allocation failed");
  h->device = device;
  h->t.ns = n_species;
  for (int k = 0; k < n_species; ++k) {
    if (!(W[k] > 0.0) || !std::isfinite(W[k])) {
      delete h;
      return fail(DG_ERR_ARG, "dg_thermo_create: molar masses must be positive");
    }
    const double* a = coeffs + 6 * k;
    h->t.W[k] = W[k];
    h->t.R[k] = kRu / W[k];
    for (int m = 0; m < 5; ++m) {
      h->t.cp[k][m] = a[m];
      h->t.h[k][m] = a[m] / (m + 1);
    }
    h->t.h[k][5] = a[5];
  }
  *out = h;
  return DG_OK;
}

extern "C" dg_status dg_thermo_destroy(dg_thermo th) {
  delete th;
  return DG_OK;
}

extern "C" dg_status dg_mech_create(dg_thermo th, int n_reactions, const double* A, const double* Ea,
                                    const int32_t* nu_r, const int32_t* nu_p, dg_mech* out) {
  if (!out) return fail(DG_ERR_ARG, "dg_mech_create: out is NULL");
  *out = nullptr;
  if (!th) return fail(DG_ERR_ARG, "dg_mech_create: null thermo");
  if (n_reactions < 1 || n_reactions > kMaxReactions) return fail(DG_ERR_ARG, "dg_mech_create: n_reactions must be 1..8");
  if (!A || !Ea || !nu_r || !nu_p) return fail(DG_ERR_ARG, "dg_mech_create: null table");
  dg_mech_s* h = new (std::nothrow) dg_mech_s();
  if (!h) return fail(DG_ERR_ALLOC, "dg_mech_create: allocation failed");
  const int ns = th->t.ns;
  h->device = th->device;
  h->m.ns = ns;
  h->m.nr = n_reactions;
  for (int k = 0; k < ns; ++k) h->m.invW[k] = 1.0 / th->t.W[k];
  for (int j = 0; j < n_reactions; ++j) {
    if (!(A[j] >= 0.0) || !std::isfinite(A[j]) || !std::isfinite(Ea[j])) {
      delete h;
      return fail(DG_ERR_ARG, "dg_mech_create: A must be >= 0 and finite, Ea finite");
    }
    h->m.A[j] = A[j];
    h->m.EaR[j] = Ea[j] / kRu;
    for (int k = 0; k < ns; ++k) {
      const int r = nu_r[j * ns + k], p = nu_p[j * ns + k];
      if (r < 0 || r > 3 || p < 0 || p > 3) {
        delete h;
        return fail(DG_ERR_ARG, "dg_mech_create: stoichiometric coefficients must be integers in 0..3");
      }
      h->m.nu_r[j][k] = r;
      h->m.Wnet[k][j] = th->t.W[k] * (p - r);
    }
  }
  *out = h;
  return DG_OK;
}

extern "C" dg_status dg_mech_destroy(dg_mech m) {
  delete m;
  return DG_OK;
}

extern "C" dg_status dg_temperature(int64_t n, const double* q, const double* T_guess, double* T_out,
                                    int32_t* iters, dg_thermo th, double tol, int max_iter, const dg_mlp_s* guess,
                                    hipStream_t stream) {
  if (!th) return fail(DG_ERR_ARG, "dg_temperature: null thermo");
  if (n < 0) return fail(DG_ERR_ARG, "dg_temperature: negative size");
  if (guess) {
    if (T_guess) return fail(DG_ERR_ARG, "dg_temperature: T_guess must be NULL when a learned guess is given");
    return dg_temperature_learned(th, const_cast<dg_mlp>(guess), n, q, kTdefault, T_out, iters, tol, max_iter,
                                  kLearnedMaxIter, nullptr, stream);
  }
  if (n == 0) return DG_OK;
  if (!q || !T_out || !iters || !aligned8(q) || !aligned8(T_out) || !aligned4(iters) ||
      (T_guess && !aligned8(T_guess)))
    return fail(DG_ERR_ARG, "dg_temperature: null or misaligned pointer");
  if (!(tol > 0.0) || max_iter < 1) return fail(DG_ERR_ARG, "dg_temperature: tol must be > 0 and max_iter >= 1");
  DeviceGuard g(th->device);
  if (!g.ok) return fail(DG_ERR_HIP, "dg_temperature: hipSetDevice failed");
  return launch_temperature(th->t, n, q, T_guess, kTdefault, T_out, iters, tol, max_iter, stream);
}

extern "C" dg_status dg_sources(int64_t n, const double* q, const double* T, double* omega, dg_mech mech,
                                hipStream_t stream) {
  if (!mech) return fail(DG_ERR_ARG, "dg_sources: null mechanism");
  if (n < 0) return fail(DG_ERR_ARG, "dg_sources: negative size");
  if (n == 0) return DG_OK;
  if (!q || !T || !omega || !aligned8(q) || !aligned8(T) || !aligned8(omega))
    return fail(DG_ERR_ARG, "dg_sources: null or misaligned pointer");
  DeviceGuard g(mech->device);
  if (!g.ok) return fail(DG_ERR_HIP, "dg_sources: hipSetDevice failed");
  return launch_sources(mech->m, n, q, T, omega, stream);
}

namespace dg {
const ThermoTable& thermo_table(const dg_thermo_s* th) { return th->t; }
const MechTable& mech_table(const dg_mech_s* mk) { return mk->m; }
int mech_device(const dg_mech_s* mk) { return mk->device; }
int thermo_device(const dg_thermo_s* th) { return th->device; }
}  // namespace dg
