// C-ABI of the learned temperature guess: network handle, parameters,
// normalisation, gradients, Adam training step, prediction and the Newton
// solve started from the prediction.
#include <cmath>
#include <cstring>
#include <new>
#include <random>
#include <string>
#include <vector>

#include "internal.hpp"
#include "mlp.hpp"

using namespace dg;

struct dg_thermo_s;  // defined with the thermo entry points
struct dg_mlp_s {
  int device = 0;
  float* master = nullptr;
  float* m = nullptr;
  float* v = nullptr;
  float* grad = nullptr;
  float* loss = nullptr;
  uint16_t* fwd = nullptr;
  uint16_t* bwd = nullptr;
  int32_t* src = nullptr;  // [(kFwdTiles + kBwdTiles) * 512] source index of every BF16 operand entry
  uint16_t* H = nullptr;   // scratch [4][64][cap]
  float* D = nullptr;      // scratch [4][64][cap]
  int64_t cap = 0;
  int64_t step = 0;        // Adam steps taken
  MlpNorm norm{};
};

namespace dg {
const ThermoTable& thermo_table(const dg_thermo_s* th);
int thermo_device(const dg_thermo_s* th);
}  // namespace dg

namespace {

bool aligned8(const void* p) { return (reinterpret_cast<uintptr_t>(p) & 7u) == 0; }

std::vector<int32_t> operand_sources() {
  std::vector<int32_t> s((kFwdTiles + kBwdTiles) * kTileElems, -1);
  for (int l = 0; l < 64; ++l)
    for (int e = 0; e < 8; ++e) {
      const int il = l % 16, g = l / 16;
      for (int rb = 0; rb < 4; ++rb) {
        const int i = 16 * rb + il;
        const int k1 = 8 * g + e;
        s[((kFwdT1 + rb) * 64 + l) * 8 + e] = k1 < kMlpIn ? kOffW1 + i * kMlpIn + k1 : -1;
        for (int ks = 0; ks < 2; ++ks) {
          const int k = hidden_unit_of_slot(ks, g, e);
          s[((kFwdT2 + rb * 2 + ks) * 64 + l) * 8 + e] = kOffW2 + i * 64 + k;
          s[((kFwdT3 + rb * 2 + ks) * 64 + l) * 8 + e] = kOffW3 + i * 64 + k;
          // transposed: rows = units of the lower layer, K = units of the upper layer
          s[((kFwdTiles + kBwdT2 + rb * 2 + ks) * 64 + l) * 8 + e] = kOffW2 + k * 64 + i;
          s[((kFwdTiles + kBwdT3 + rb * 2 + ks) * 64 + l) * 8 + e] = kOffW3 + k * 64 + i;
        }
      }
      for (int ks = 0; ks < 2; ++ks)
        s[((kFwdT4 + ks) * 64 + l) * 8 + e] = il == 0 ? kOffW4 + hidden_unit_of_slot(ks, g, e) : -1;
    }
  return s;
}

MlpView view_of(const dg_mlp_s* h) {
  MlpView v;
  v.master = h->master;
  v.fwd = h->fwd;
  v.bwd = h->bwd;
  v.norm = h->norm;
  return v;
}

struct DeviceScope {
  int prev = 0;
  bool ok;
  explicit DeviceScope(int d) { hipGetDevice(&prev); ok = hipSetDevice(d) == hipSuccess; }
  ~DeviceScope() { hipSetDevice(prev); }
};

dg_status regenerate_layouts(dg_mlp_s* h, hipStream_t s) {
  dg_status st = launch_mlp_layouts(h->master, h->src, h->fwd, static_cast<int64_t>(kFwdTiles) * kTileElems, s);
  if (st != DG_OK) return st;
  return launch_mlp_layouts(h->master, h->src + kFwdTiles * kTileElems, h->bwd,
                            static_cast<int64_t>(kBwdTiles) * kTileElems, s);
}

dg_status ensure_scratch(dg_mlp_s* h, int64_t bpad) {
  if (bpad <= h->cap) return DG_OK;
  hipFree(h->H);
  hipFree(h->D);
  h->H = nullptr;
  h->D = nullptr;
  h->cap = 0;
  const size_t nh = static_cast<size_t>(4) * 64 * bpad;
  if (hipMalloc(&h->H, nh * sizeof(uint16_t)) != hipSuccess || hipMalloc(&h->D, nh * sizeof(float)) != hipSuccess)
    return fail(DG_ERR_ALLOC, "mlp: scratch allocation failed");
  // rows that are never written (feature padding, output-delta padding) must read as zero
  DG_HIP(hipMemset(h->H, 0, nh * sizeof(uint16_t)));
  DG_HIP(hipMemset(h->D, 0, nh * sizeof(float)));
  h->cap = bpad;
  return DG_OK;
}

dg_status check_batch(const char* who, int64_t batch, int64_t ld, const double* q, const int64_t* idx,
                      const double* T) {
  if (batch < 1 || ld < 1) return fail(DG_ERR_ARG, std::string(who) + ": batch and ld must be >= 1");
  if (!q || !idx || !T || !aligned8(q) || !aligned8(idx) || !aligned8(T))
    return fail(DG_ERR_ARG, std::string(who) + ": null or misaligned pointer");
  return DG_OK;
}

}  // namespace

extern "C" dg_status dg_mlp_create(int device, uint64_t seed, dg_mlp* out) {
  if (!out) return fail(DG_ERR_ARG, "dg_mlp_create: out is NULL");
  *out = nullptr;
  int ndev = 0;
  if (hipGetDeviceCount(&ndev) != hipSuccess || device < 0 || device >= ndev)
    return fail(DG_ERR_ARG, "dg_mlp_create: invalid device");
  DeviceScope ds(device);
  dg_mlp_s* h = new (std::nothrow) dg_mlp_s();
  if (!h) return fail(DG_ERR_ALLOC, "dg_mlp_create: allocation failed");
  h->device = device;
  for (int k = 0; k < kMlpIn; ++k) { h->norm.mean[k] = 0.0; h->norm.inv_std[k] = 1.0; }
  h->norm.T_mean = 0.0;
  h->norm.T_std = 1.0;
  bool ok = hipMalloc(&h->master, kMlpParams * 4) == hipSuccess && hipMalloc(&h->m, kMlpParams * 4) == hipSuccess &&
            hipMalloc(&h->v, kMlpParams * 4) == hipSuccess && hipMalloc(&h->grad, kMlpParams * 4) == hipSuccess &&
            hipMalloc(&h->loss, 4) == hipSuccess &&
            hipMalloc(&h->fwd, kFwdTiles * kTileElems * 2) == hipSuccess &&
            hipMalloc(&h->bwd, kBwdTiles * kTileElems * 2) == hipSuccess &&
            hipMalloc(&h->src, (kFwdTiles + kBwdTiles) * kTileElems * 4) == hipSuccess;
  if (!ok) { dg_mlp_destroy(h); return fail(DG_ERR_ALLOC, "dg_mlp_create: device allocation failed"); }
  // Glorot-uniform weights, zero biases
  std::vector<float> p(kMlpParams, 0.f);
  std::mt19937_64 rng(seed);
  const int fi[4] = {kMlpIn, 64, 64, 64}, fo[4] = {64, 64, 64, 1}, off[4] = {kOffW1, kOffW2, kOffW3, kOffW4};
  for (int l = 0; l < 4; ++l) {
    std::uniform_real_distribution<double> U(-std::sqrt(6.0 / (fi[l] + fo[l])), std::sqrt(6.0 / (fi[l] + fo[l])));
    for (int i = 0; i < fi[l] * fo[l]; ++i) p[off[l] + i] = static_cast<float>(U(rng));
  }
  const std::vector<int32_t> src = operand_sources();
  dg_status st = DG_OK;
  if (hipMemcpy(h->src, src.data(), src.size() * 4, hipMemcpyHostToDevice) != hipSuccess) st = DG_ERR_HIP;
  if (st == DG_OK) st = dg_mlp_set_params(h, p.data());
  if (st != DG_OK) { dg_mlp_destroy(h); return st == DG_ERR_HIP ? fail(st, "dg_mlp_create: copy failed") : st; }
  *out = h;
  return DG_OK;
}

extern "C" dg_status dg_mlp_destroy(dg_mlp h) {
  if (!h) return DG_OK;
  DeviceScope ds(h->device);
  hipFree(h->master); hipFree(h->m); hipFree(h->v); hipFree(h->grad); hipFree(h->loss);
  hipFree(h->fwd); hipFree(h->bwd); hipFree(h->src); hipFree(h->H); hipFree(h->D);
  delete h;
  return DG_OK;
}

extern "C" dg_status dg_mlp_set_params(dg_mlp h, const float* params) {
  if (!h || !params) return fail(DG_ERR_ARG, "dg_mlp_set_params: null argument");
  DeviceScope ds(h->device);
  DG_HIP(hipMemcpy(h->master, params, kMlpParams * 4, hipMemcpyHostToDevice));
  DG_HIP(hipMemset(h->m, 0, kMlpParams * 4));
  DG_HIP(hipMemset(h->v, 0, kMlpParams * 4));
  h->step = 0;
  dg_status st = regenerate_layouts(h, nullptr);
  if (st != DG_OK) return st;
  DG_HIP(hipDeviceSynchronize());
  return DG_OK;
}

extern "C" dg_status dg_mlp_get_params(dg_mlp h, float* params) {
  if (!h || !params) return fail(DG_ERR_ARG, "dg_mlp_get_params: null argument");
  DeviceScope ds(h->device);
  DG_HIP(hipDeviceSynchronize());
  DG_HIP(hipMemcpy(params, h->master, kMlpParams * 4, hipMemcpyDeviceToHost));
  return DG_OK;
}

extern "C" dg_status dg_mlp_set_normalization(dg_mlp h, const double* feat_mean, const double* feat_std, double T_mean,
                                              double T_std) {
  if (!h || !feat_mean || !feat_std) return fail(DG_ERR_ARG, "dg_mlp_set_normalization: null argument");
  for (int k = 0; k < kMlpIn; ++k)
    if (!(feat_std[k] > 0.0) || !std::isfinite(feat_mean[k])) return fail(DG_ERR_ARG, "dg_mlp_set_normalization: std must be > 0");
  if (!(T_std > 0.0) || !std::isfinite(T_mean)) return fail(DG_ERR_ARG, "dg_mlp_set_normalization: T_std must be > 0");
  for (int k = 0; k < kMlpIn; ++k) { h->norm.mean[k] = feat_mean[k]; h->norm.inv_std[k] = 1.0 / feat_std[k]; }
  h->norm.T_mean = T_mean;
  h->norm.T_std = T_std;
  return DG_OK;
}

extern "C" dg_status dg_mlp_get_normalization(dg_mlp h, double* feat_mean, double* feat_std, double* T_mean,
                                              double* T_std) {
  if (!h) return fail(DG_ERR_ARG, "dg_mlp_get_normalization: null handle");
  for (int k = 0; k < kMlpIn; ++k) {
    if (feat_mean) feat_mean[k] = h->norm.mean[k];
    if (feat_std) feat_std[k] = 1.0 / h->norm.inv_std[k];
  }
  if (T_mean) *T_mean = h->norm.T_mean;
  if (T_std) *T_std = h->norm.T_std;
  return DG_OK;
}

extern "C" dg_status dg_mlp_fit_normalization(dg_mlp h, int64_t n, int64_t ld, const double* q, const int64_t* idx,
                                              const double* T) {
  if (!h) return fail(DG_ERR_ARG, "dg_mlp_fit_normalization: null handle");
  if (n < 2) return fail(DG_ERR_ARG, "dg_mlp_fit_normalization: need at least 2 samples");
  dg_status st = check_batch("dg_mlp_fit_normalization", n, ld, q, idx, T);
  if (st != DG_OK) return st;
  DeviceScope ds(h->device);
  double* acc = nullptr;
  if (hipMalloc(&acc, 20 * sizeof(double)) != hipSuccess) return fail(DG_ERR_ALLOC, "dg_mlp_fit_normalization: allocation failed");
  double host[20];
  st = DG_OK;
  if (hipMemset(acc, 0, 20 * sizeof(double)) != hipSuccess) st = fail(DG_ERR_HIP, "dg_mlp_fit_normalization: memset failed");
  if (st == DG_OK) st = launch_mlp_moments(n, ld, q, idx, T, acc, nullptr);
  if (st == DG_OK && hipMemcpy(host, acc, sizeof(host), hipMemcpyDeviceToHost) != hipSuccess)
    st = fail(DG_ERR_HIP, "dg_mlp_fit_normalization: copy failed");
  hipFree(acc);
  if (st != DG_OK) return st;
  double mean[10], sd[10];
  for (int k = 0; k < 10; ++k) {
    mean[k] = host[k] / n;
    const double var = host[10 + k] / n - mean[k] * mean[k];
    sd[k] = std::sqrt(var > 0.0 ? var : 0.0);
    // a (numerically) constant feature is centred but not scaled
    if (!(sd[k] >= 1e-6 * std::fmax(std::fabs(mean[k]), 1.0))) sd[k] = 1.0;
  }
  return dg_mlp_set_normalization(h, mean, sd, mean[9], sd[9]);
}

extern "C" dg_status dg_mlp_loss_grad(dg_mlp h, int64_t batch, int64_t ld, const double* q, const int64_t* idx,
                                      const double* T, float* grad_out, float* loss_out, hipStream_t s) {
  if (!h) return fail(DG_ERR_ARG, "dg_mlp_loss_grad: null handle");
  dg_status st = check_batch("dg_mlp_loss_grad", batch, ld, q, idx, T);
  if (st != DG_OK) return st;
  DeviceScope ds(h->device);
  const int64_t bpad = (batch + 31) / 32 * 32;
  st = ensure_scratch(h, bpad);
  if (st != DG_OK) return st;
  st = launch_mlp_zero(h->loss, 1, s);  // a kernel, not a memset node, should the caller capture this
  if (st != DG_OK) return st;
  st = launch_mlp_forward_backward(view_of(h), batch, bpad, ld, q, idx, T, h->H, h->D, h->loss, s);
  if (st != DG_OK) return st;
  st = launch_mlp_weight_grads(bpad, h->H, h->D, h->grad, s);
  if (st != DG_OK) return st;
  if (grad_out) DG_HIP(hipMemcpyAsync(grad_out, h->grad, kMlpParams * 4, hipMemcpyDeviceToDevice, s));
  if (loss_out) DG_HIP(hipMemcpyAsync(loss_out, h->loss, 4, hipMemcpyDeviceToDevice, s));
  return DG_OK;
}

extern "C" dg_status dg_mlp_train_step(dg_mlp h, int64_t batch, int64_t ld, const double* q, const int64_t* idx,
                                       const double* T, float lr, float* loss_out, hipStream_t s) {
  if (!h) return fail(DG_ERR_ARG, "dg_mlp_train_step: null handle");
  if (!(lr > 0.f) || !std::isfinite(lr)) return fail(DG_ERR_ARG, "dg_mlp_train_step: lr must be > 0");
  dg_status st = dg_mlp_loss_grad(h, batch, ld, q, idx, T, nullptr, loss_out, s);
  if (st != DG_OK) return st;
  DeviceScope ds(h->device);
  h->step += 1;
  const float b1 = 0.9f, b2 = 0.999f, eps = 1e-8f;
  const float c1 = static_cast<float>(1.0 - std::pow(0.9, static_cast<double>(h->step)));
  const float c2 = static_cast<float>(1.0 - std::pow(0.999, static_cast<double>(h->step)));
  st = launch_mlp_adam(h->master, h->m, h->v, h->grad, lr, b1, b2, eps, c1, c2, s);
  if (st != DG_OK) return st;
  return regenerate_layouts(h, s);
}

extern "C" dg_status dg_mlp_predict(dg_mlp h, int64_t n, int64_t ld, const double* q, double* T_pred, hipStream_t s) {
  if (!h) return fail(DG_ERR_ARG, "dg_mlp_predict: null handle");
  if (n < 0 || ld < n) return fail(DG_ERR_ARG, "dg_mlp_predict: need 0 <= n <= ld");
  if (n == 0) return DG_OK;
  if (!q || !T_pred || !aligned8(q) || !aligned8(T_pred)) return fail(DG_ERR_ARG, "dg_mlp_predict: null or misaligned pointer");
  DeviceScope ds(h->device);
  return launch_mlp_predict(view_of(h), n, ld, q, T_pred, s);
}

extern "C" dg_status dg_temperature_learned(dg_thermo th, dg_mlp h, int64_t n, const double* q, double T_default,
                                            double* T_out, int32_t* iters, double tol, int max_iter,
                                            int learned_max_iter, int32_t* fallback_count, hipStream_t s) {
  if (!th || !h) return fail(DG_ERR_ARG, "dg_temperature_learned: null handle");
  if (n < 0) return fail(DG_ERR_ARG, "dg_temperature_learned: negative size");
  if (n == 0) return DG_OK;
  if (thermo_table(th).ns != 7) return fail(DG_ERR_ARG, "dg_temperature_learned: the network takes 7 species");
  if (!q || !T_out || !iters || !aligned8(q) || !aligned8(T_out))
    return fail(DG_ERR_ARG, "dg_temperature_learned: null or misaligned pointer");
  if (!(tol > 0.0) || max_iter < 1 || learned_max_iter < 1)
    return fail(DG_ERR_ARG, "dg_temperature_learned: tol > 0, max_iter >= 1, learned_max_iter >= 1 required");
  if (!(T_default >= kTmin && T_default <= kTmax)) return fail(DG_ERR_ARG, "dg_temperature_learned: T_default out of range");
  DeviceScope ds(h->device);
  return launch_temperature_learned(thermo_table(th), view_of(h), n, q, T_default, T_out, iters, tol, max_iter,
                                    learned_max_iter, fallback_count, s);
}
