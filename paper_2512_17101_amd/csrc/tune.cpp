// C-ABI of a single mesh's launch configuration and its autotuner.
#include <cmath>
#include <cstdio>
#include <map>
#include <string>
#include <vector>

#include "internal.hpp"
#include "json_cache.hpp"

using namespace dg;

namespace {

bool valid_prec(dg_precision p) { return p == DG_FP64 || p == DG_FP32 || p == DG_SPLIT_BF16; }

// a cached field that converts to int without overflow (0 .. 64 covers
// every valid value; anything else is rejected before the conversion)
bool in_int_range(double v) { return v >= 0.0 && v <= 64.0; }

bool valid_launch(const dg_launch_config& c) {
  return (c.waves_per_block == 2 || c.waves_per_block == 4) && (c.rk_fused == 0 || c.rk_fused == 1) &&
         (c.lds_stage == 0 || c.lds_stage == 1) && c.xcd_run >= 1 && c.xcd_run <= 64;
}

const char* prec_name(dg_precision p) { return p == DG_FP64 ? "fp64" : p == DG_FP32 ? "fp32" : "split_bf16"; }

}  // namespace

extern "C" dg_status dg_mesh_set_launch(dg_mesh h, dg_precision prec, const dg_launch_config* cfg) {
  if (!h || !cfg) return fail(DG_ERR_ARG, "dg_mesh_set_launch: null argument");
  if (!valid_prec(prec)) return fail(DG_ERR_ARG, "dg_mesh_set_launch: unknown precision");
  if (!valid_launch(*cfg))
    return fail(DG_ERR_ARG,
                "dg_mesh_set_launch: waves_per_block must be 2 or 4, rk_fused and lds_stage 0 or 1, xcd_run 1..64");
  reinterpret_cast<Mesh*>(h)->launch[prec] = *cfg;
  return DG_OK;
}

extern "C" dg_status dg_mesh_get_launch(dg_mesh h, dg_precision prec, dg_launch_config* cfg) {
  if (!h || !cfg) return fail(DG_ERR_ARG, "dg_mesh_get_launch: null argument");
  if (!valid_prec(prec)) return fail(DG_ERR_ARG, "dg_mesh_get_launch: unknown precision");
  *cfg = reinterpret_cast<const Mesh*>(h)->launch[prec];
  return DG_OK;
}

extern "C" dg_status dg_autotune(dg_mesh h, const dg_params* prm, dg_precision prec, const char* cache_path,
                                 int trials, dg_launch_config* chosen, double* best_ms, hipStream_t stream) {
  if (!h || !prm) return fail(DG_ERR_ARG, "dg_autotune: null argument");
  if (!valid_prec(prec)) return fail(DG_ERR_ARG, "dg_autotune: unknown precision");
  if (prm->model != 0 || !(prm->gamma > 1.0) || !std::isfinite(prm->gamma))
    return fail(DG_ERR_ARG, "dg_autotune: Euler model with gamma > 1 required");
  if (trials < 1 || trials > 1000) return fail(DG_ERR_ARG, "dg_autotune: trials must be in 1..1000");
  Mesh& m = *reinterpret_cast<Mesh*>(h);
  DeviceGuard g(m.device);
  if (!g.ok) return fail(DG_ERR_HIP, "dg_autotune: hipSetDevice failed");
  char key[256];
  std::snprintf(key, sizeof key, "%s:%s:p%d:E%lld", device_key(m.device).c_str(), prec_name(prec), m.p,
                static_cast<long long>(m.E));
  std::map<std::string, std::string> cache;
  if (cache_path) {
    cache = read_cache(cache_path);
    const auto it = cache.find(key);
    double w, f, l, x;
    if (it != cache.end() && cache_field(it->second, "waves_per_block", w) && cache_field(it->second, "rk_fused", f) &&
        cache_field(it->second, "lds_stage", l) && cache_field(it->second, "xcd_run", x) &&
        in_int_range(w) && in_int_range(f) && in_int_range(l) && in_int_range(x)) {
      const dg_launch_config c{static_cast<int>(w), static_cast<int>(f), static_cast<int>(l), static_cast<int>(x)};
      if (valid_launch(c)) {
        m.launch[prec] = c;
        if (chosen) *chosen = c;
        if (best_ms) *best_ms = -1.0;
        return DG_OK;
      }
    }
  }

  // a uniform state (rho = 1, u = 0, p = 1) in temporary buffers: the kernels'
  // work does not depend on the values
  const int64_t nn = m.E * m.Np;
  const size_t n = static_cast<size_t>(5) * nn;
  double* buf = nullptr;
  if (hipMalloc(&buf, 3 * n * sizeof(double)) != hipSuccess)
    return fail(DG_ERR_ALLOC, "dg_autotune: no room for the temporary state");
  struct Free {
    double* p;
    ~Free() { hipFree(p); }
  } free_buf{buf};
  const double v[5] = {1.0, 0.0, 0.0, 0.0, 1.0 / (prm->gamma - 1.0)};
  dg_status st = launch_fill_state(buf, nn, v, stream);
  if (st != DG_OK) return st;
  hipEvent_t e0, e1;
  DG_HIP(hipEventCreate(&e0));
  DG_HIP(hipEventCreate(&e1));
  struct Ev {
    hipEvent_t a, b;
    ~Ev() {
      hipEventDestroy(a);
      hipEventDestroy(b);
    }
  } ev{e0, e1};

  // tiles per block x fused stages x LDS staging path (only where the
  // direct global-to-LDS staging exists: FP64 / FP32 with Np % 4 == 0) x
  // XCD run length (9 and 27 blocks were the good runs measured on box
  // meshes, 1 is the plain order)
  const bool has_dma = m.Np % 4 == 0 && prec != DG_SPLIT_BF16;
  std::vector<dg_launch_config> cands;
  for (int w : {4, 2}) {
    if (w == 4 && m.p >= 4) continue;  // runs as 2
    for (int f : {1, 0})
      for (int l : {1, 0}) {
        if (l == 0 && !has_dma) continue;  // the same kernel as l = 1
        for (int x : {1, 9, 27}) cands.push_back(dg_launch_config{w, f, l, x});
      }
  }
  const dg_launch_config prev = m.launch[prec];
  dg_launch_config best = prev;
  double best_t = -1.0;
  const double dt = 1e-3;
  for (const dg_launch_config& c : cands) {
    m.launch[prec] = c;
    st = dg_rk_step(h, prm, prec, buf, buf + n, 0.0, dt, stream);  // warm-up
    if (st != DG_OK) break;
    if (hipEventRecord(e0, stream) != hipSuccess) {
      st = fail(DG_ERR_HIP, "dg_autotune: hipEventRecord failed");
      break;
    }
    for (int t = 0; t < trials && st == DG_OK; ++t) st = dg_rk_step(h, prm, prec, buf, buf + n, 0.0, dt, stream);
    if (st != DG_OK) break;
    float ms = 0.f;
    if (hipEventRecord(e1, stream) != hipSuccess || hipEventSynchronize(e1) != hipSuccess ||
        hipEventElapsedTime(&ms, e0, e1) != hipSuccess) {
      st = fail(DG_ERR_HIP, "dg_autotune: event timing failed");
      break;
    }
    const double per = static_cast<double>(ms) / trials;
    if (best_t < 0.0 || per < best_t) {
      best_t = per;
      best = c;
    }
  }
  const hipError_t es = hipStreamSynchronize(stream);  // before the buffers are freed
  if (st == DG_OK && es != hipSuccess) st = hip_fail(es, "dg_autotune");
  if (st != DG_OK) {
    m.launch[prec] = prev;
    return st;
  }
  m.launch[prec] = best;
  if (chosen) *chosen = best;
  if (best_ms) *best_ms = best_t;
  if (cache_path) {
    char obj[224];
    std::snprintf(obj, sizeof obj,
                  "{\"waves_per_block\": %d, \"rk_fused\": %d, \"lds_stage\": %d, \"xcd_run\": %d, \"ms\": %.6g}",
                  best.waves_per_block, best.rk_fused, best.lds_stage, best.xcd_run, best_t);
    cache[key] = obj;
    if (!write_cache(cache_path, cache))
      return fail(DG_ERR_ARG, std::string("dg_autotune: cannot write cache file ") + cache_path);
  }
  return DG_OK;
}
