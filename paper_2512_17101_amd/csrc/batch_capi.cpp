// C-ABI of batched stepping: work lists, binding, graph capture / replay and
// the launch-shape autotuner with its JSON cache.
#include <algorithm>
#include <cmath>
#include <cstdio>
#include <fstream>
#include <map>
#include <memory>
#include <sstream>
#include <string>
#include <vector>

#include "batch.hpp"
#include "internal.hpp"
#include "json_cache.hpp"

using namespace dg;

namespace {

constexpr int kMaxBlocksPerCu = 4;
constexpr int kXcds = 8;

}  // namespace

struct dg_batch_s {
  int device = 0;
  dg_precision prec = DG_FP32;
  int n = 0;
  int cus = 256;
  std::string arch;
  std::vector<const Mesh*> meshes;
  BatchTables tabs{};
  int64_t n_items = 0, n_elem = 0;
  BatchMesh* d_meshes = nullptr;
  BatchItem* d_items[2] = {nullptr, nullptr};  // by dg_batch_config::order
  std::vector<BatchMesh> host_meshes;
  int64_t p_begin[5] = {0, 0, 0, 0, 0}, p_end[5] = {0, 0, 0, 0, 0};  // in list 0 (grouped by order)
  const double* dt = nullptr;
  bool bound = false;
  dg_batch_config cfg{4, 2, 0, 0, 1};
  hipStream_t cap_stream = nullptr;
  hipStream_t side[3] = {nullptr, nullptr, nullptr};  // per-order chains after the first
  hipEvent_t fork_ev = nullptr, join_ev[3] = {nullptr, nullptr, nullptr};
  hipGraph_t graph = nullptr;
  hipGraphExec_t exec = nullptr;
  double graph_gamma = 0.0;
  dg_batch_config graph_cfg{};

  void drop_graph() {
    if (exec) hipGraphExecDestroy(exec);
    if (graph) hipGraphDestroy(graph);
    exec = nullptr;
    graph = nullptr;
  }
  ~dg_batch_s() {
    drop_graph();
    if (cap_stream) hipStreamDestroy(cap_stream);
    for (hipStream_t x : side)
      if (x) hipStreamDestroy(x);
    if (fork_ev) hipEventDestroy(fork_ev);
    for (hipEvent_t e : join_ev)
      if (e) hipEventDestroy(e);
    hipFree(d_meshes);
    hipFree(d_items[0]);
    hipFree(d_items[1]);
  }
};

namespace {

bool aligned8(const void* p) { return (reinterpret_cast<uintptr_t>(p) & 7u) == 0; }

bool valid_config(const dg_batch_config& c) {
  return (c.waves_per_block == 2 || c.waves_per_block == 4 || c.waves_per_block == 8) && c.blocks_per_cu >= 1 &&
         c.blocks_per_cu <= kMaxBlocksPerCu && (c.order == 0 || c.order == 1) &&
         (c.xcd_chunks == 0 || c.xcd_chunks == 1) && c.per_order >= 0 && c.per_order <= 2;
}

// Resolves a configuration into a launch: grid size from the CU count, the
// blocks per CU (capped by occupancy) and the number of items.
dg_status make_launch(const dg_batch_s& b, const dg_batch_config& c, double gamma, BatchLaunch& L) {
  const int occ = batch_stage_occupancy(b.prec, c.waves_per_block, b.tabs.lds_bytes);
  if (occ < 1) return fail(DG_ERR_HIP, "dg_batch: stage kernel cannot be resident with this shape");
  const int bpc = std::min(c.blocks_per_cu, occ);
  int64_t blocks = static_cast<int64_t>(bpc) * b.cus;
  const int64_t needed = (b.n_items + c.waves_per_block - 1) / c.waves_per_block;
  if (blocks > needed) blocks = needed;
  if (c.xcd_chunks) blocks = std::max<int64_t>(kXcds, (blocks + kXcds - 1) / kXcds * kXcds);
  if (blocks < 1) blocks = 1;
  L.meshes = b.d_meshes;
  L.items = b.d_items[c.per_order ? 0 : c.order];
  L.n_items = b.n_items;
  for (int p = 0; p < 5; ++p) {
    L.p_begin[p] = b.p_begin[p];
    L.p_end[p] = b.p_end[p];
  }
  L.dt = b.dt;
  L.gamma = gamma;
  L.flags = device_flags();
  L.tabs = b.tabs;
  L.waves_per_block = c.waves_per_block;
  L.blocks = static_cast<int>(blocks);
  L.xcd_chunks = c.xcd_chunks;
  return DG_OK;
}

// The launches of one step: five fused stages (q -> tmp -> q ... ending in
// tmp) and the copy back to q.  In the per-order modes each stage is one
// launch per order present: with per_order == 1 each order's chain of five
// stages and its copy runs on a stream of its own (the first on s, the others
// on the batch's side streams, forked from s and joined back into it); with
// per_order == 2 everything runs on s, stage by stage, and one copy follows.
dg_status enqueue_step(const dg_batch_s& b, const dg_batch_config& c, double gamma, hipStream_t s) {
  BatchLaunch L;
  dg_status st = make_launch(b, c, gamma, L);
  if (st != DG_OK) return st;
  if (!c.per_order) {
    for (int k = 0; k < 5; ++k) {
      st = launch_batch_stage(b.prec, L, kLsrkA[k], kLsrkB[k], k & 1, s);
      if (st != DG_OK) return st;
    }
    return launch_batch_copy(L, 0, L.n_items, s);
  }
  std::vector<int> orders;
  for (int p = 4; p >= 1; --p)
    if (b.p_end[p] > b.p_begin[p]) orders.push_back(p);
  if (c.per_order == 2) {
    for (int k = 0; k < 5; ++k)
      for (int p : orders) {
        st = launch_batch_order_stage(b.prec, L, p, kLsrkA[k], kLsrkB[k], k & 1, s);
        if (st != DG_OK) return st;
      }
    return launch_batch_copy(L, 0, L.n_items, s);
  }
  if (orders.size() > 1) {
    DG_HIP(hipEventRecord(b.fork_ev, s));
    for (size_t j = 1; j < orders.size(); ++j) DG_HIP(hipStreamWaitEvent(b.side[j - 1], b.fork_ev, 0));
  }
  for (size_t j = 0; j < orders.size(); ++j) {
    const int p = orders[j];
    hipStream_t sj = j == 0 ? s : b.side[j - 1];
    for (int k = 0; k < 5 && st == DG_OK; ++k) st = launch_batch_order_stage(b.prec, L, p, kLsrkA[k], kLsrkB[k], k & 1, sj);
    if (st == DG_OK) st = launch_batch_copy(L, b.p_begin[p], b.p_end[p], sj);
    if (j > 0) {
      // join even after a failed launch, so a capture in progress stays well formed
      const hipError_t e1 = hipEventRecord(b.join_ev[j - 1], sj);
      const hipError_t e2 = e1 == hipSuccess ? hipStreamWaitEvent(s, b.join_ev[j - 1], 0) : e1;
      if (st == DG_OK && e2 != hipSuccess) st = hip_fail(e2, "dg_batch: stream join");
    }
  }
  return st;
}

dg_status capture(dg_batch_s& b, double gamma) {
  b.drop_graph();
  DG_HIP(hipStreamBeginCapture(b.cap_stream, hipStreamCaptureModeThreadLocal));
  const dg_status st = enqueue_step(b, b.cfg, gamma, b.cap_stream);
  hipGraph_t g = nullptr;
  const hipError_t e = hipStreamEndCapture(b.cap_stream, &g);
  if (st != DG_OK) {
    if (g) hipGraphDestroy(g);
    return st;
  }
  if (e != hipSuccess) return hip_fail(e, "hipStreamEndCapture");
  b.graph = g;
  const hipError_t ei = hipGraphInstantiate(&b.exec, b.graph, nullptr, nullptr, 0);
  if (ei != hipSuccess) {
    b.drop_graph();
    return hip_fail(ei, "hipGraphInstantiate");
  }
  b.graph_gamma = gamma;
  b.graph_cfg = b.cfg;
  return DG_OK;
}

bool same_cfg(const dg_batch_config& a, const dg_batch_config& c) {
  return a.waves_per_block == c.waves_per_block && a.blocks_per_cu == c.blocks_per_cu && a.order == c.order &&
         a.xcd_chunks == c.xcd_chunks && a.per_order == c.per_order;
}

dg_status set_config(dg_batch_s& b, const dg_batch_config& c) {
  if (!valid_config(c))
    return fail(DG_ERR_ARG,
                "dg_batch: waves_per_block in {2,4,8}, blocks_per_cu in 1..4, order and xcd_chunks in {0,1}, "
                "per_order in {0,1,2}");
  const dg_status st = batch_prepare(b.prec, c.waves_per_block, b.tabs.lds_bytes);
  if (st != DG_OK) return st;
  b.cfg = c;
  return DG_OK;
}


std::string cache_key(const dg_batch_s& b) {
  std::vector<std::pair<int, int64_t>> ms;
  for (const Mesh* m : b.meshes) ms.emplace_back(m->p, m->E);
  std::sort(ms.begin(), ms.end());
  uint64_t h = 1469598103934665603ull;  // FNV-1a, 64 bit
  auto mix = [&h](uint64_t v) {
    for (int i = 0; i < 8; ++i) {
      h ^= (v >> (8 * i)) & 0xffu;
      h *= 1099511628211ull;
    }
  };
  for (const auto& pe : ms) {
    mix(static_cast<uint64_t>(pe.first));
    mix(static_cast<uint64_t>(pe.second));
  }
  char buf[256];
  std::snprintf(buf, sizeof buf, "%s:%dcu:%s:n%d:E%lld:%016llx", b.arch.c_str(), b.cus,
                b.prec == DG_FP32 ? "fp32" : "split_bf16", b.n, static_cast<long long>(b.n_elem),
                static_cast<unsigned long long>(h));
  return buf;
}

bool parse_entry(const std::string& obj, dg_batch_config& c) {
  double w, bp, o, x, po;
  if (!cache_field(obj, "waves_per_block", w) || !cache_field(obj, "blocks_per_cu", bp) || !cache_field(obj, "order", o) ||
      !cache_field(obj, "xcd_chunks", x) || !cache_field(obj, "per_order", po))
    return false;
  c = dg_batch_config{static_cast<int>(w), static_cast<int>(bp), static_cast<int>(o), static_cast<int>(x),
                      static_cast<int>(po)};
  return valid_config(c);
}

}  // namespace

extern "C" dg_status dg_batch_create(const dg_mesh* meshes, int n, dg_precision prec, dg_batch* out) {
  if (!out) return fail(DG_ERR_ARG, "dg_batch_create: out is NULL");
  *out = nullptr;
  if (!meshes || n < 1) return fail(DG_ERR_ARG, "dg_batch_create: need at least one mesh");
  if (prec == DG_FP64)
    return fail(DG_ERR_UNSUPPORTED, "dg_batch_create: batched stepping runs DG_FP32 or DG_SPLIT_BF16 contractions");
  if (prec != DG_FP32 && prec != DG_SPLIT_BF16) return fail(DG_ERR_ARG, "dg_batch_create: unknown precision");
  auto b = std::make_unique<dg_batch_s>();
  b->prec = prec;
  b->n = n;
  for (int i = 0; i < n; ++i) {
    if (!meshes[i]) return fail(DG_ERR_ARG, "dg_batch_create: null mesh");
    const Mesh* m = reinterpret_cast<const Mesh*>(meshes[i]);
    if (i > 0 && m->device != b->meshes[0]->device)
      return fail(DG_ERR_ARG, "dg_batch_create: all meshes must live on one device");
    b->meshes.push_back(m);
  }
  b->device = b->meshes[0]->device;
  DeviceGuard g(b->device);
  if (!g.ok) return fail(DG_ERR_HIP, "dg_batch_create: hipSetDevice failed");
  hipDeviceProp_t prop;
  DG_HIP(hipGetDeviceProperties(&prop, b->device));
  b->cus = prop.multiProcessorCount;
  b->arch = prop.gcnArchName;
  const size_t colon = b->arch.find(':');
  if (colon != std::string::npos) b->arch.resize(colon);

  // tables of each order present, from its first mesh, laid out in LDS
  int off = 0;
  for (const Mesh* m : b->meshes) {
    const int p = m->p;
    if (b->tabs.op[p]) continue;
    const LowpLayout L = lowp_layout(p);
    b->tabs.op[p] = prec == DG_FP32 ? reinterpret_cast<const uint32_t*>(m->d_op32)
                                    : reinterpret_cast<const uint32_t*>(m->d_opbf);
    b->tabs.nb[p] = m->d_nbtab;
    b->tabs.fm[p] = m->d_fmask;
    b->tabs.nb_bytes[p] = 4 * 24 * L.Nfp;
    b->tabs.fm_n[p] = 4 * L.Nfp;
  }
  for (int p = 1; p <= 4; ++p) {
    if (!b->tabs.op[p]) continue;
    b->tabs.fm_off[p] = off;
    off += (b->tabs.fm_n[p] * 4 + 15) / 16 * 16;
  }
  for (int p = 1; p <= 4; ++p) {
    if (!b->tabs.op[p]) continue;
    b->tabs.nb_off[p] = off;
    off += (b->tabs.nb_bytes[p] + 15) / 16 * 16;
  }
  b->tabs.lds_bytes = off;

  // work lists: order 0 = highest order first (mesh order within an order),
  // order 1 = mesh order; tiles ascending within a mesh
  std::vector<int> by_cost(n);
  for (int i = 0; i < n; ++i) by_cost[i] = i;
  std::stable_sort(by_cost.begin(), by_cost.end(),
                   [&](int x, int y) { return b->meshes[x]->p > b->meshes[y]->p; });
  std::vector<BatchItem> items[2];
  for (int o = 0; o < 2; ++o) {
    for (int k = 0; k < n; ++k) {
      const int i = o == 0 ? by_cost[k] : k;
      const int64_t tiles = b->meshes[i]->Epad / 16;
      for (int64_t t = 0; t < tiles; ++t) items[o].push_back(BatchItem{i, static_cast<int>(t)});
    }
  }
  b->n_items = static_cast<int64_t>(items[0].size());
  for (int64_t k = 0; k < b->n_items; ++k) {  // list 0 is grouped by order
    const int p = b->meshes[items[0][k].mesh]->p;
    if (b->p_end[p] == 0) b->p_begin[p] = k;
    b->p_end[p] = k + 1;
  }
  for (const Mesh* m : b->meshes) b->n_elem += m->E;
  for (int o = 0; o < 2; ++o) {
    if (hipMalloc(&b->d_items[o], std::max<size_t>(1, items[o].size()) * sizeof(BatchItem)) != hipSuccess)
      return fail(DG_ERR_ALLOC, "dg_batch_create: work list allocation failed");
    DG_HIP(hipMemcpy(b->d_items[o], items[o].data(), items[o].size() * sizeof(BatchItem), hipMemcpyHostToDevice));
  }
  if (hipMalloc(&b->d_meshes, n * sizeof(BatchMesh)) != hipSuccess)
    return fail(DG_ERR_ALLOC, "dg_batch_create: descriptor allocation failed");
  b->host_meshes.resize(n);
  DG_HIP(hipStreamCreateWithFlags(&b->cap_stream, hipStreamNonBlocking));
  for (hipStream_t& x : b->side) DG_HIP(hipStreamCreateWithFlags(&x, hipStreamNonBlocking));
  DG_HIP(hipEventCreateWithFlags(&b->fork_ev, hipEventDisableTiming));
  for (hipEvent_t& e : b->join_ev) DG_HIP(hipEventCreateWithFlags(&e, hipEventDisableTiming));
  const dg_status st = set_config(*b, b->cfg);
  if (st != DG_OK) return st;
  *out = b.release();
  return DG_OK;
}

extern "C" dg_status dg_batch_destroy(dg_batch b) {
  if (!b) return DG_OK;
  DeviceGuard g(b->device);
  delete b;
  return DG_OK;
}

extern "C" dg_status dg_batch_bind(dg_batch b, double* const* q, double* const* work, const double* dt) {
  if (!b) return fail(DG_ERR_ARG, "dg_batch_bind: null batch");
  if (!q || !work || !dt || !aligned8(dt)) return fail(DG_ERR_ARG, "dg_batch_bind: null or misaligned argument");
  for (int i = 0; i < b->n; ++i) {
    const Mesh& m = *b->meshes[i];
    if (!q[i] || !work[i] || !aligned8(q[i]) || !aligned8(work[i]))
      return fail(DG_ERR_ARG, "dg_batch_bind: null or misaligned state pointer of mesh " + std::to_string(i));
    const size_t len = static_cast<size_t>(5) * m.E * m.Np;
    if (work[i] < q[i] + len && q[i] < work[i] + 2 * len)
      return fail(DG_ERR_ARG, "dg_batch_bind: work overlaps q for mesh " + std::to_string(i));
    BatchMesh& d = b->host_meshes[i];
    d.q = q[i];
    d.res = work[i];
    d.tmp = work[i] + len;
    d.geo = m.d_geo;
    d.conn = m.d_conn;
    d.E = m.E;
    d.Epad = m.Epad;
    d.p = m.p;
    d.pad = 0;
  }
  DeviceGuard g(b->device);
  if (!g.ok) return fail(DG_ERR_HIP, "dg_batch_bind: hipSetDevice failed");
  b->drop_graph();
  b->bound = false;
  DG_HIP(hipMemcpy(b->d_meshes, b->host_meshes.data(), b->n * sizeof(BatchMesh), hipMemcpyHostToDevice));
  b->dt = dt;
  b->bound = true;
  return DG_OK;
}

extern "C" dg_status dg_batch_set_config(dg_batch b, const dg_batch_config* cfg) {
  if (!b || !cfg) return fail(DG_ERR_ARG, "dg_batch_set_config: null argument");
  DeviceGuard g(b->device);
  return set_config(*b, *cfg);
}

extern "C" dg_status dg_batch_get_config(dg_batch b, dg_batch_config* cfg) {
  if (!b || !cfg) return fail(DG_ERR_ARG, "dg_batch_get_config: null argument");
  *cfg = b->cfg;
  return DG_OK;
}

extern "C" dg_status dg_batch_rk_step(dg_batch b, const dg_params* prm, int use_graph, hipStream_t stream) {
  if (!b || !prm) return fail(DG_ERR_ARG, "dg_batch_rk_step: null argument");
  if (prm->model != 0 || !(prm->gamma > 1.0) || !std::isfinite(prm->gamma))
    return fail(DG_ERR_ARG, "dg_batch_rk_step: Euler model with gamma > 1 required");
  if (!b->bound) return fail(DG_ERR_ARG, "dg_batch_rk_step: no state bound (dg_batch_bind)");
  DeviceGuard g(b->device);
  if (!g.ok) return fail(DG_ERR_HIP, "dg_batch_rk_step: hipSetDevice failed");
  if (!use_graph) return enqueue_step(*b, b->cfg, prm->gamma, stream);
  if (!b->exec || b->graph_gamma != prm->gamma || !same_cfg(b->graph_cfg, b->cfg)) {
    const dg_status st = capture(*b, prm->gamma);
    if (st != DG_OK) return st;
  }
  DG_HIP(hipGraphLaunch(b->exec, stream));
  return DG_OK;
}

extern "C" dg_status dg_batch_info(dg_batch b, int64_t* n_items, int64_t* n_elem, int* graph_kernel_nodes) {
  if (!b) return fail(DG_ERR_ARG, "dg_batch_info: null batch");
  if (n_items) *n_items = b->n_items;
  if (n_elem) *n_elem = b->n_elem;
  if (graph_kernel_nodes) {
    *graph_kernel_nodes = 0;
    if (b->graph) {
      size_t count = 0;
      DG_HIP(hipGraphGetNodes(b->graph, nullptr, &count));
      std::vector<hipGraphNode_t> nodes(count);
      DG_HIP(hipGraphGetNodes(b->graph, nodes.data(), &count));
      for (size_t i = 0; i < count; ++i) {
        hipGraphNodeType t;
        DG_HIP(hipGraphNodeGetType(nodes[i], &t));
        if (t == hipGraphNodeTypeKernel) ++*graph_kernel_nodes;
      }
    }
  }
  return DG_OK;
}

extern "C" dg_status dg_batch_autotune(dg_batch b, const dg_params* prm, const char* cache_path, int trials,
                                       dg_batch_config* chosen, double* best_ms, hipStream_t stream) {
  if (!b || !prm) return fail(DG_ERR_ARG, "dg_batch_autotune: null argument");
  if (prm->model != 0 || !(prm->gamma > 1.0) || !std::isfinite(prm->gamma))
    return fail(DG_ERR_ARG, "dg_batch_autotune: Euler model with gamma > 1 required");
  if (trials < 1 || trials > 1000) return fail(DG_ERR_ARG, "dg_batch_autotune: trials must be in 1..1000");
  if (!b->bound) return fail(DG_ERR_ARG, "dg_batch_autotune: no state bound (dg_batch_bind)");
  DeviceGuard g(b->device);
  if (!g.ok) return fail(DG_ERR_HIP, "dg_batch_autotune: hipSetDevice failed");
  const std::string key = cache_key(*b);
  std::map<std::string, std::string> cache;
  if (cache_path) {
    cache = read_cache(cache_path);
    const auto it = cache.find(key);
    dg_batch_config c;
    if (it != cache.end() && parse_entry(it->second, c)) {
      const dg_status st = set_config(*b, c);
      if (st != DG_OK) return st;
      if (chosen) *chosen = c;
      if (best_ms) *best_ms = -1.0;
      return DG_OK;
    }
  }

  // save the bound states
  std::vector<size_t> len(b->n);
  size_t total = 0;
  for (int i = 0; i < b->n; ++i) {
    len[i] = static_cast<size_t>(5) * b->meshes[i]->E * b->meshes[i]->Np;
    total += len[i];
  }
  double* save = nullptr;
  if (hipMalloc(&save, total * sizeof(double)) != hipSuccess)
    return fail(DG_ERR_ALLOC, "dg_batch_autotune: no room to save the bound state");
  struct Free {
    double* p;
    ~Free() { hipFree(p); }
  } free_save{save};
  {
    size_t o = 0;
    for (int i = 0; i < b->n; ++i) {
      DG_HIP(hipMemcpyAsync(save + o, b->host_meshes[i].q, len[i] * sizeof(double), hipMemcpyDeviceToDevice, stream));
      o += len[i];
    }
  }
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

  const dg_batch_config prev = b->cfg;
  dg_batch_config best = prev;
  double best_t = -1.0;
  dg_status st = DG_OK;
  std::vector<dg_batch_config> cands{dg_batch_config{4, 2, 0, 0, 1}, dg_batch_config{4, 2, 0, 0, 2}};
  for (int w : {2, 4, 8}) {
    const int occ = batch_stage_occupancy(b->prec, w, b->tabs.lds_bytes);
    for (int bp = 1; bp <= std::min(occ, kMaxBlocksPerCu); ++bp)  // more than occ: the same grid as the cap
      for (int o = 0; o < 2; ++o)
        for (int x = 0; x < 2; ++x) cands.push_back(dg_batch_config{w, bp, o, x, 0});
  }
  for (const dg_batch_config& c : cands) {
    st = set_config(*b, c);
    if (st != DG_OK) break;
    st = enqueue_step(*b, c, prm->gamma, stream);  // warm-up
    if (st != DG_OK) break;
    if (hipEventRecord(e0, stream) != hipSuccess) {
      st = fail(DG_ERR_HIP, "dg_batch_autotune: hipEventRecord failed");
      break;
    }
    for (int t = 0; t < trials && st == DG_OK; ++t) st = enqueue_step(*b, c, prm->gamma, stream);
    if (st != DG_OK) break;
    if (hipEventRecord(e1, stream) != hipSuccess || hipEventSynchronize(e1) != hipSuccess) {
      st = fail(DG_ERR_HIP, "dg_batch_autotune: event timing failed");
      break;
    }
    float ms = 0.f;
    if (hipEventElapsedTime(&ms, e0, e1) != hipSuccess) {
      st = fail(DG_ERR_HIP, "dg_batch_autotune: hipEventElapsedTime failed");
      break;
    }
    const double per = static_cast<double>(ms) / trials;
    if (best_t < 0.0 || per < best_t) {
      best_t = per;
      best = c;
    }
  }
  // restore the bound states whatever happened
  {
    size_t o = 0;
    for (int i = 0; i < b->n; ++i) {
      hipMemcpyAsync(b->host_meshes[i].q, save + o, len[i] * sizeof(double), hipMemcpyDeviceToDevice, stream);
      o += len[i];
    }
    const hipError_t e = hipStreamSynchronize(stream);
    if (st == DG_OK && e != hipSuccess) st = hip_fail(e, "dg_batch_autotune: restore");
  }
  if (st != DG_OK) {
    set_config(*b, prev);
    return st;
  }
  st = set_config(*b, best);
  if (st != DG_OK) return st;
  if (chosen) *chosen = best;
  if (best_ms) *best_ms = best_t;
  if (cache_path) {
    char buf[256];
    std::snprintf(buf, sizeof buf,
                  "{\"waves_per_block\": %d, \"blocks_per_cu\": %d, \"order\": %d, \"xcd_chunks\": %d, "
                  "\"per_order\": %d, \"ms\": %.6g}",
                  best.waves_per_block, best.blocks_per_cu, best.order, best.xcd_chunks, best.per_order, best_t);
    cache[key] = buf;
    if (!write_cache(cache_path, cache))
      return fail(DG_ERR_ARG, std::string("dg_batch_autotune: cannot write cache file ") + cache_path);
  }
  return DG_OK;
}
