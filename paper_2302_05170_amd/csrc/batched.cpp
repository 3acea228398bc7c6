// Batched launches of many uneven instances (one persistent fused kernel
// over a longest-M-first work queue), their hipGraph cache, and the launch-
// plan autotuner.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <chrono>
#include <cmath>
#include <cstdio>
#include <cstring>
#include <fstream>
#include <map>
#include <memory>
#include <mutex>
#include <sstream>
#include <string>
#include <vector>

#include "sl7_host.hpp"

using namespace sl7;

namespace {

uint64_t fnv1a(const void* p, size_t n, uint64_t h = 1469598103934665603ull) {
  const unsigned char* c = (const unsigned char*)p;
  for (size_t i = 0; i < n; ++i) {
    h ^= c[i];
    h *= 1099511628211ull;
  }
  return h;
}

// A captured launch sequence with buffers of its own, so replays need no
// upload and are not disturbed by other calls on the device.
struct GraphEntry {
  std::string key;  // everything the captured nodes depend on (see graph_key)
  Workspace ws;
  hipGraph_t graph = nullptr;
  hipGraphExec_t exec = nullptr;
  hipStream_t capture = nullptr;
  sl7_stats* host = nullptr;
  int n = 0;
  ~GraphEntry() {
    if (exec) (void)hipGraphExecDestroy(exec);
    if (graph) (void)hipGraphDestroy(graph);
    if (capture) (void)hipStreamDestroy(capture);
    if (host) (void)hipHostFree(host);
  }
};

struct GraphCache {
  std::mutex mu;
  std::map<uint64_t, std::unique_ptr<GraphEntry>> entries;
  std::vector<uint64_t> lru;
};

GraphCache& graph_cache() {
  static GraphCache c;
  return c;
}

int check_batch(const sl7_problem* prs, int n, const Mlp* H, int prec) {
  if (!prs) return fail(SL7_EINVAL, "prs is NULL");
  if (n < 1 || n > 65536) return fail(SL7_EINVAL, "n=%d outside [1, 65536]", n);
  if (!H) return fail(SL7_EUNSUPPORTED, "batched launches need a network");
  if (prec == SL7_F64)
    return fail(SL7_EUNSUPPORTED, "batched launches run in F32, BF16, F16, BF16X3, F16X3, PWL32 or PWL64");
  char name[32];
  for (int k = 0; k < n; ++k) {
    snprintf(name, sizeof(name), "prs[%d]", k);
    int rc = check_problem(&prs[k], H, prec, name);
    if (rc) return rc;
    if (prs[k].m != prs[0].m) return fail(SL7_EINVAL, "prs[%d].m differs from prs[0].m", k);
  }
  return SL7_OK;
}

}  // namespace

extern "C" int sl7_simulate_batched(const sl7_problem* prs, int n, const sl7_mlp* Hc, int prec,
                                    uint64_t seed, sl7_stats* stats_host, const sl7_plan* plan_in,
                                    int use_graph, void* stream) {
  Mlp* H = const_cast<Mlp*>(reinterpret_cast<const Mlp*>(Hc));
  int rc = check_batch(prs, n, H, prec);
  if (rc) return rc;
  if (!stats_host) return fail(SL7_EINVAL, "stats_host is NULL");
  int dev;
  rc = current_device(&dev);
  if (rc) return rc;
  sl7_plan plan;
  if (plan_in) plan = *plan_in;
  else default_plan(prec, total_blocks(prs, n), workspace(dev).n_cu, &plan);
  rc = check_plan(&plan, prec);
  if (rc) return rc;
  rc = H->ensure_device(prec);
  if (rc) return rc;
  hipStream_t s = (hipStream_t)stream;
  std::vector<sl7_problem> p(prs, prs + n);
  for (int k = 0; k < n; ++k) p[k].instance = prs[k].instance;
  if (!use_graph) {
    Workspace& ws = workspace(dev);
    WsLease lease(ws, s);
    rc = lease.begin();
    if (rc) return rc;
    rc = run_instances(p.data(), n, H, prec, seed, nullptr, &plan, s, ws);
    if (rc) return rc;
    return fetch_stats(ws, n, stats_host, s);
  }
  // graph path: the entry is found by a hash of everything the captured
  // nodes depend on (the problems, plan, seed, precision, device, the
  // network's version, which changes with its parameters and is unique in
  // the process, and its device weights) and used only if all of it matches
  std::string full;
  auto add = [&full](const void* b, size_t nb) { full.append((const char*)b, nb); };
  add(p.data(), sizeof(sl7_problem) * n);
  add(&plan, sizeof(plan));
  add(&seed, sizeof(seed));
  add(&prec, sizeof(prec));
  add(&dev, sizeof(dev));
  add(&H->version, sizeof(H->version));
  if (!is_pwl(prec)) {
    const void* wp = H->pack[prec]->p;
    add(&wp, sizeof(wp));
    add(&H->pack[prec]->generation, sizeof(uint64_t));
  }
  const uint64_t key = fnv1a(full.data(), full.size());
  GraphCache& gc = graph_cache();
  std::lock_guard<std::mutex> lk(gc.mu);
  auto it = gc.entries.find(key);
  if (it != gc.entries.end() && it->second->key != full) {  // a hash collision: rebuild
    gc.entries.erase(it);
    gc.lru.erase(std::remove(gc.lru.begin(), gc.lru.end(), key), gc.lru.end());
    it = gc.entries.end();
  }
  GraphEntry* E = nullptr;
  if (it == gc.entries.end()) {
    std::unique_ptr<GraphEntry> ne(new GraphEntry());
    ne->key = full;
    ne->ws.n_cu = workspace(dev).n_cu;
    ne->n = n;
    hipError_t e = hipStreamCreateWithFlags(&ne->capture, hipStreamNonBlocking);
    if (e != hipSuccess) return hip_fail(e, "hipStreamCreate");
    e = hipHostMalloc((void**)&ne->host, sizeof(sl7_stats) * n, 0);
    if (e != hipSuccess) return fail(SL7_ENOMEM, "hipHostMalloc(stats)");
    SimArgs a;
    rc = prepare_instances(p.data(), n, H, prec, seed, nullptr, ne->capture, ne->ws, a);
    if (rc) return rc;
    e = hipStreamSynchronize(ne->capture);
    if (e != hipSuccess) return hip_fail(e, "upload instance table");
    e = hipStreamBeginCapture(ne->capture, hipStreamCaptureModeThreadLocal);
    if (e != hipSuccess) return hip_fail(e, "hipStreamBeginCapture");
    rc = launch_instances(a, n, p[0].N, H, prec, plan, ne->capture, ne->ws);
    if (!rc) {
      e = hipMemcpyAsync(ne->host, ne->ws.stats.p, sizeof(sl7_stats) * n, hipMemcpyDeviceToHost,
                         ne->capture);
      if (e != hipSuccess) rc = hip_fail(e, "capture statistics copy");
    }
    hipGraph_t g = nullptr;
    const hipError_t e2 = hipStreamEndCapture(ne->capture, &g);
    if (rc) {
      if (g) (void)hipGraphDestroy(g);
      return rc;
    }
    if (e2 != hipSuccess) return hip_fail(e2, "hipStreamEndCapture");
    ne->graph = g;
    e = hipGraphInstantiate(&ne->exec, g, nullptr, nullptr, 0);
    if (e != hipSuccess) return hip_fail(e, "hipGraphInstantiate");
    E = ne.get();
    gc.entries[key] = std::move(ne);
    gc.lru.push_back(key);
    while (gc.lru.size() > 8) {
      gc.entries.erase(gc.lru.front());
      gc.lru.erase(gc.lru.begin());
    }
  } else {
    E = it->second.get();
  }
  hipError_t e = hipGraphLaunch(E->exec, s);
  if (e == hipSuccess) e = hipStreamSynchronize(s);
  if (e != hipSuccess) return hip_fail(e, "hipGraphLaunch");
  std::memcpy(stats_host, E->host, sizeof(sl7_stats) * n);
  for (int k = 0; k < n; ++k)
    if (!std::isfinite(stats_host[k].mean[0])) return fail(SL7_ENUMERIC, "instance %d: non-finite mean", k);
  return SL7_OK;
}

// ---------------------------------------------------------------------------
// Autotuner: times each candidate plan on the given shape and keeps the
// fastest; results are cached as JSON lines keyed by (arch, prec, d_in, m).
// ---------------------------------------------------------------------------
namespace {

std::string plan_key(int prec, const Mlp* H) {
  char b[96];
  snprintf(b, sizeof(b), "gfx950/prec%d/din%d/m%d", prec, H->d.d_in, H->d.m);
  return b;
}

bool cache_lookup(const char* path, const std::string& key, int prec, sl7_plan* out) {
  std::ifstream f(path);
  if (!f) return false;
  std::string line;
  bool found = false;
  while (std::getline(f, line)) {
    const std::string tag = "\"key\": \"" + key + "\"";
    if (line.find(tag) == std::string::npos) continue;
    sl7_plan p;
    std::memset(&p, 0, sizeof(p));
    const char* s = line.c_str();
    const char* w = strstr(s, "\"waves_per_block\":");
    const char* b = strstr(s, "\"blocks_per_cu\":");
    const char* g = strstr(s, "\"grab\":");
    if (!w || !b || !g) continue;
    p.waves_per_block = atoi(w + 18);
    p.blocks_per_cu = atoi(b + 16);
    p.grab = atoi(g + 7);
    if (check_plan(&p, prec) == SL7_OK) {
      *out = p;
      found = true;  // last matching line wins
    }
  }
  return found;
}

}  // namespace

namespace {

// Times every candidate plan on the n prepared instances and returns the
// fastest.  The default plan comes first and a candidate must beat the best
// so far by 2 % to replace it, so timing noise does not pick a plan.
int time_candidates(const sl7_problem* prs, int n, Mlp* H, int prec, hipStream_t s, Workspace& ws,
                    sl7_plan* bestp_out, float* best_out) {
  std::vector<sl7_plan> cands(1);
  default_plan(prec, total_blocks(prs, n), ws.n_cu, &cands[0]);
  const int wpb[] = {1, 2, 4, kWavesX3L};
  const int bpc[] = {1, 2, 3, 4, 8, 16};
  const int grabs[] = {1, 4};
  for (int w : wpb)
    for (int b : bpc)
      for (int g : grabs) {
        if (w * b > 32 || (w == kWavesX3L && !is_x3(prec))) continue;
        sl7_plan p = {w, b, g, 0};
        if (p.waves_per_block == cands[0].waves_per_block && p.blocks_per_cu == cands[0].blocks_per_cu &&
            p.grab == cands[0].grab)
          continue;
        cands.push_back(p);
      }
  hipEvent_t e0, e1;
  if (hipEventCreate(&e0) != hipSuccess || hipEventCreate(&e1) != hipSuccess)
    return fail(SL7_EHIP, "hipEventCreate");
  SimArgs a;
  int rc = prepare_instances(prs, n, H, prec, 1, nullptr, s, ws, a);
  float best = INFINITY;
  sl7_plan bestp = cands[0];
  for (size_t c = 0; c < cands.size() && !rc; ++c) {
    rc = launch_instances(a, n, prs[0].N, H, prec, cands[c], s, ws);  // warm-up
    float ms = INFINITY;
    for (int t = 0; t < 2 && !rc; ++t) {  // best of two timings of three launches
      (void)hipEventRecord(e0, s);
      for (int r = 0; r < 3 && !rc; ++r) rc = launch_instances(a, n, prs[0].N, H, prec, cands[c], s, ws);
      (void)hipEventRecord(e1, s);
      if (hipEventSynchronize(e1) != hipSuccess) { rc = fail(SL7_EHIP, "hipEventSynchronize"); break; }
      float t_ms = 0.f;
      (void)hipEventElapsedTime(&t_ms, e0, e1);
      ms = std::min(ms, t_ms);
    }
    if (rc) break;
    if (c == 0 || ms < 0.98f * best) { best = ms; bestp = cands[c]; }
  }
  (void)hipEventDestroy(e0);
  (void)hipEventDestroy(e1);
  if (rc) return rc;
  *bestp_out = bestp;
  *best_out = best / 3.f;
  return SL7_OK;
}

int cache_store(const char* cache_path, const std::string& key, const sl7_plan& p, float ms,
                int64_t path_steps) {
  FILE* f = fopen(cache_path, "a");
  if (!f) return fail(SL7_EIO, "cannot append to %s", cache_path);
  fprintf(f, "{\"key\": \"%s\", \"waves_per_block\": %d, \"blocks_per_cu\": %d, \"grab\": %d, "
             "\"ms_per_launch\": %.5f, \"path_steps\": %lld}\n",
          key.c_str(), p.waves_per_block, p.blocks_per_cu, p.grab, ms, (long long)path_steps);
  fclose(f);
  return SL7_OK;
}

}  // namespace

extern "C" int sl7_autotune(const sl7_problem* shape, const sl7_mlp* Hc, int prec,
                            const char* cache_path, sl7_plan* out, void* stream) {
  Mlp* H = const_cast<Mlp*>(reinterpret_cast<const Mlp*>(Hc));
  if (!out) return fail(SL7_EINVAL, "out is NULL");
  if (!H) return fail(SL7_EUNSUPPORTED, "the tuner times the network kernels; H is NULL");
  int rc = check_problem(shape, H, prec, "shape");
  if (rc) return rc;
  if (prec == SL7_F64) return fail(SL7_EUNSUPPORTED, "F64 runs the per-lane kernel (no plan)");
  const std::string key = plan_key(prec, H);
  if (cache_path && cache_lookup(cache_path, key, prec, out)) return SL7_OK;
  rc = H->ensure_device(prec);
  if (rc) return rc;
  int dev;
  rc = current_device(&dev);
  if (rc) return rc;
  Workspace& ws = workspace(dev);
  WsLease lease(ws, (hipStream_t)stream);
  rc = lease.begin();
  if (rc) return rc;
  // time on at least 2^20 paths so that each launch fills the chip for
  // several milliseconds
  sl7_problem sh = *shape;
  sh.N = std::max<int64_t>(shape->N, int64_t(1) << 20);
  sl7_plan best;
  float ms = 0.f;
  rc = time_candidates(&sh, 1, H, prec, (hipStream_t)stream, ws, &best, &ms);
  if (rc) return rc;
  *out = best;
  return cache_path ? cache_store(cache_path, key, best, ms, sh.N * sh.M) : SL7_OK;
}

extern "C" int sl7_autotune_batched(const sl7_problem* prs, int n, const sl7_mlp* Hc, int prec,
                                    const char* cache_path, sl7_plan* out, void* stream) {
  Mlp* H = const_cast<Mlp*>(reinterpret_cast<const Mlp*>(Hc));
  if (!out) return fail(SL7_EINVAL, "out is NULL");
  int rc = check_batch(prs, n, H, prec);
  if (rc) return rc;
  // the key names the batch by its shapes: model, m, M and N of every instance
  uint64_t h = fnv1a(&n, sizeof(n));
  for (int k = 0; k < n; ++k) {
    const int32_t v[3] = {prs[k].model, prs[k].m, prs[k].M};
    h = fnv1a(v, sizeof(v), h);
    h = fnv1a(&prs[k].N, sizeof(prs[k].N), h);
  }
  char hb[40];
  snprintf(hb, sizeof(hb), "/batch%016llx", (unsigned long long)h);
  const std::string key = plan_key(prec, H) + hb;
  if (cache_path && cache_lookup(cache_path, key, prec, out)) return SL7_OK;
  rc = H->ensure_device(prec);
  if (rc) return rc;
  int dev;
  rc = current_device(&dev);
  if (rc) return rc;
  Workspace& ws = workspace(dev);
  WsLease lease(ws, (hipStream_t)stream);
  rc = lease.begin();
  if (rc) return rc;
  std::vector<sl7_problem> p(prs, prs + n);
  sl7_plan best;
  float ms = 0.f;
  rc = time_candidates(p.data(), n, H, prec, (hipStream_t)stream, ws, &best, &ms);
  if (rc) return rc;
  *out = best;
  int64_t ps = 0;
  for (int k = 0; k < n; ++k) ps += prs[k].N * prs[k].M;
  return cache_path ? cache_store(cache_path, key, best, ms, ps) : SL7_OK;
}
