// Host driver and C ABI of the nested-parallel BFS / SSSP library.
//
// A traversal is: one init kernel, then HIP-graph replays of K captured level
// steps (the step kernel reads its level, frontier and counters from the
// workspace, so one instantiated graph serves every call with the same
// arguments), with one stream synchronisation per replay to read the done
// flag.  Instantiated graphs are cached by their exact kernel arguments.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <cstdlib>
#include <cstring>
#include <mutex>
#include <vector>

#include "dpo.h"
#include "dpo_internal.h"

namespace dpo {
namespace {

constexpr int kDefaultSteps = 16;
constexpr int kMaxCachedGraphs = 64;
constexpr uint64_t kTicksPerMs = 100000;  // s_memrealtime runs at 100 MHz
constexpr uint64_t kDefaultWatchdogMs = 4000;

size_t align_up(size_t x) { return (x + 255) & ~(size_t)255; }

struct Layout {
  size_t state, grp_packed, grp_done, front0, front1, visit, rec, desc_a, desc_b, total;
  int32_t ngroups_cap, desc_cap;
};

int gran_of(const dpo_options& o) {
  if (o.mode == DPO_MODE_FLAT) return AGG_FLAT;
  switch (o.agg) {
    case DPO_AGG_NONE: return AGG_NONE;
    case DPO_AGG_WAVE: return AGG_WAVE;
    case DPO_AGG_BLOCK: return AGG_BLOCK;
    case DPO_AGG_MULTIBLOCK: return AGG_MULTI;
    default: return -1;
  }
}

Layout layout_for(int32_t n, const dpo_options& o) {
  Layout L{};
  const int gran = gran_of(o);
  const int64_t nvb = (n + PB - 1) / PB;
  const int64_t k = (gran == AGG_MULTI) ? o.agg_blocks : 1;
  L.ngroups_cap = (gran == AGG_MULTI) ? (int32_t)((nvb + k - 1) / k) : 1;
  switch (gran) {
    case AGG_NONE: L.desc_cap = n; break;
    case AGG_WAVE: L.desc_cap = (n + 63) / 64; break;
    case AGG_BLOCK: L.desc_cap = (int32_t)nvb; break;
    case AGG_MULTI: L.desc_cap = L.ngroups_cap; break;
    default: L.desc_cap = 1; break;
  }
  size_t off = 0;
  L.state = off; off = align_up(off + sizeof(State));
  L.grp_packed = off; off = align_up(off + 3 * (size_t)L.ngroups_cap * 8);
  L.grp_done = off; off = align_up(off + 3 * (size_t)L.ngroups_cap * 4);
  L.front0 = off; off = align_up(off + (size_t)n * 4);
  L.front1 = off; off = align_up(off + (size_t)n * 4);
  L.visit = off; off = align_up(off + (size_t)n * 4);
  L.rec = off; off = align_up(off + (size_t)n * 16);
  L.desc_a = off; off = align_up(off + (size_t)L.desc_cap * 8);
  L.desc_b = off; off = align_up(off + (size_t)L.desc_cap * 8);
  L.total = off;
  return L;
}

dpo_status check_options(const dpo_options& o) {
  if (o.mode != DPO_MODE_NESTED && o.mode != DPO_MODE_FLAT) return DPO_ERR_ARG;
  if (o.threshold < 0) return DPO_ERR_ARG;
  if (o.coarsen != 1 && o.coarsen != 2 && o.coarsen != 4 && o.coarsen != 8 && o.coarsen != 16)
    return DPO_ERR_ARG;
  if (o.agg < DPO_AGG_NONE || o.agg > DPO_AGG_MULTIBLOCK) return DPO_ERR_ARG;
  if (o.agg == DPO_AGG_MULTIBLOCK && (o.agg_blocks < 2 || o.agg_blocks > 1024)) return DPO_ERR_ARG;
  if (o.child_block != 64 && o.child_block != 128 && o.child_block != 256) return DPO_ERR_ARG;
  if (o.steps_per_replay < 0 || o.steps_per_replay > 1024) return DPO_ERR_ARG;
  return DPO_OK;
}

dpo_status check_graph(const dpo_csr* g, bool need_w) {
  if (!g || g->n < 1 || g->m < 0 || !g->row_ptr) return DPO_ERR_ARG;
  if (g->m > 0 && !g->col_idx) return DPO_ERR_ARG;
  if (need_w && g->m > 0 && !g->weights) return DPO_ERR_ARG;
  return DPO_OK;
}

struct CachedGraph {
  const void* kernel;
  int grid;
  int steps;
  Args args;
  hipGraphExec_t exec;
  uint64_t last_use;
};

struct Runtime {
  std::mutex mu;
  std::vector<CachedGraph> graphs;
  uint64_t tick = 0;
  uint32_t* host_flags = nullptr;  // pinned: level, done, error, levels_run
  unsigned long long* host_stats = nullptr;
  int cu_count = 0;
  uint64_t watchdog_ticks = 0;
  std::vector<std::pair<const void*, int>> grids;
};

Runtime& rt() {
  static Runtime r;
  return r;
}

dpo_status hip_ok(hipError_t e) { return e == hipSuccess ? DPO_OK : DPO_ERR_HIP; }

dpo_status ensure_runtime(Runtime& r) {
  if (r.host_flags) return DPO_OK;
  int dev = 0;
  if (hipGetDevice(&dev) != hipSuccess) return DPO_ERR_HIP;
  if (hipDeviceGetAttribute(&r.cu_count, hipDeviceAttributeMultiprocessorCount, dev) != hipSuccess)
    return DPO_ERR_HIP;
  void* p = nullptr;
  if (hipHostMalloc(&p, 256, hipHostMallocDefault) != hipSuccess) return DPO_ERR_HIP;
  r.host_flags = (uint32_t*)p;
  r.host_stats = (unsigned long long*)((char*)p + 64);
  uint64_t ms = kDefaultWatchdogMs;
  if (const char* env = std::getenv("DPO_WATCHDOG_MS")) {
    long v = std::atol(env);
    if (v > 0) ms = (uint64_t)v;
  }
  r.watchdog_ticks = ms * kTicksPerMs;
  return DPO_OK;
}

// Persistent grid: as many workgroups as can be resident at once.
int persistent_grid(Runtime& r, const void* kernel) {
  for (auto& e : r.grids)
    if (e.first == kernel) return e.second;
  int per_cu = 0;
  if (hipOccupancyMaxActiveBlocksPerMultiprocessor(&per_cu, kernel, PB, 0) != hipSuccess ||
      per_cu < 1)
    per_cu = 1;
  if (per_cu > 8) per_cu = 8;
  int grid = per_cu * r.cu_count;
  r.grids.emplace_back(kernel, grid);
  return grid;
}

dpo_status get_exec(Runtime& r, const void* kernel, int grid, int steps, const Args& args,
                    hipGraphExec_t* out) {
  for (auto& e : r.graphs) {
    if (e.kernel == kernel && e.grid == grid && e.steps == steps &&
        std::memcmp(&e.args, &args, sizeof(Args)) == 0) {
      e.last_use = ++r.tick;
      *out = e.exec;
      return DPO_OK;
    }
  }
  hipGraph_t graph;
  if (hipGraphCreate(&graph, 0) != hipSuccess) return DPO_ERR_HIP;
  Args a = args;
  void* params[] = {&a};
  hipKernelNodeParams kp{};
  kp.func = const_cast<void*>(kernel);
  kp.gridDim = dim3(grid);
  kp.blockDim = dim3(PB);
  kp.sharedMemBytes = 0;
  kp.kernelParams = params;
  kp.extra = nullptr;
  hipGraphNode_t prev = nullptr;
  for (int i = 0; i < steps; ++i) {
    hipGraphNode_t node;
    if (hipGraphAddKernelNode(&node, graph, prev ? &prev : nullptr, prev ? 1 : 0, &kp) !=
        hipSuccess) {
      hipGraphDestroy(graph);
      return DPO_ERR_HIP;
    }
    prev = node;
  }
  hipGraphExec_t exec;
  hipError_t e = hipGraphInstantiate(&exec, graph, nullptr, nullptr, 0);
  hipGraphDestroy(graph);
  if (e != hipSuccess) return DPO_ERR_HIP;
  if ((int)r.graphs.size() >= kMaxCachedGraphs) {
    size_t victim = 0;
    for (size_t i = 1; i < r.graphs.size(); ++i)
      if (r.graphs[i].last_use < r.graphs[victim].last_use) victim = i;
    hipGraphExecDestroy(r.graphs[victim].exec);
    r.graphs.erase(r.graphs.begin() + victim);
  }
  r.graphs.push_back(CachedGraph{kernel, grid, steps, args, exec, ++r.tick});
  *out = exec;
  return DPO_OK;
}

dpo_status traverse(int problem, const dpo_csr* g, int32_t source, const dpo_options* o,
                    void* out, void* ws, size_t ws_bytes, void* stream_, dpo_stats* st) {
  if (!o || !out || !ws) return DPO_ERR_ARG;
  dpo_status s = check_graph(g, problem == PROB_SSSP);
  if (s != DPO_OK) return s;
  s = check_options(*o);
  if (s != DPO_OK) return s;
  if (problem == PROB_SSSP && g->n > 16843009) return DPO_ERR_ARG;
  if (source < 0 || source >= g->n) return DPO_ERR_SOURCE;
  const Layout lay = layout_for(g->n, *o);
  if (ws_bytes < lay.total) return DPO_ERR_WORKSPACE;
  const int gran = gran_of(*o);
  const void* kernel = step_kernel_ptr(problem, gran, gran == AGG_FLAT ? 1 : o->coarsen);
  if (!kernel) return DPO_ERR_UNSUPPORTED;
  hipStream_t stream = (hipStream_t)stream_;

  Runtime& r = rt();
  std::lock_guard<std::mutex> lock(r.mu);
  s = ensure_runtime(r);
  if (s != DPO_OK) return s;

  char* base = (char*)ws;
  Args a;
  std::memset(&a, 0, sizeof(a));  // padding too: cached graphs are keyed by these bytes
  a.rp = g->row_ptr;
  a.col = g->col_idx;
  a.w = g->weights;
  a.level = problem == PROB_BFS ? (int32_t*)out : nullptr;
  a.dist = problem == PROB_SSSP ? (uint32_t*)out : nullptr;
  a.st = (State*)(base + lay.state);
  a.grp_packed = (unsigned long long*)(base + lay.grp_packed);
  a.grp_done = (uint32_t*)(base + lay.grp_done);
  a.front0 = (int32_t*)(base + lay.front0);
  a.front1 = (int32_t*)(base + lay.front1);
  a.visit = (uint32_t*)(base + lay.visit);
  a.rec = (int4*)(base + lay.rec);
  a.desc_a = (unsigned long long*)(base + lay.desc_a);
  a.desc_b = (unsigned long long*)(base + lay.desc_b);
  a.n = g->n;
  a.m = g->m;
  a.T = o->threshold;
  a.CB = o->child_block;
  a.k = (gran == AGG_MULTI) ? o->agg_blocks : 1;
  a.ngroups_cap = lay.ngroups_cap;
  a.desc_cap = lay.desc_cap;
  a.count_stats = st ? 1 : 0;
  a.watchdog_ticks = r.watchdog_ticks;

  const int grid = persistent_grid(r, kernel);
  const int steps = o->steps_per_replay ? o->steps_per_replay : kDefaultSteps;
  hipGraphExec_t exec;
  s = get_exec(r, kernel, grid, steps, a, &exec);
  if (s != DPO_OK) return s;

  // init: enough workgroups to sweep n (and the descriptor flags) quickly
  int init_grid = (int)((std::max<int64_t>(g->n, lay.desc_cap) + PB - 1) / PB);
  if (init_grid > 4 * r.cu_count) init_grid = 4 * r.cu_count;
  if (init_grid < 1) init_grid = 1;
  void* iparams[] = {&a, &source};
  if (hipLaunchKernel(init_kernel_ptr(problem), dim3(init_grid), dim3(PB), iparams, 0, stream) !=
      hipSuccess)
    return DPO_ERR_HIP;

  // Each non-empty step advances the level by one; a traversal has at most n
  // non-empty steps (BFS levels; Bellman-Ford frontier iterations).
  const int64_t max_replays = (int64_t)g->n / steps + 2;
  bool finished = false;
  for (int64_t rep = 0; rep < max_replays; ++rep) {
    if (hipGraphLaunch(exec, stream) != hipSuccess) return DPO_ERR_HIP;
    if (hipMemcpyAsync(r.host_flags, a.st, 16, hipMemcpyDeviceToHost, stream) != hipSuccess)
      return DPO_ERR_HIP;
    if (hipStreamSynchronize(stream) != hipSuccess) return DPO_ERR_HIP;
    if (r.host_flags[2] != 0) return (dpo_status)(-(int32_t)r.host_flags[2]);
    if (r.host_flags[1]) {
      finished = true;
      break;
    }
  }
  if (!finished) return DPO_ERR_TIMEOUT;
  if (st) {
    if (hipMemcpyAsync(r.host_stats, a.st->stats, 8 * sizeof(unsigned long long),
                       hipMemcpyDeviceToHost, stream) != hipSuccess ||
        hipStreamSynchronize(stream) != hipSuccess)
      return DPO_ERR_HIP;
    std::memset(st, 0, sizeof(*st));
    st->levels = (int32_t)r.host_flags[3];
    st->frontier_total = (int64_t)r.host_stats[0];
    st->serial_parents = (int64_t)r.host_stats[1];
    st->records = (int64_t)r.host_stats[2];
    st->child_blocks = (int64_t)r.host_stats[3];
    st->edges_serial = (int64_t)r.host_stats[4];
    st->edges_child = (int64_t)r.host_stats[5];
    st->descriptors = (int64_t)r.host_stats[6];
  }
  return DPO_OK;
}

}  // namespace
}  // namespace dpo

extern "C" {

void dpo_default_options(dpo_options* o) {
  if (!o) return;
  o->mode = DPO_MODE_NESTED;
  o->threshold = 128;
  o->coarsen = 8;
  o->agg = DPO_AGG_MULTIBLOCK;
  o->agg_blocks = 4;
  o->child_block = 256;
  o->steps_per_replay = 0;
}

size_t dpo_workspace_bytes(const dpo_csr* g, const dpo_options* o) {
  if (!g || !o || g->n < 1 || dpo::check_options(*o) != DPO_OK) return 0;
  return dpo::layout_for(g->n, *o).total;
}

dpo_status dpo_bfs(const dpo_csr* g, int32_t source, const dpo_options* o, int32_t* levels,
                   void* ws, size_t ws_bytes, void* stream, dpo_stats* st) {
  return dpo::traverse(dpo::PROB_BFS, g, source, o, levels, ws, ws_bytes, stream, st);
}

dpo_status dpo_sssp(const dpo_csr* g, int32_t source, const dpo_options* o, uint32_t* dist,
                    void* ws, size_t ws_bytes, void* stream, dpo_stats* st) {
  return dpo::traverse(dpo::PROB_SSSP, g, source, o, dist, ws, ws_bytes, stream, st);
}

const char* dpo_strerror(int32_t status) {
  switch (status) {
    case DPO_OK: return "ok";
    case DPO_ERR_ARG: return "invalid argument";
    case DPO_ERR_SOURCE: return "source vertex out of range";
    case DPO_ERR_WORKSPACE: return "workspace too small";
    case DPO_ERR_CAPACITY: return "device queue capacity exceeded";
    case DPO_ERR_TIMEOUT: return "device wait exceeded its watchdog or level cap";
    case DPO_ERR_HIP: return "HIP runtime error";
    case DPO_ERR_UNSUPPORTED: return "option combination not built";
    default: return "unknown status";
  }
}

}  // extern "C"
