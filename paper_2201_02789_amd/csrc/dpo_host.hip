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

size_t align_up(size_t x) { return (x + 255) & ~(size_t)255; }

struct Layout {
  size_t state, grp_packed, grp_done, front0, front1, visit, rec, desc, stats, total;
  int32_t ngroups_cap, desc_cap, fcap;
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

int64_t cdiv(int64_t a, int64_t b) { return (a + b - 1) / b; }

Layout layout_for(int32_t n, const dpo_options& o) {
  Layout L{};
  const int gran = gran_of(o);
  const int64_t nvb = cdiv(n, PB);
  const int64_t k = (gran == AGG_MULTI) ? o.agg_blocks : 1;
  L.ngroups_cap = (gran == AGG_MULTI) ? (int32_t)cdiv(nvb, k) : 1;
  // descriptors per queue: virtual block vb publishes to queue vb % NQD
  // (multi-block group g to queue g % NQD)
  switch (gran) {
    case AGG_NONE: L.desc_cap = (int32_t)(PB * cdiv(nvb, NQD)); break;
    case AGG_WAVE: L.desc_cap = (int32_t)(NW * cdiv(nvb, NQD)); break;
    case AGG_BLOCK: L.desc_cap = (int32_t)cdiv(nvb, NQD); break;
    case AGG_MULTI: L.desc_cap = (int32_t)cdiv(L.ngroups_cap, NQD); break;
    default: L.desc_cap = 1; break;
  }
  L.fcap = (int32_t)(2 * cdiv(n, NQF) + 64);
  const size_t fslots = (size_t)NQF * L.fcap + (size_t)n;
  size_t off = 0;
  L.state = off; off = align_up(off + sizeof(State));
  L.grp_packed = off; off = align_up(off + 3 * (size_t)L.ngroups_cap * 8);
  L.grp_done = off; off = align_up(off + 3 * (size_t)L.ngroups_cap * 4);
  L.front0 = off; off = align_up(off + fslots * 4);
  L.front1 = off; off = align_up(off + fslots * 4);
  L.visit = off; off = align_up(off + (size_t)n * 4);
  L.rec = off; off = align_up(off + (size_t)n * 16);
  L.desc = off; off = align_up(off + (size_t)NQD * L.desc_cap * 16);
  L.stats = off; off = align_up(off + (size_t)MAX_GRID * NSTAT * 8);
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
  const void* parent;
  const void* child;
  int pgrid, cgrid, steps;
  Args args;
  hipGraphExec_t exec;
  uint64_t last_use;
};

struct Runtime {
  std::mutex mu;
  std::vector<CachedGraph> graphs;
  uint64_t tick = 0;
  uint32_t* host_flags = nullptr;  // pinned: base, done, error, levels_run
  unsigned long long* host_stats = nullptr;  // pinned: MAX_GRID * NSTAT
  int cu_count = 0;
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
  if (hipHostMalloc(&p, 256 + (size_t)MAX_GRID * NSTAT * 8, hipHostMallocDefault) != hipSuccess)
    return DPO_ERR_HIP;
  r.host_flags = (uint32_t*)p;
  r.host_stats = (unsigned long long*)((char*)p + 256);
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
  if (grid > MAX_GRID) grid = MAX_GRID;
  r.grids.emplace_back(kernel, grid);
  return grid;
}

dpo_status add_node(hipGraph_t graph, hipGraphNode_t* prev, const void* fn, int grid, int block,
                    void** params) {
  hipKernelNodeParams kp{};
  kp.func = const_cast<void*>(fn);
  kp.gridDim = dim3(grid);
  kp.blockDim = dim3(block);
  kp.sharedMemBytes = 0;
  kp.kernelParams = params;
  kp.extra = nullptr;
  hipGraphNode_t node;
  if (hipGraphAddKernelNode(&node, graph, *prev ? prev : nullptr, *prev ? 1 : 0, &kp) !=
      hipSuccess)
    return DPO_ERR_HIP;
  *prev = node;
  return DPO_OK;
}

// K level steps (parent kernel, then child kernel unless flat) and the
// advance of the level base, as one instantiated graph.
dpo_status get_exec(Runtime& r, const void* parent, const void* child, int pgrid, int cgrid,
                    int steps, const Args& args, hipGraphExec_t* out) {
  for (auto& e : r.graphs) {
    if (e.parent == parent && e.child == child && e.pgrid == pgrid && e.cgrid == cgrid &&
        e.steps == steps && std::memcmp(&e.args, &args, sizeof(Args)) == 0) {
      e.last_use = ++r.tick;
      *out = e.exec;
      return DPO_OK;
    }
  }
  hipGraph_t graph;
  if (hipGraphCreate(&graph, 0) != hipSuccess) return DPO_ERR_HIP;
  Args a = args;
  std::vector<uint32_t> step_ids(steps);
  hipGraphNode_t prev = nullptr;
  dpo_status s = DPO_OK;
  for (int i = 0; i < steps && s == DPO_OK; ++i) {
    step_ids[i] = (uint32_t)i;
    void* params[] = {&a, &step_ids[i]};
    s = add_node(graph, &prev, parent, pgrid, PB, params);
    if (s == DPO_OK && child) s = add_node(graph, &prev, child, cgrid, PB, params);
  }
  State* st = a.st;
  uint32_t k = (uint32_t)steps;
  void* aparams[] = {&st, &k};
  if (s == DPO_OK) s = add_node(graph, &prev, advance_kernel_ptr(), 1, 64, aparams);
  hipGraphExec_t exec;
  if (s == DPO_OK && hipGraphInstantiate(&exec, graph, nullptr, nullptr, 0) != hipSuccess)
    s = DPO_ERR_HIP;
  (void)hipGraphDestroy(graph);
  if (s != DPO_OK) return s;
  if ((int)r.graphs.size() >= kMaxCachedGraphs) {
    size_t victim = 0;
    for (size_t i = 1; i < r.graphs.size(); ++i)
      if (r.graphs[i].last_use < r.graphs[victim].last_use) victim = i;
    (void)hipGraphExecDestroy(r.graphs[victim].exec);
    r.graphs.erase(r.graphs.begin() + victim);
  }
  r.graphs.push_back(CachedGraph{parent, child, pgrid, cgrid, steps, args, exec, ++r.tick});
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
  const void* parent = parent_kernel_ptr(problem, gran);
  const void* child = gran == AGG_FLAT ? nullptr : child_kernel_ptr(problem, o->coarsen);
  if (!parent || (gran != AGG_FLAT && !child)) return DPO_ERR_UNSUPPORTED;
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
  a.desc = (int4*)(base + lay.desc);
  a.stats = (unsigned long long*)(base + lay.stats);
  a.n = g->n;
  a.m = g->m;
  a.T = o->threshold;
  a.CB = o->child_block;
  a.CF = o->coarsen;
  a.k = (gran == AGG_MULTI) ? o->agg_blocks : 1;
  a.ngroups_cap = lay.ngroups_cap;
  a.desc_cap = lay.desc_cap;
  a.fcap = lay.fcap;
  a.count_stats = st ? 1 : 0;

  const int pgrid = persistent_grid(r, parent);
  const int cgrid = child ? persistent_grid(r, child) : 0;
  const int steps = o->steps_per_replay ? o->steps_per_replay : kDefaultSteps;
  hipGraphExec_t exec;
  s = get_exec(r, parent, child, pgrid, cgrid, steps, a, &exec);
  if (s != DPO_OK) return s;

  // init: enough workgroups to sweep n quickly
  int init_grid = (int)((std::max<int64_t>(g->n, MAX_GRID * NSTAT) + PB - 1) / PB);
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
    if (hipMemcpyAsync(r.host_stats, a.stats, (size_t)MAX_GRID * NSTAT * 8, hipMemcpyDeviceToHost,
                       stream) != hipSuccess ||
        hipStreamSynchronize(stream) != hipSuccess)
      return DPO_ERR_HIP;
    int64_t sum[NSTAT] = {0};
    for (int w = 0; w < MAX_GRID; ++w)
      for (int k = 0; k < NSTAT; ++k) sum[k] += (int64_t)r.host_stats[w * NSTAT + k];
    std::memset(st, 0, sizeof(*st));
    st->levels = (int32_t)r.host_flags[3];
    st->frontier_total = sum[S_FRONT];
    st->serial_parents = sum[S_SERIAL];
    st->records = sum[S_REC];
    st->child_blocks = sum[S_CHILD];
    st->edges_serial = sum[S_ESER];
    st->edges_child = sum[S_ECHILD];
    st->descriptors = sum[S_DESC];
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
