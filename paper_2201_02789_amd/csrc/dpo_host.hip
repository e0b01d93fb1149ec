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
  size_t state, queries, grp_packed, grp_done, front0, front1, visit, rec, rec_q, desc, stats, total;
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
int64_t round32(int64_t x) { return (x + 31) & ~(int64_t)31; }

// Workspace for `slots` output slots (frontier entries) and `nq` queries.
Layout layout_for(int64_t slots, int32_t nq, const dpo_options& o) {
  Layout L{};
  const int gran = gran_of(o);
  const int64_t nvb = cdiv(slots, PB);
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
  L.fcap = (int32_t)(2 * cdiv(slots, NQF) + 64);
  const size_t fslots = (size_t)NQF * L.fcap + (size_t)slots;
  size_t off = 0;
  L.state = off; off = align_up(off + sizeof(State));
  L.queries = off; off = align_up(off + (size_t)nq * sizeof(Query));
  L.grp_packed = off; off = align_up(off + 3 * (size_t)L.ngroups_cap * 8);
  L.grp_done = off; off = align_up(off + 3 * (size_t)L.ngroups_cap * 4);
  L.front0 = off; off = align_up(off + fslots * 4);
  L.front1 = off; off = align_up(off + fslots * 4);
  L.visit = off; off = align_up(off + (size_t)slots * 4);
  L.rec = off; off = align_up(off + (size_t)slots * 16);
  L.rec_q = off; off = align_up(off + (size_t)slots * 4);
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

struct GridEntry {
  const void* first;
  int second;
  unsigned third;
};

struct Runtime {
  std::mutex mu;
  std::vector<CachedGraph> graphs;
  uint64_t tick = 0;
  uint32_t* host_flags = nullptr;  // pinned: base, done, error, levels_run
  unsigned long long* host_stats = nullptr;  // pinned: MAX_GRID * NSTAT
  Query* host_q = nullptr;                   // pinned: MAX_QUERIES query records
  int cu_count = 0;
  std::vector<GridEntry> grids;
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
  const size_t qbytes = (size_t)MAX_QUERIES * sizeof(Query);
  if (hipHostMalloc(&p, 256 + (size_t)MAX_GRID * NSTAT * 8 + qbytes, hipHostMallocDefault) !=
      hipSuccess)
    return DPO_ERR_HIP;
  r.host_flags = (uint32_t*)p;
  r.host_stats = (unsigned long long*)((char*)p + 256);
  r.host_q = (Query*)((char*)p + 256 + (size_t)MAX_GRID * NSTAT * 8);
  return DPO_OK;
}

// Persistent grid: as many workgroups as can be resident at once.
int persistent_grid(Runtime& r, const void* kernel, unsigned shmem = 0) {
  for (auto& e : r.grids)
    if (e.first == kernel && e.third == shmem) return e.second;
  int per_cu = 0;
  if (hipOccupancyMaxActiveBlocksPerMultiprocessor(&per_cu, kernel, PB, shmem) != hipSuccess ||
      per_cu < 1)
    per_cu = 1;
  if (per_cu > 8) per_cu = 8;
  int grid = per_cu * r.cu_count;
  if (grid > MAX_GRID) grid = MAX_GRID;
  r.grids.push_back(GridEntry{kernel, grid, shmem});
  return grid;
}

dpo_status add_node(hipGraph_t graph, hipGraphNode_t* prev, const void* fn, int grid, int block,
                    void** params, unsigned shmem = 0) {
  hipKernelNodeParams kp{};
  kp.func = const_cast<void*>(fn);
  kp.gridDim = dim3(grid);
  kp.blockDim = dim3(block);
  kp.sharedMemBytes = shmem;
  kp.kernelParams = params;
  kp.extra = nullptr;
  hipGraphNode_t node;
  if (hipGraphAddKernelNode(&node, graph, *prev ? prev : nullptr, *prev ? 1 : 0, &kp) !=
      hipSuccess)
    return DPO_ERR_HIP;
  *prev = node;
  return DPO_OK;
}

// Dynamic LDS of the parent kernel: the queries' first slots and live bits.
unsigned parent_shmem(int32_t nq) { return (unsigned)(nq + (nq + 31) / 32) * 4u; }

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
    s = add_node(graph, &prev, parent, pgrid, PB, params, parent_shmem(a.nq));
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

// One set of queries run together: per-query tables, workspace carving and
// the replay loop shared by the single, batch and serving entry points.
struct SetRun {
  int problem = PROB_BFS;
  Layout lay{};
  Args a{};
  const void* parent = nullptr;
  const void* child = nullptr;
  int pgrid = 0, cgrid = 0, steps = kDefaultSteps;
  hipStream_t stream = nullptr;
};

dpo_status prepare_set(Runtime& r, int problem, const dpo_csr* g, const dpo_options& o,
                       int64_t slots, int32_t nq, void* out, void* ws, size_t ws_bytes,
                       void* stream, bool count_stats, SetRun* sr) {
  if (slots < 1 || slots > INT32_MAX || nq < 1 || nq > MAX_QUERIES) return DPO_ERR_ARG;
  const Layout lay = layout_for(slots, nq, o);
  if (ws_bytes < lay.total) return DPO_ERR_WORKSPACE;
  const int gran = gran_of(o);
  sr->problem = problem;
  sr->lay = lay;
  sr->parent = parent_kernel_ptr(problem, gran);
  sr->child = gran == AGG_FLAT ? nullptr : child_kernel_ptr(problem);
  if (!sr->parent) return DPO_ERR_UNSUPPORTED;
  char* base = (char*)ws;
  Args& a = sr->a;
  std::memset(&a, 0, sizeof(a));  // padding too: cached graphs are keyed by these bytes
  a.rp = g->row_ptr;
  a.col = g->col_idx;
  a.w = g->weights;
  a.level = problem == PROB_BFS ? (int32_t*)out : nullptr;
  a.dist = problem == PROB_SSSP ? (uint32_t*)out : nullptr;
  a.st = (State*)(base + lay.state);
  a.q = (Query*)(base + lay.queries);
  a.grp_packed = (unsigned long long*)(base + lay.grp_packed);
  a.grp_done = (uint32_t*)(base + lay.grp_done);
  a.front0 = (int32_t*)(base + lay.front0);
  a.front1 = (int32_t*)(base + lay.front1);
  a.visit = (uint32_t*)(base + lay.visit);
  a.rec = (int4*)(base + lay.rec);
  a.rec_q = (int32_t*)(base + lay.rec_q);
  a.desc = (int4*)(base + lay.desc);
  a.stats = (unsigned long long*)(base + lay.stats);
  a.slots = (int32_t)slots;
  a.m = g->m;
  a.nq = nq;
  a.CB = o.child_block;
  a.k = (gran == AGG_MULTI) ? o.agg_blocks : 1;
  a.ngroups_cap = lay.ngroups_cap;
  a.desc_cap = lay.desc_cap;
  a.fcap = lay.fcap;
  a.count_stats = count_stats ? 1 : 0;
  sr->pgrid = persistent_grid(r, sr->parent, parent_shmem(nq));
  sr->cgrid = sr->child ? persistent_grid(r, sr->child) : 0;
  sr->steps = o.steps_per_replay ? o.steps_per_replay : kDefaultSteps;
  sr->stream = (hipStream_t)stream;
  return DPO_OK;
}

int init_grid(Runtime& r, int64_t work) {
  int64_t gsz = cdiv(std::max<int64_t>(work, (int64_t)MAX_GRID * NSTAT), PB);
  if (gsz > 4 * r.cu_count) gsz = 4 * r.cu_count;
  return (int)std::max<int64_t>(gsz, 1);
}

// Upload host query records [q_first, q_first + count) and start them.
dpo_status admit(Runtime& r, SetRun& sr, const Query* hq, int32_t q_first, int32_t count,
                 int32_t reset, int64_t work) {
  if (count <= 0) return DPO_OK;
  if (hipMemcpyAsync(sr.a.q + q_first, hq + q_first, (size_t)count * sizeof(Query),
                     hipMemcpyHostToDevice, sr.stream) != hipSuccess)
    return DPO_ERR_HIP;
  void* p1[] = {&sr.a, &q_first, &count, &reset};
  if (hipLaunchKernel(admit_kernel_ptr(sr.problem), dim3(init_grid(r, work)), dim3(PB), p1, 0,
                      sr.stream) != hipSuccess)
    return DPO_ERR_HIP;
  void* p2[] = {&sr.a, &q_first, &count};
  if (hipLaunchKernel(admit_sources_kernel_ptr(), dim3((unsigned)cdiv(count, PB)), dim3(PB), p2, 0,
                      sr.stream) != hipSuccess)
    return DPO_ERR_HIP;
  return DPO_OK;
}

dpo_status start_set(Runtime& r, SetRun& sr) {
  void* p[] = {&sr.a};
  if (hipLaunchKernel(init_kernel_ptr(sr.problem), dim3(init_grid(r, sr.lay.ngroups_cap)), dim3(PB),
                      p, 0, sr.stream) != hipSuccess)
    return DPO_ERR_HIP;
  return DPO_OK;
}

// One replay of K level steps; reads back base, done, error, levels_run.
dpo_status replay(Runtime& r, SetRun& sr, hipGraphExec_t exec) {
  if (hipGraphLaunch(exec, sr.stream) != hipSuccess) return DPO_ERR_HIP;
  if (hipMemcpyAsync(r.host_flags, sr.a.st, 16, hipMemcpyDeviceToHost, sr.stream) != hipSuccess)
    return DPO_ERR_HIP;
  if (hipStreamSynchronize(sr.stream) != hipSuccess) return DPO_ERR_HIP;
  if (r.host_flags[2] != 0) return (dpo_status)(-(int32_t)r.host_flags[2]);
  return DPO_OK;
}

// Runs replays until every query has finished.
dpo_status run_to_completion(Runtime& r, SetRun& sr, int64_t max_levels) {
  hipGraphExec_t exec;
  dpo_status s = get_exec(r, sr.parent, sr.child, sr.pgrid, sr.cgrid, sr.steps, sr.a, &exec);
  if (s != DPO_OK) return s;
  const int64_t max_replays = max_levels / sr.steps + 2;
  for (int64_t rep = 0; rep < max_replays; ++rep) {
    s = replay(r, sr, exec);
    if (s != DPO_OK) return s;
    if (r.host_flags[1]) return DPO_OK;
  }
  return DPO_ERR_TIMEOUT;
}

dpo_status read_stats(Runtime& r, SetRun& sr, dpo_stats* st) {
  if (!st) return DPO_OK;
  if (hipMemcpyAsync(r.host_stats, sr.a.stats, (size_t)MAX_GRID * NSTAT * 8, hipMemcpyDeviceToHost,
                     sr.stream) != hipSuccess ||
      hipMemcpyAsync(r.host_flags, sr.a.st, 16, hipMemcpyDeviceToHost, sr.stream) != hipSuccess ||
      hipStreamSynchronize(sr.stream) != hipSuccess)
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
  return DPO_OK;
}

dpo_status traverse(int problem, const dpo_csr* g, int32_t source, const dpo_options* o,
                    void* out, void* ws, size_t ws_bytes, void* stream, dpo_stats* st) {
  if (!o || !out || !ws) return DPO_ERR_ARG;
  dpo_status s = check_graph(g, problem == PROB_SSSP);
  if (s != DPO_OK) return s;
  s = check_options(*o);
  if (s != DPO_OK) return s;
  if (problem == PROB_SSSP && g->n > 16843009) return DPO_ERR_ARG;
  if (source < 0 || source >= g->n) return DPO_ERR_SOURCE;
  if (ws_bytes < layout_for(round32(g->n), 1, *o).total) return DPO_ERR_WORKSPACE;
  Runtime& r = rt();
  std::lock_guard<std::mutex> lock(r.mu);
  s = ensure_runtime(r);
  if (s != DPO_OK) return s;
  SetRun sr;
  s = prepare_set(r, problem, g, *o, round32(g->n), 1, out, ws, ws_bytes, stream, st != nullptr, &sr);
  if (s != DPO_OK) return s;
  Query* hq = r.host_q;
  hq[0] = Query{0, g->n, 0, 0, o->threshold, o->coarsen, 0, source};
  if ((s = start_set(r, sr)) != DPO_OK) return s;
  if ((s = admit(r, sr, hq, 0, 1, 0, g->n)) != DPO_OK) return s;
  if ((s = run_to_completion(r, sr, g->n)) != DPO_OK) return s;
  return read_stats(r, sr, st);
}

dpo_status check_arena(const dpo_arena* ar, bool need_w) {
  if (!ar || ar->ngraphs < 1 || !ar->graph_vbase) return DPO_ERR_ARG;
  dpo_status s = check_graph(&ar->csr, need_w);
  if (s != DPO_OK) return s;
  if (ar->graph_vbase[0] != 0 || ar->graph_vbase[ar->ngraphs] != ar->csr.n) return DPO_ERR_ARG;
  for (int32_t g = 0; g < ar->ngraphs; ++g)
    if (ar->graph_vbase[g + 1] <= ar->graph_vbase[g]) return DPO_ERR_ARG;
  return DPO_OK;
}

// Output slots of a batch: query q occupies [slot0[q], slot0[q] + n_{graph(q)}),
// slot0 32-aligned, in query order.  Returns the total, or -1 on bad input.
int64_t batch_slots(const dpo_arena* ar, const dpo_query* qs, int32_t nq, int64_t* slot0) {
  int64_t tot = 0;
  for (int32_t i = 0; i < nq; ++i) {
    const int32_t g = qs[i].graph;
    if (g < 0 || g >= ar->ngraphs) return -1;
    if (slot0) slot0[i] = tot;
    tot += round32(ar->graph_vbase[g + 1] - ar->graph_vbase[g]);
  }
  if (slot0) slot0[nq] = tot;
  return tot;
}

dpo_status traverse_batch(int problem, const dpo_arena* ar, const dpo_query* qs, int32_t nq,
                          const dpo_options* bopts, int32_t nb, void* out, void* ws,
                          size_t ws_bytes, void* stream, dpo_stats* st) {
  if (!qs || !bopts || nb < 1 || !out || !ws || nq < 1 || nq > MAX_QUERIES) return DPO_ERR_ARG;
  dpo_status s = check_arena(ar, problem == PROB_SSSP);
  if (s != DPO_OK) return s;
  for (int32_t b = 0; b < nb; ++b)
    if ((s = check_options(bopts[b])) != DPO_OK) return s;
  if (problem == PROB_SSSP && ar->csr.n > 16843009) return DPO_ERR_ARG;
  const int64_t slots = batch_slots(ar, qs, nq, nullptr);
  if (slots < 0) return DPO_ERR_ARG;
  int64_t max_n = 0;
  for (int32_t i = 0; i < nq; ++i) {
    const int32_t g = qs[i].graph;
    const int32_t n = ar->graph_vbase[g + 1] - ar->graph_vbase[g];
    if (qs[i].source < 0 || qs[i].source >= n) return DPO_ERR_SOURCE;
    if (qs[i].bucket < 0 || qs[i].bucket >= nb) return DPO_ERR_ARG;
    max_n = std::max<int64_t>(max_n, n);
  }
  if (ws_bytes < layout_for(slots, nq, bopts[0]).total) return DPO_ERR_WORKSPACE;
  Runtime& r = rt();
  std::lock_guard<std::mutex> lock(r.mu);
  s = ensure_runtime(r);
  if (s != DPO_OK) return s;
  SetRun sr;
  s = prepare_set(r, problem, &ar->csr, bopts[0], slots, nq, out, ws, ws_bytes, stream,
                  st != nullptr, &sr);
  if (s != DPO_OK) return s;
  Query* hq = r.host_q;
  int64_t slot = 0;
  for (int32_t i = 0; i < nq; ++i) {
    const int32_t g = qs[i].graph;
    const int32_t n = ar->graph_vbase[g + 1] - ar->graph_vbase[g];
    const dpo_options& bo = bopts[qs[i].bucket];
    hq[i] = Query{(int32_t)slot, n, ar->graph_vbase[g], 0, bo.threshold, bo.coarsen, 0,
                  qs[i].source};
    slot += round32(n);
  }
  if ((s = start_set(r, sr)) != DPO_OK) return s;
  if ((s = admit(r, sr, hq, 0, nq, 0, max_n)) != DPO_OK) return s;
  if ((s = run_to_completion(r, sr, slots)) != DPO_OK) return s;
  return read_stats(r, sr, st);
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
  return dpo::layout_for(dpo::round32(g->n), 1, *o).total;
}

int64_t dpo_batch_slots(const dpo_arena* ar, const dpo_query* q, int32_t nq, int64_t* slot0) {
  if (!q || nq < 1 || dpo::check_arena(ar, false) != DPO_OK) return -1;
  return dpo::batch_slots(ar, q, nq, slot0);
}

size_t dpo_batch_workspace_bytes(const dpo_arena* ar, const dpo_query* q, int32_t nq,
                                 const dpo_options* o) {
  if (!o || dpo::check_options(*o) != DPO_OK || nq < 1 || nq > dpo::MAX_QUERIES) return 0;
  const int64_t slots = dpo_batch_slots(ar, q, nq, nullptr);
  if (slots < 1) return 0;
  return dpo::layout_for(slots, nq, *o).total;
}

dpo_status dpo_bfs_batch(const dpo_arena* ar, const dpo_query* q, int32_t nq,
                         const dpo_options* bucket_opts, int32_t nbuckets, int32_t* levels,
                         void* ws, size_t ws_bytes, void* stream, dpo_stats* st) {
  return dpo::traverse_batch(dpo::PROB_BFS, ar, q, nq, bucket_opts, nbuckets, levels, ws, ws_bytes,
                             stream, st);
}

dpo_status dpo_sssp_batch(const dpo_arena* ar, const dpo_query* q, int32_t nq,
                          const dpo_options* bucket_opts, int32_t nbuckets, uint32_t* dist,
                          void* ws, size_t ws_bytes, void* stream, dpo_stats* st) {
  return dpo::traverse_batch(dpo::PROB_SSSP, ar, q, nq, bucket_opts, nbuckets, dist, ws, ws_bytes,
                             stream, st);
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
