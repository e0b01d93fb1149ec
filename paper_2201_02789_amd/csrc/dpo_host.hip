// Host driver and C ABI of the nested-parallel BFS / SSSP library.
//
// A traversal is: one init kernel, then HIP-graph replays of K captured level
// steps (the step kernel reads its level, frontier and counters from the
// workspace, so one instantiated graph serves every call with the same
// arguments), with one stream synchronisation per replay to read the done
// flag.  Instantiated graphs are cached by their exact kernel arguments.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <deque>
#include <map>
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
  size_t state, queries, qlist, qmap, grp_packed, grp_done, front0, front1, visit, dist2, rec, rec_q,
      rec_slot, ser, desc, stats, sercnt, total;
  int32_t ngroups_cap, desc_cap, fcap;
};

int64_t cdiv(int64_t a, int64_t b) { return (a + b - 1) / b; }
int64_t round32(int64_t x) { return (x + 31) & ~(int64_t)31; }

// Byte offset of the found bytes in the visit region (BFS: after the two
// bitmaps and the per-XCD copies)
size_t found_offset(int64_t slots) { return align_up((size_t)(2 + NHINT) * cdiv(slots, 32) * 4); }

int gran_of(const dpo_options& o) {
  if (o.mode == DPO_MODE_FLAT) return AGG_FLAT;
  switch (o.agg) {
    case DPO_AGG_NONE: return AGG_NONE;
    case DPO_AGG_WAVE: return AGG_WAVE;
    case DPO_AGG_BLOCK: return AGG_BLOCK;
    case DPO_AGG_MULTIBLOCK: return AGG_MULTI;
    case DPO_AGG_GRID: return AGG_MULTI;  // one group holding every virtual block
    default: return -1;
  }
}

// Blocks per multi-block group: agg_blocks, or every virtual block of the level
// for grid granularity.
int64_t group_blocks(const dpo_options& o, int64_t slots) {
  return o.agg == DPO_AGG_GRID ? std::max<int64_t>(cdiv(slots, PB), 1) : o.agg_blocks;
}


// Workspace for `slots` output slots (frontier entries) and `nq` queries.
Layout layout_for(int64_t slots, int32_t nq, const dpo_options& o) {
  Layout L{};
  const int gran = gran_of(o);
  const int64_t nvb = cdiv(slots, PB);
  const int64_t k = (gran == AGG_MULTI) ? group_blocks(o, slots) : 1;
  L.ngroups_cap = (gran == AGG_MULTI) ? (int32_t)cdiv(nvb, k) : 1;
  // descriptors per queue: virtual block vb publishes to queue vb % NQD
  // (multi-block group g to queue g % NQD)
  // an aggregation threshold lets every parent of a wave / block launch alone
  const bool solo = o.agg_threshold > 0 && (gran == AGG_WAVE || gran == AGG_BLOCK);
  switch (solo ? AGG_NONE : gran) {
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
  L.qlist = off; off = align_up(off + (size_t)(2 * nq + 1) * 4);  // list + workgroup prefix
  L.qmap = off; off = align_up(off + (size_t)cdiv(slots, 32) * 4);
  L.grp_packed = off; off = align_up(off + 3 * (size_t)L.ngroups_cap * 8);
  L.grp_done = off; off = align_up(off + 3 * (size_t)L.ngroups_cap * 4);
  L.front0 = off; off = align_up(off + fslots * 4);
  L.front1 = off; off = align_up(off + fslots * 4);
  // SSSP stamps / two BFS bitmaps and the NHINT per-XCD copies; then the found
  // bytes (which SSSP, having no stamps when it uses them, lets overlap these)
  L.visit = off; off = align_up(off + std::max((size_t)slots * 4, found_offset(slots) + (size_t)cdiv(slots, 32) * 32));
  L.dist2 = off; off = align_up(off + (size_t)slots * 4);  // SSSP second distance array
  L.rec = off; off = align_up(off + (size_t)slots * 16);
  L.rec_q = off; off = align_up(off + (size_t)slots * 4);
  L.rec_slot = off; off = align_up(off + (size_t)slots * 4);  // SSSP
  L.ser = off; off = align_up(off + (size_t)cdiv(slots, PB) * PB * 16);
  L.desc = off; off = align_up(off + (size_t)NQD * L.desc_cap * 16);
  L.stats = off; off = align_up(off + (size_t)MAX_GRID * NSTAT * 8);
  L.sercnt = off; off = align_up(off + (size_t)MAX_GRID * 4);
  L.total = off;
  return L;
}

dpo_status check_options(const dpo_options& o) {
  if (o.mode != DPO_MODE_NESTED && o.mode != DPO_MODE_FLAT) return DPO_ERR_ARG;
  if (o.threshold < 0) return DPO_ERR_ARG;
  if (o.coarsen != 1 && o.coarsen != 2 && o.coarsen != 4 && o.coarsen != 8 && o.coarsen != 16)
    return DPO_ERR_ARG;
  if (o.agg < DPO_AGG_NONE || o.agg > DPO_AGG_GRID) return DPO_ERR_ARG;
  if (o.agg_threshold < 0) return DPO_ERR_ARG;
  if (o.split_min < 0) return DPO_ERR_ARG;
  if (o.serial_wave != 0 && o.serial_wave != 1) return DPO_ERR_ARG;
  if (o.dyn_share < 0 || o.dyn_share > 100) return DPO_ERR_ARG;
  if (o.claim_hint < DPO_HINT_AUTO || o.claim_hint > DPO_HINT_OFF) return DPO_ERR_ARG;
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
  const void* third;
  const void* fourth;
  int pgrid, cgrid, tgrid, fgrid, steps;
  Args args;
  hipGraphExec_t exec;
  uint64_t last_use;
};

struct GridEntry {
  const void* first;
  int second;
  unsigned third;
};

constexpr int kMaxGridEntries = 64;

struct Runtime {
  std::mutex mu;
  std::vector<CachedGraph> graphs;
  uint64_t tick = 0;
  uint32_t* host_flags = nullptr;  // pinned: base, done, error, levels_run
  unsigned long long* host_stats = nullptr;  // pinned: MAX_GRID * NSTAT
  Query* host_q = nullptr;                   // pinned: MAX_QUERIES query records
  int32_t* host_list = nullptr;              // pinned: MAX_QUERIES query indices + prefix
  int cu_count = 0;
  // persistent grid sizes per kernel (fixed storage: the no-allocation entry
  // point uses them too)
  GridEntry grids[kMaxGridEntries];
  int ngrids = 0;
};

Runtime& rt() {
  static Runtime r;
  return r;
}

dpo_status hip_ok(hipError_t e) { return e == hipSuccess ? DPO_OK : DPO_ERR_HIP; }

// Compute-unit count of the current device (no allocation).
dpo_status ensure_device(Runtime& r) {
  if (r.cu_count > 0) return DPO_OK;
  int dev = 0;
  if (hipGetDevice(&dev) != hipSuccess) return DPO_ERR_HIP;
  if (hipDeviceGetAttribute(&r.cu_count, hipDeviceAttributeMultiprocessorCount, dev) != hipSuccess)
    return DPO_ERR_HIP;
  return DPO_OK;
}

dpo_status ensure_runtime(Runtime& r) {
  if (r.host_flags) return DPO_OK;
  if (ensure_device(r) != DPO_OK) return DPO_ERR_HIP;
  void* p = nullptr;
  const size_t qbytes = (size_t)MAX_QUERIES * (sizeof(Query) + 8) + 4;
  if (hipHostMalloc(&p, 256 + (size_t)MAX_GRID * NSTAT * 8 + qbytes, hipHostMallocDefault) !=
      hipSuccess)
    return DPO_ERR_HIP;
  r.host_flags = (uint32_t*)p;
  r.host_stats = (unsigned long long*)((char*)p + 256);
  r.host_q = (Query*)((char*)p + 256 + (size_t)MAX_GRID * NSTAT * 8);
  r.host_list = (int32_t*)(r.host_q + MAX_QUERIES);
  return DPO_OK;
}

// Persistent grid: as many workgroups as can be resident at once.
int persistent_grid(Runtime& r, const void* kernel, unsigned shmem = 0) {
  for (int i = 0; i < r.ngrids; ++i)
    if (r.grids[i].first == kernel && r.grids[i].third == shmem) return r.grids[i].second;
  int per_cu = 0;
  if (hipOccupancyMaxActiveBlocksPerMultiprocessor(&per_cu, kernel, PB, shmem) != hipSuccess ||
      per_cu < 1)
    per_cu = 1;
  if (per_cu > 8) per_cu = 8;
  int grid = per_cu * r.cu_count;
  if (grid > MAX_GRID) grid = MAX_GRID;
  if (r.ngrids < kMaxGridEntries) r.grids[r.ngrids++] = GridEntry{kernel, grid, shmem};
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

// K level steps (parent kernel, then child kernel unless flat, then the third
// kernel if any: SSSP's thresholded children, on the parent kernel's grid, or
// BFS's harvest; then the fourth if any: SSSP's harvest) and the advance of the
// level base, as one instantiated graph.
dpo_status get_exec(Runtime& r, const void* parent, const void* child, const void* third,
                    const void* fourth, int pgrid, int cgrid, int tgrid, int fgrid, int steps,
                    const Args& args, hipGraphExec_t* out, bool cached = true) {
  for (auto& e : r.graphs) {
    if (!cached) break;
    if (e.parent == parent && e.child == child && e.third == third && e.fourth == fourth &&
        e.pgrid == pgrid && e.cgrid == cgrid && e.tgrid == tgrid && e.fgrid == fgrid &&
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
    if (s == DPO_OK && third) s = add_node(graph, &prev, third, tgrid, PB, params);
    if (s == DPO_OK && fourth) s = add_node(graph, &prev, fourth, fgrid, PB, params);
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
  if (!cached) {  // owned by the caller
    *out = exec;
    return DPO_OK;
  }
  if ((int)r.graphs.size() >= kMaxCachedGraphs) {
    size_t victim = 0;
    for (size_t i = 1; i < r.graphs.size(); ++i)
      if (r.graphs[i].last_use < r.graphs[victim].last_use) victim = i;
    (void)hipGraphExecDestroy(r.graphs[victim].exec);
    r.graphs.erase(r.graphs.begin() + victim);
  }
  r.graphs.push_back(
      CachedGraph{parent, child, third, fourth, pgrid, cgrid, tgrid, fgrid, steps, args, exec,
                  ++r.tick});
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
  // after the child kernel: SSSP's thresholded children, or BFS's harvest
  // (per-XCD copies); then SSSP's harvest (found bytes)
  const void* third = nullptr;
  const void* fourth = nullptr;
  int pgrid = 0, cgrid = 0, tgrid = 0, fgrid = 0, steps = kDefaultSteps;
  hipStream_t stream = nullptr;
  int32_t* qlist = nullptr;  // device: indices of the queries being admitted
};

// tm: phase-timing rows; non-null selects the timed instantiations of the
// level kernels, run at the grid sizes of the product ones (same schedule).
dpo_status prepare_set(Runtime& r, int problem, const dpo_csr* g, const dpo_options& o,
                       int64_t slots, int32_t nq, void* out, void* ws, size_t ws_bytes,
                       void* stream, bool count_stats, SetRun* sr,
                       unsigned long long* tm = nullptr, bool batch_call = false) {
  if (slots < 1 || slots > INT32_MAX || nq < 1 || nq > MAX_QUERIES) return DPO_ERR_ARG;
  const Layout lay = layout_for(slots, nq, o);
  if (ws_bytes < lay.total) return DPO_ERR_WORKSPACE;
  const int gran = gran_of(o);
  sr->problem = problem;
  sr->lay = lay;
  // Found bytes and the harvest (BFS: with per-XCD copies): single traversals
  // and the serving engine (not a batch call) on graphs whose average degree
  // is at least HINT_AUTO_MIN_DEGREE, unless the options say otherwise.  The
  // harvest adds a kernel launch to every level step; a graph of low average
  // degree runs many narrow levels and rarely a wide one.
  const bool dense = g->m >= (int64_t)HINT_AUTO_MIN_DEGREE * g->n;
  const bool hint = o.claim_hint == DPO_HINT_ON ||
                    (o.claim_hint == DPO_HINT_AUTO && !batch_call && dense);
  const bool bfs = problem == PROB_BFS;
  sr->parent = parent_kernel_ptr(problem, gran);
  sr->child = gran == AGG_FLAT ? nullptr : child_kernel_ptr(problem, false, hint);
  sr->third = bfs ? (hint ? harvest_kernel_ptr(problem) : nullptr) : serial_kernel_ptr(problem, gran);
  sr->fourth = !bfs && hint ? harvest_kernel_ptr(problem) : nullptr;
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
  // SSSP with found bytes has no iteration stamps: the bytes overlap them
  a.found = (uint8_t*)(base + lay.visit + found_offset(slots));
  a.dist2 = problem == PROB_SSSP ? (uint32_t*)(base + lay.dist2) : nullptr;
  a.vwords = (int32_t)cdiv(slots, 32);
  a.rec = (int4*)(base + lay.rec);
  a.rec_q = (int32_t*)(base + lay.rec_q);
  a.rec_slot = (int32_t*)(base + lay.rec_slot);
  a.ser = (int4*)(base + lay.ser);
  a.qmap = (int32_t*)(base + lay.qmap);
  a.desc = (int4*)(base + lay.desc);
  a.stats = (unsigned long long*)(base + lay.stats);
  a.sercnt = (uint32_t*)(base + lay.sercnt);
  a.slots = (int32_t)slots;
  a.m = g->m;
  a.nq = nq;
  a.CB = o.child_block;
  a.k = (gran == AGG_MULTI) ? (int32_t)group_blocks(o, slots) : 1;
  a.agg_threshold = o.agg_threshold;
  a.split_min = o.split_min;
  a.serial_wave = o.serial_wave;
  a.dyn_pct = o.dyn_share;
  a.hint = hint ? 1 : 0;
  a.ngroups_cap = lay.ngroups_cap;
  a.desc_cap = lay.desc_cap;
  a.fcap = lay.fcap;
  a.count_stats = count_stats ? 1 : 0;
  sr->qlist = (int32_t*)(base + lay.qlist);
  sr->pgrid = persistent_grid(r, sr->parent);
  // the thresholded children's kernel walks the lists of the parent kernel's
  // workgroups: one grid for both, all of it resident in either
  if (sr->third && !bfs) sr->pgrid = std::min(sr->pgrid, persistent_grid(r, sr->third));
  sr->cgrid = sr->child ? persistent_grid(r, sr->child) : 0;
  // the harvest: as many workgroups as its rounds need, at most the parent
  // grid (a small graph's many narrow levels launch it empty)
  const int hgrid = (int)std::min<int64_t>(sr->pgrid, cdiv(slots, (int64_t)PB * HARVEST_RUNS));
  sr->tgrid = !sr->third ? 0 : bfs ? hgrid : sr->pgrid;
  sr->fgrid = sr->fourth ? hgrid : 0;
  sr->steps = o.steps_per_replay ? o.steps_per_replay : kDefaultSteps;
  sr->stream = (hipStream_t)stream;
  if (tm) {
    sr->parent = parent_kernel_ptr(problem, gran, true);
    sr->child = sr->child ? child_kernel_ptr(problem, true, hint) : nullptr;
    sr->third = bfs ? (hint ? harvest_kernel_ptr(problem, true) : nullptr)
                    : serial_kernel_ptr(problem, gran, true);
    sr->fourth = !bfs && hint ? harvest_kernel_ptr(problem, true) : nullptr;
    // a timed kernel that needs more registers than its product one runs on
    // the grid that is resident at its own occupancy (a larger grid would run
    // in two rounds and time the second round's wait as work)
    sr->pgrid = std::min(sr->pgrid, persistent_grid(r, sr->parent));
    if (sr->third && !bfs) sr->pgrid = std::min(sr->pgrid, persistent_grid(r, sr->third));
    if (sr->child) sr->cgrid = std::min(sr->cgrid, persistent_grid(r, sr->child));
    sr->tgrid = !sr->third ? 0 : !bfs ? sr->pgrid
                : std::min(sr->tgrid, persistent_grid(r, sr->third));
    if (sr->fourth) sr->fgrid = std::min(sr->fgrid, persistent_grid(r, sr->fourth));
    a.tm = tm;
  }
  return DPO_OK;
}

int init_grid(Runtime& r, int64_t work) {
  int64_t gsz = cdiv(std::max<int64_t>(work, (int64_t)MAX_GRID * NSTAT), PB);
  if (gsz > 4 * r.cu_count) gsz = 4 * r.cu_count;
  return (int)std::max<int64_t>(gsz, 1);
}

// Admit workgroups: hlist[count + k] = first workgroup of query hlist[k]
// (one per ADMIT_CHUNK of its slots, at least one); returns the total.
int32_t admit_prefix(const Query* hq, int32_t* hlist, int32_t count) {
  int32_t* pre = hlist + count;
  int64_t t = 0;
  for (int32_t k = 0; k < count; ++k) {
    pre[k] = (int32_t)t;
    t += std::max<int64_t>(1, cdiv(hq[hlist[k]].n, ADMIT_CHUNK));
  }
  pre[count] = (int32_t)t;
  return (int32_t)t;
}

dpo_status launch_admit(SetRun& sr, int32_t* hlist, int32_t count, int32_t reset, int32_t groups) {
  if (hipMemcpyAsync(sr.qlist, hlist, (size_t)(2 * count + 1) * 4, hipMemcpyHostToDevice,
                     sr.stream) != hipSuccess)
    return DPO_ERR_HIP;
  int32_t* dl = sr.qlist;
  void* p1[] = {&sr.a, &dl, &count, &reset};
  if (hipLaunchKernel(admit_kernel_ptr(sr.problem), dim3((unsigned)groups), dim3(PB), p1, 0,
                      sr.stream) != hipSuccess)
    return DPO_ERR_HIP;
  void* p2[] = {&sr.a, &dl, &count};
  if (hipLaunchKernel(admit_sources_kernel_ptr(), dim3((unsigned)cdiv(count, PB)), dim3(PB), p2, 0,
                      sr.stream) != hipSuccess)
    return DPO_ERR_HIP;
  return DPO_OK;
}

// Start the queries hlist[0 .. count) whose records are already in hq (host,
// pinned; hlist has room for 2 * count + 1 entries): upload those records,
// the index list and the workgroup prefix, then the admit kernels.
dpo_status admit(Runtime& r, SetRun& sr, const Query* hq, int32_t* hlist, int32_t count,
                 int32_t reset) {
  (void)r;
  if (count <= 0) return DPO_OK;
  for (int32_t k = 0; k < count; ++k)
    if (hipMemcpyAsync(sr.a.q + hlist[k], hq + hlist[k], sizeof(Query), hipMemcpyHostToDevice,
                       sr.stream) != hipSuccess)
      return DPO_ERR_HIP;
  return launch_admit(sr, hlist, count, reset, admit_prefix(hq, hlist, count));
}

// Batch start: the whole table in one upload, then the admit kernels.
dpo_status admit_all(Runtime& r, SetRun& sr, const Query* hq, int32_t* hlist, int32_t nq) {
  (void)r;
  if (hipMemcpyAsync(sr.a.q, hq, (size_t)nq * sizeof(Query), hipMemcpyHostToDevice, sr.stream) !=
      hipSuccess)
    return DPO_ERR_HIP;
  return launch_admit(sr, hlist, nq, 0, admit_prefix(hq, hlist, nq));
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
  dpo_status s =
      get_exec(r, sr.parent, sr.child, sr.third, sr.fourth, sr.pgrid, sr.cgrid, sr.tgrid, sr.fgrid,
               sr.steps, sr.a, &exec);
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
                    void* out, void* ws, size_t ws_bytes, void* stream, dpo_stats* st,
                    unsigned long long* tm = nullptr) {
  if (!o || !out || !ws) return DPO_ERR_ARG;
  dpo_status s = check_graph(g, problem == PROB_SSSP);
  if (s != DPO_OK) return s;
  s = check_options(*o);
  if (s != DPO_OK) return s;
  if (source < 0 || source >= g->n) return DPO_ERR_SOURCE;
  if (ws_bytes < layout_for(round32(g->n), 1, *o).total) return DPO_ERR_WORKSPACE;
  Runtime& r = rt();
  std::lock_guard<std::mutex> lock(r.mu);
  s = ensure_runtime(r);
  if (s != DPO_OK) return s;
  SetRun sr;
  s = prepare_set(r, problem, g, *o, round32(g->n), 1, out, ws, ws_bytes, stream, st != nullptr, &sr,
                  tm);
  if (s != DPO_OK) return s;
  if (tm && hipMemsetAsync(tm, 0, DPO_TIMING_BYTES, sr.stream) != hipSuccess) return DPO_ERR_HIP;
  Query* hq = r.host_q;
  hq[0] = Query{0, g->n, 0, 0, o->threshold, o->coarsen, 0, source};
  int32_t* hl = r.host_list;
  hl[0] = 0;
  if ((s = start_set(r, sr)) != DPO_OK) return s;
  if ((s = admit(r, sr, hq, hl, 1, 0)) != DPO_OK) return s;
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
  const int64_t slots = batch_slots(ar, qs, nq, nullptr);
  if (slots < 0) return DPO_ERR_ARG;
  for (int32_t i = 0; i < nq; ++i) {
    const int32_t g = qs[i].graph;
    const int32_t n = ar->graph_vbase[g + 1] - ar->graph_vbase[g];
    if (qs[i].source < 0 || qs[i].source >= n) return DPO_ERR_SOURCE;
    if (qs[i].bucket < 0 || qs[i].bucket >= nb) return DPO_ERR_ARG;
  }
  if (ws_bytes < layout_for(slots, nq, bopts[0]).total) return DPO_ERR_WORKSPACE;
  Runtime& r = rt();
  std::lock_guard<std::mutex> lock(r.mu);
  s = ensure_runtime(r);
  if (s != DPO_OK) return s;
  SetRun sr;
  s = prepare_set(r, problem, &ar->csr, bopts[0], slots, nq, out, ws, ws_bytes, stream,
                  st != nullptr, &sr, nullptr, /*batch_call=*/true);
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
  int32_t* hl = r.host_list;
  for (int32_t i = 0; i < nq; ++i) hl[i] = i;
  if ((s = start_set(r, sr)) != DPO_OK) return s;
  if ((s = admit_all(r, sr, hq, hl, nq)) != DPO_OK) return s;
  if ((s = run_to_completion(r, sr, slots)) != DPO_OK) return s;
  return read_stats(r, sr, st);
}


// ------------------------------------------------------------ no allocation
// Workspace of dpo_bfs_noalloc: a static device array that every GPU the
// library runs on holds until the process ends.  Host code never passes the
// array's name to a kernel (on the host it is only a stand-in for the
// symbol); it uses the device address that hipGetSymbolAddress returns, kept
// per device.
static __device__ __align__(256) unsigned char scratch[DPO_NOALLOC_SCRATCH_BYTES];

constexpr int kMaxDevices = 64;
void* g_scratch_ptr[kMaxDevices];  // device address of `scratch` per device (under r.mu)

dpo_status scratch_of_current_device(void** out) {
  int dev = 0;
  if (hipGetDevice(&dev) != hipSuccess || dev < 0 || dev >= kMaxDevices) return DPO_ERR_HIP;
  if (!g_scratch_ptr[dev]) {
    void* p = nullptr;
    if (hipGetSymbolAddress(&p, HIP_SYMBOL(scratch)) != hipSuccess || !p) return DPO_ERR_HIP;
    g_scratch_ptr[dev] = p;
  }
  *out = g_scratch_ptr[dev];
  return DPO_OK;
}

// One level step launched kernel by kernel (no HIP graph: instantiating one
// allocates).
dpo_status launch_step(SetRun& sr, uint32_t step) {
  void* p[] = {&sr.a, &step};
  if (hipLaunchKernel(sr.parent, dim3((unsigned)sr.pgrid), dim3(PB), p, 0, sr.stream) != hipSuccess)
    return DPO_ERR_HIP;
  if (sr.child &&
      hipLaunchKernel(sr.child, dim3((unsigned)sr.cgrid), dim3(PB), p, 0, sr.stream) != hipSuccess)
    return DPO_ERR_HIP;
  if (sr.third &&
      hipLaunchKernel(sr.third, dim3((unsigned)sr.tgrid), dim3(PB), p, 0, sr.stream) != hipSuccess)
    return DPO_ERR_HIP;
  if (sr.fourth &&
      hipLaunchKernel(sr.fourth, dim3((unsigned)sr.fgrid), dim3(PB), p, 0, sr.stream) != hipSuccess)
    return DPO_ERR_HIP;
  return DPO_OK;
}

dpo_status traverse_noalloc(int problem, const dpo_csr* g, int32_t source, const dpo_options* o,
                            void* out, void* stream) {
  if (!o || !out) return DPO_ERR_ARG;
  dpo_status s = check_graph(g, problem == PROB_SSSP);
  if (s != DPO_OK) return s;
  if ((s = check_options(*o)) != DPO_OK) return s;
  if (source < 0 || source >= g->n) return DPO_ERR_SOURCE;
  // the static workspace bounds the graph size (checked before any HIP call)
  if (layout_for(round32(g->n), 1, *o).total > (size_t)DPO_NOALLOC_SCRATCH_BYTES)
    return DPO_ERR_WORKSPACE;
  Runtime& r = rt();
  std::lock_guard<std::mutex> lock(r.mu);
  if ((s = ensure_device(r)) != DPO_OK) return s;
  void* ws = nullptr;
  if ((s = scratch_of_current_device(&ws)) != DPO_OK) return s;
  SetRun sr;
  s = prepare_set(r, problem, g, *o, round32(g->n), 1, out, ws, DPO_NOALLOC_SCRATCH_BYTES, stream,
                  false, &sr);
  if (s != DPO_OK) return s;
  // the query record, its index and the admit prefix, from host stack memory
  // (copied by the runtime before hipMemcpyAsync returns)
  Query hq[1] = {Query{0, g->n, 0, 0, o->threshold, o->coarsen, 0, source}};
  int32_t hl[3] = {0, 0, 0};
  // init_kernel clears the state, the level sets, the group counters and the
  // statistics rows, and the admit kernels the outputs and visited state, so
  // nothing left in the array by an earlier call is read
  if ((s = start_set(r, sr)) != DPO_OK) return s;
  if ((s = admit(r, sr, hq, hl, 1, 0)) != DPO_OK) return s;
  uint32_t flags[4] = {0, 0, 0, 0};  // base, done, error, levels_run
  const int64_t max_replays = (int64_t)g->n / sr.steps + 2;
  State* st = sr.a.st;
  uint32_t k = (uint32_t)sr.steps;
  for (int64_t rep = 0; rep < max_replays; ++rep) {
    for (int i = 0; i < sr.steps; ++i)
      if ((s = launch_step(sr, (uint32_t)i)) != DPO_OK) return s;
    void* ap[] = {&st, &k};
    if (hipLaunchKernel(advance_kernel_ptr(), dim3(1), dim3(64), ap, 0, sr.stream) != hipSuccess)
      return DPO_ERR_HIP;
    if (hipMemcpyAsync(flags, st, sizeof(flags), hipMemcpyDeviceToHost, sr.stream) != hipSuccess ||
        hipStreamSynchronize(sr.stream) != hipSuccess)
      return DPO_ERR_HIP;
    if (flags[2] != 0) return (dpo_status)(-(int32_t)flags[2]);
    if (flags[1]) return DPO_OK;
  }
  return DPO_ERR_TIMEOUT;
}

// ------------------------------------------------------------ serving engine
// Continuous batching: queries are admitted at replay boundaries while
// others are running, as long as their output slots (footprint) and a query
// table entry are free; finished queries are retired and their slots reused.
struct Pending {
  uint64_t ticket;
  int32_t graph, source;
  void* out;
};

struct Running {
  bool used = false;
  uint64_t ticket = 0;
  void* out = nullptr;
  int32_t n = 0;
  int64_t slot0 = 0;
  int64_t footprint = 0;
};

}  // namespace
}  // namespace dpo

struct dpo_engine {
  int problem = dpo::PROB_BFS;
  dpo_csr csr{};
  std::vector<int32_t> vbase;
  std::vector<dpo_options> bopts;
  std::vector<int32_t> gbucket;
  dpo::SetRun sr;
  int32_t max_queries = 0;
  int64_t max_slots = 0;
  char* out_arena = nullptr;
  std::map<int64_t, int64_t> free_slots;  // start -> length, 32-aligned
  std::vector<dpo::Running> run;
  std::vector<int32_t> free_q;
  std::deque<dpo::Pending> pending;
  std::deque<uint64_t> completed;
  uint64_t next_ticket = 1;
  int32_t running = 0;
  bool inflight = false;
  hipGraphExec_t exec = nullptr;
  dpo::Query* hq = nullptr;   // pinned mirror of the device query table
  int32_t* hlist = nullptr;   // pinned
  uint32_t* hflags = nullptr; // pinned
  int64_t max_n = 0;
};

namespace dpo {
namespace {

bool slots_alloc(dpo_engine* e, int64_t len, int64_t* start) {
  for (auto it = e->free_slots.begin(); it != e->free_slots.end(); ++it) {
    if (it->second >= len) {
      *start = it->first;
      const int64_t rest = it->second - len;
      const int64_t nstart = it->first + len;
      e->free_slots.erase(it);
      if (rest > 0) e->free_slots[nstart] = rest;
      return true;
    }
  }
  return false;
}

void slots_free(dpo_engine* e, int64_t start, int64_t len) {
  auto it = e->free_slots.emplace(start, len).first;
  auto nx = std::next(it);
  if (nx != e->free_slots.end() && it->first + it->second == nx->first) {
    it->second += nx->second;
    e->free_slots.erase(nx);
  }
  if (it != e->free_slots.begin()) {
    auto pv = std::prev(it);
    if (pv->first + pv->second == it->first) {
      pv->second += it->second;
      e->free_slots.erase(it);
    }
  }
}

dpo_status engine_step(dpo_engine* e) {
  Runtime& r = rt();
  SetRun& sr = e->sr;
  dpo_status s = DPO_OK;
  if (e->inflight) {
    if (hipStreamSynchronize(sr.stream) != hipSuccess) return DPO_ERR_HIP;
    e->inflight = false;
    if (e->hflags[2] != 0) return (dpo_status)(-(int32_t)e->hflags[2]);
    // queries without frontier entries at the last level run have finished
    const int32_t last_level = (int32_t)e->hflags[0] - 1;
    const bool all_done = e->hflags[1] != 0;
    int32_t retired = 0;
    for (int32_t q = 0; q < e->max_queries; ++q) {
      Running& ru = e->run[q];
      if (!ru.used || !(all_done || e->hq[q].last < last_level)) continue;
      const size_t bytes = (size_t)ru.n * 4;
      if (hipMemcpyAsync(ru.out, e->out_arena + ru.slot0 * 4, bytes, hipMemcpyDeviceToDevice,
                         sr.stream) != hipSuccess)
        return DPO_ERR_HIP;
      slots_free(e, ru.slot0, ru.footprint);
      e->completed.push_back(ru.ticket);
      ru = Running{};
      e->free_q.push_back(q);
      --e->running;
      ++retired;
    }
    if (retired && hipStreamSynchronize(sr.stream) != hipSuccess) return DPO_ERR_HIP;
  }
  // admit in arrival order while a table entry and the footprint fit
  int32_t count = 0;
  const bool reset = e->running == 0;
  while (!e->pending.empty() && !e->free_q.empty()) {
    const Pending& p = e->pending.front();
    const int32_t n = e->vbase[p.graph + 1] - e->vbase[p.graph];
    int64_t slot0;
    if (!slots_alloc(e, round32(n), &slot0)) break;
    const int32_t q = e->free_q.back();
    e->free_q.pop_back();
    const dpo_options& bo = e->bopts[e->gbucket[p.graph]];
    e->hq[q] = Query{(int32_t)slot0, n, e->vbase[p.graph], 0, bo.threshold, bo.coarsen, 0,
                     p.source};
    Running& ru = e->run[q];
    ru.used = true;
    ru.ticket = p.ticket;
    ru.out = p.out;
    ru.n = n;
    ru.slot0 = slot0;
    ru.footprint = round32(n);
    e->hlist[count++] = q;
    ++e->running;
    e->pending.pop_front();
  }
  if (count) {
    if (reset) {
      // nothing was running: restart the level sets (and their counters)
      if ((s = start_set(r, sr)) != DPO_OK) return s;
    }
    if ((s = admit(r, sr, e->hq, e->hlist, count, 0)) != DPO_OK) return s;
  }
  if (e->running > 0) {
    if (hipGraphLaunch(e->exec, sr.stream) != hipSuccess) return DPO_ERR_HIP;
    if (hipMemcpyAsync(e->hflags, sr.a.st, 16, hipMemcpyDeviceToHost, sr.stream) != hipSuccess ||
        hipMemcpyAsync(e->hq, sr.a.q, (size_t)e->max_queries * sizeof(Query),
                       hipMemcpyDeviceToHost, sr.stream) != hipSuccess)
      return DPO_ERR_HIP;
    e->inflight = true;
  }
  return DPO_OK;
}

}  // namespace
}  // namespace dpo

extern "C" {

size_t dpo_engine_workspace_bytes(const dpo_options* o, int32_t max_queries, int64_t max_slots) {
  if (!o || dpo::check_options(*o) != DPO_OK || max_queries < 1 ||
      max_queries > dpo::MAX_QUERIES || max_slots < 32 || max_slots > INT32_MAX)
    return 0;
  return dpo::layout_for(dpo::round32(max_slots), max_queries, *o).total;
}

dpo_status dpo_engine_create(const dpo_arena* arena, int32_t kind, const dpo_options* bucket_opts,
                             int32_t nbuckets, const int32_t* graph_bucket, int32_t max_queries,
                             int64_t max_slots, void* ws, size_t ws_bytes, void* out_arena,
                             void* stream, dpo_engine** out) {
  using namespace dpo;
  if (!out || !bucket_opts || nbuckets < 1 || !ws || !out_arena || (kind != 0 && kind != 1))
    return DPO_ERR_ARG;
  *out = nullptr;
  const int problem = kind == 0 ? PROB_BFS : PROB_SSSP;
  dpo_status s = check_arena(arena, problem == PROB_SSSP);
  if (s != DPO_OK) return s;
  for (int32_t b = 0; b < nbuckets; ++b)
    if ((s = check_options(bucket_opts[b])) != DPO_OK) return s;
  if (max_queries < 1 || max_queries > MAX_QUERIES || max_slots < 32 || max_slots > INT32_MAX)
    return DPO_ERR_ARG;
  max_slots = round32(max_slots);
  if (ws_bytes < layout_for(max_slots, max_queries, bucket_opts[0]).total) return DPO_ERR_WORKSPACE;
  if (graph_bucket)
    for (int32_t g = 0; g < arena->ngraphs; ++g)
      if (graph_bucket[g] < 0 || graph_bucket[g] >= nbuckets) return DPO_ERR_ARG;
  Runtime& r = rt();
  std::lock_guard<std::mutex> lock(r.mu);
  if ((s = ensure_runtime(r)) != DPO_OK) return s;
  dpo_engine* e = new dpo_engine();
  e->problem = problem;
  e->csr = arena->csr;
  e->vbase.assign(arena->graph_vbase, arena->graph_vbase + arena->ngraphs + 1);
  e->bopts.assign(bucket_opts, bucket_opts + nbuckets);
  e->gbucket.assign(arena->ngraphs, 0);
  if (graph_bucket) e->gbucket.assign(graph_bucket, graph_bucket + arena->ngraphs);
  e->max_queries = max_queries;
  e->max_slots = max_slots;
  e->out_arena = (char*)out_arena;
  e->free_slots[0] = max_slots;
  e->run.assign(max_queries, Running{});
  for (int32_t q = max_queries - 1; q >= 0; --q) e->free_q.push_back(q);
  s = prepare_set(r, problem, &e->csr, bucket_opts[0], max_slots, max_queries, out_arena, ws,
                  ws_bytes, stream, false, &e->sr);
  void* p = nullptr;
  if (s == DPO_OK &&
      hipHostMalloc(&p, 64 + (size_t)max_queries * (sizeof(Query) + 8) + 4, hipHostMallocDefault) !=
          hipSuccess)
    s = DPO_ERR_HIP;
  if (s == DPO_OK) {
    e->hflags = (uint32_t*)p;
    e->hq = (Query*)((char*)p + 64);
    e->hlist = (int32_t*)(e->hq + max_queries);
    std::memset(e->hq, 0, (size_t)max_queries * sizeof(Query));
    s = get_exec(r, e->sr.parent, e->sr.child, e->sr.third, e->sr.fourth, e->sr.pgrid,
                 e->sr.cgrid, e->sr.tgrid, e->sr.fgrid, e->sr.steps, e->sr.a, &e->exec, false);
  }
  if (s == DPO_OK) s = start_set(r, e->sr);
  if (s == DPO_OK && e->sr.a.hint) {
    // no query has been admitted to any slot yet: no found vertex anywhere
    void* cp[] = {&e->sr.a};
    if (hipLaunchKernel(clear_found_kernel_ptr(), dim3(init_grid(r, max_slots / 4)), dim3(PB), cp,
                        0, e->sr.stream) != hipSuccess)
      s = DPO_ERR_HIP;
  }
  if (s == DPO_OK &&
      hipMemcpyAsync(e->sr.a.q, e->hq, (size_t)max_queries * sizeof(Query), hipMemcpyHostToDevice,
                     e->sr.stream) != hipSuccess)
    s = DPO_ERR_HIP;
  if (s == DPO_OK && hipStreamSynchronize(e->sr.stream) != hipSuccess) s = DPO_ERR_HIP;
  if (s != DPO_OK) {
    if (e->exec) (void)hipGraphExecDestroy(e->exec);
    if (p) (void)hipHostFree(p);
    delete e;
    return s;
  }
  *out = e;
  return DPO_OK;
}

dpo_status dpo_engine_submit(dpo_engine* e, int32_t graph, int32_t source, void* out,
                             uint64_t* ticket) {
  if (!e || !out || graph < 0 || graph >= (int32_t)e->vbase.size() - 1) return DPO_ERR_ARG;
  const int32_t n = e->vbase[graph + 1] - e->vbase[graph];
  if (source < 0 || source >= n) return DPO_ERR_SOURCE;
  if (dpo::round32(n) > e->max_slots) return DPO_ERR_CAPACITY;
  const uint64_t t = e->next_ticket++;
  e->pending.push_back(dpo::Pending{t, graph, source, out});
  if (ticket) *ticket = t;
  return DPO_OK;
}

dpo_status dpo_engine_step(dpo_engine* e, int32_t* running, int32_t* pending) {
  if (!e) return DPO_ERR_ARG;
  dpo::Runtime& r = dpo::rt();
  dpo_status s;
  {
    std::lock_guard<std::mutex> lock(r.mu);
    s = dpo::engine_step(e);
  }
  if (running) *running = e->running;
  if (pending) *pending = (int32_t)e->pending.size();
  return s;
}

int32_t dpo_engine_poll(dpo_engine* e, uint64_t* tickets, int32_t cap) {
  if (!e || !tickets || cap < 1) return 0;
  int32_t k = 0;
  while (k < cap && !e->completed.empty()) {
    tickets[k++] = e->completed.front();
    e->completed.pop_front();
  }
  return k;
}

void dpo_engine_destroy(dpo_engine* e) {
  if (!e) return;
  if (e->inflight) (void)hipStreamSynchronize(e->sr.stream);
  if (e->exec) (void)hipGraphExecDestroy(e->exec);
  if (e->hflags) (void)hipHostFree(e->hflags);
  delete e;
}

}  // extern "C"


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
  o->agg_threshold = 0;
  o->split_min = 65536;
  o->serial_wave = 1;
  o->dyn_share = 0;
  o->claim_hint = DPO_HINT_AUTO;
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

dpo_status dpo_bfs_noalloc(const dpo_csr* g, int32_t source, const dpo_options* o, int32_t* levels,
                           void* stream) {
  return dpo::traverse_noalloc(dpo::PROB_BFS, g, source, o, levels, stream);
}

dpo_status dpo_traverse_timed(int32_t kind, const dpo_csr* g, int32_t source, const dpo_options* o,
                              void* out, void* ws, size_t ws_bytes, void* stream, void* timing,
                              size_t timing_bytes) {
  if ((kind != 0 && kind != 1) || !timing || timing_bytes < (size_t)DPO_TIMING_BYTES)
    return DPO_ERR_ARG;
  return dpo::traverse(kind == 0 ? dpo::PROB_BFS : dpo::PROB_SSSP, g, source, o, out, ws, ws_bytes,
                       stream, nullptr, (unsigned long long*)timing);
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
