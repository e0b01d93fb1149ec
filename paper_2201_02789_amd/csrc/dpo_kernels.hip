// Device code: level-synchronous nested-parallel BFS / SSSP for gfx950.
//
// Each level is two kernels, the parent kernel and the child kernel; for SSSP
// the parent kernel's second pass (the thresholded children) runs as a third
// kernel after the child kernel, and with found bytes (single traversals, the
// serving engine) a harvest kernel ends the level.
//
// Parent kernel: the parent grid.  Workgroups (256 lanes = 4 wave64) take
// virtual parent blocks of 256 frontier entries in a grid-stride loop; lane i
// is the parent thread of frontier vertex u with child-thread count deg(u)
// (Sec. III-D):
//
//   deg == 0            nothing to do
//   0 < deg < T         thresholding (Sec. III-B): the parent runs the child
//                       body for each neighbour itself, serially
//   deg >= max(T, 1)    launch: gDim = ceil(deg / CB) original child blocks,
//                       coarsened to ceil(gDim / CF) blocks (Sec. IV-B); the
//                       parent writes a launch record {row start, deg, scanned
//                       offset, parent value} and takes part in aggregation
//
// Aggregation (Sec. II-B, V-A) fuses the child grids of a group of parents
// into one grid: an exclusive scan of the coarsened grid sizes gives each
// record its offset.  Granularities: none (each parent publishes its own
// grid), wave (64 parents), block (256 parents) and multi-block (k blocks).
// Multi-block groups take their record slot and offset from one packed 64-bit
// atomic per group (hi = records, lo = child blocks; Sec. V-A increments both
// counters as one integer), pre-aggregated per block; a group-wide done
// counter picks the last block, which publishes the aggregated grid.
//
// HIP has no device-side launch.  "Publishing" appends a descriptor {record
// base, record count, child-block base} to one of eight queues through a
// packed 64-bit counter (hi = descriptors, lo = child blocks), so block bases
// grow with the descriptor index.  The launch itself is the stream-ordered
// child kernel that follows: the kernel boundary makes records visible
// without the release/acquire fences an in-kernel hand-off would need.
//
// Child kernel: the aggregated child grids.  Workgroup w runs a contiguous
// share of the child blocks, finds the parent of its first block by 64-ary
// wave searches of the descriptor bases and the scanned record offsets (the
// disaggregation of Sec. V-A), then advances along the scanned offsets.  Each
// coarsened block runs the coarsening loop over CF original blocks of CB lanes
// (Sec. IV-B) with coalesced col_idx reads.
//
// Child body: BFS probes a visited bitmap (one bit per output slot,
// L2-resident), claims v in a second bitmap and writes its level; SSSP relaxes
// a second distance array with atomicMin and queues v once per iteration
// through an iteration stamp, or, for single traversals and the serving
// engine, records v as found and leaves the queueing to the harvest kernel.
// The probed and the updated copies swap every level.  BFS single traversals and the serving engine instead give each XCD a
// probed copy of its own on wide levels and record discoveries as bytes, which
// a third kernel, the harvest, turns into levels and the next frontier (Vis,
// vis_of, harvest_kernel).
//
// Queries: a launch may carry many traversals ("queries") over graphs packed
// in one CSR arena.  Query q owns the output slots [slot0, slot0 + n) (slot0 a
// multiple of 32, so bitmap words never straddle queries); frontier entries
// are slots.  A single traversal is a batch of one.  Queries may start at
// different level indices (continuous batching): a vertex found at level
// index L + 1 gets level L + 1 - lstart.  New frontier vertices are
// staged per wave in LDS and appended to one of 64 frontier queues with one
// atomic per flush, so no counter sees more than a few dozen atomics a level.
#include <hip/hip_runtime.h>
#include <stdint.h>

#include "dpo_internal.h"

namespace dpo {

__device__ __forceinline__ uint32_t lane_rank(unsigned long long mask) {
  return __builtin_amdgcn_mbcnt_hi((uint32_t)(mask >> 32),
                                   __builtin_amdgcn_mbcnt_lo((uint32_t)mask, 0u));
}

__device__ __forceinline__ uint32_t wave_incl_scan(uint32_t x, int lane) {
#pragma unroll
  for (int d = 1; d < 64; d <<= 1) {
    uint32_t y = __shfl_up(x, d, 64);
    if (lane >= d) x += y;
  }
  return x;
}

__device__ __forceinline__ void wave_lds_sync() {
  __builtin_amdgcn_fence(__ATOMIC_RELEASE, "wavefront");
  __builtin_amdgcn_wave_barrier();
  __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "wavefront");
}

__device__ __forceinline__ void set_error(State* st, uint32_t code) {
  atomicCAS(&st->error, 0u, code);
}

__device__ __forceinline__ uint32_t ceil_div(uint32_t a, uint32_t b) { return (a + b - 1) / b; }

// ------------------------------------------------------------ frontier queues
// Next frontier = NQF queues of fcap slots plus an overflow queue of n slots.
struct Reserve {
  uint32_t q, pos, inseg, obase;
};

// Reserve `cnt` slots in queue q (one lane).  Slots past fcap spill into the
// overflow queue.
__device__ __forceinline__ Reserve reserve_slots(const Args& a, LevelSet* ls, uint32_t q,
                                                 uint32_t cnt) {
  Reserve r{q, 0u, 0u, 0u};
  const uint32_t old = atomicAdd(&ls->fcnt[q], cnt);
  r.pos = old;
  r.inseg = old >= (uint32_t)a.fcap ? 0u : min(cnt, (uint32_t)a.fcap - old);
  if (r.inseg < cnt) {
    const uint32_t rest = cnt - r.inseg;
    r.obase = atomicAdd(&ls->fcnt[NQF], rest);
    if ((uint64_t)r.obase + rest > (uint64_t)a.slots) set_error(a.st, ERR_CAPACITY);
  }
  return r;
}

__device__ __forceinline__ void put_slot(const Args& a, int32_t* buf, const Reserve& r, uint32_t p,
                                         int32_t v) {
  if (p < r.inseg) {
    buf[(size_t)r.q * a.fcap + r.pos + p] = v;
  } else {
    const uint32_t o = r.obase + (p - r.inseg);
    if (o < (uint32_t)a.slots) buf[(size_t)NQF * a.fcap + o] = v;
  }
}

struct Stage {
  int32_t* buf;  // STAGE LDS slots owned by this wave
  uint32_t cnt;  // wave-uniform fill
};

// Flush one wave's staged vertices (wave-uniform call).
__device__ __forceinline__ void stage_flush(Stage& s, const Args& a, LevelSet* ls, int32_t* fout,
                                         int lane) {
  if (s.cnt == 0) return;
  Reserve r{0u, 0u, 0u, 0u};
  if (lane == 0) r = reserve_slots(a, ls, blockIdx.x % NQF, s.cnt);
  r.q = __shfl(r.q, 0, 64);
  r.pos = __shfl(r.pos, 0, 64);
  r.inseg = __shfl(r.inseg, 0, 64);
  r.obase = __shfl(r.obase, 0, 64);
  wave_lds_sync();
  for (uint32_t i = lane; i < s.cnt; i += 64) put_slot(a, fout, r, i, s.buf[i]);
  wave_lds_sync();
  s.cnt = 0;
}

// Wave-uniform call: every lane of the wave must reach it.
__device__ __forceinline__ void stage_push(Stage& s, bool found, int32_t v, const Args& a,
                                           LevelSet* ls, int32_t* fout, int lane) {
  const unsigned long long m = __ballot(found);
  if (m == 0) return;
  const uint32_t c = (uint32_t)__popcll(m);
  if (s.cnt + c > STAGE) stage_flush(s, a, ls, fout, lane);
  if (found) s.buf[s.cnt + lane_rank(m)] = v;
  s.cnt += c;
}

// End of kernel: one reservation for the whole workgroup.  Block-uniform call.
__device__ __forceinline__ void block_flush(Stage& s, const Args& a, LevelSet* ls, int32_t* fout, int tid,
                            uint32_t* s_cnt /* LDS [NW + 5] */) {
  const int lane = tid & 63, wave = tid >> 6;
  if (lane == 0) s_cnt[wave] = s.cnt;
  __syncthreads();
  if (tid == 0) {
    uint32_t tot = 0;
    for (int w = 0; w < NW; ++w) tot += s_cnt[w];
    Reserve r{0u, 0u, 0u, 0u};
    if (tot) r = reserve_slots(a, ls, blockIdx.x % NQF, tot);
    s_cnt[NW] = tot;
    s_cnt[NW + 1] = r.q;
    s_cnt[NW + 2] = r.pos;
    s_cnt[NW + 3] = r.inseg;
    s_cnt[NW + 4] = r.obase;
  }
  __syncthreads();
  if (s_cnt[NW] == 0) return;
  const Reserve r{s_cnt[NW + 1], s_cnt[NW + 2], s_cnt[NW + 3], s_cnt[NW + 4]};
  uint32_t off = 0;
  for (int w = 0; w < wave; ++w) off += s_cnt[w];
  for (uint32_t i = lane; i < s.cnt; i += 64) put_slot(a, fout, r, off + i, s.buf[i]);
  s.cnt = 0;
}

// ------------------------------------------------------------ child body
// Per-element context: query bounds and where its outputs live.
struct Elem {
  int32_t vbase;  // graph vertex 0 in the CSR arena
  int32_t n;      // graph vertices
  int32_t sbase;  // slot0 - vbase: slot of global vertex v is v + sbase
  int32_t lv;     // level value written for a discovery (BFS)
  uint32_t du;    // parent distance (SSSP)
};

// Visited state in two copies.  Device atomics on lines that other waves keep
// probing with plain loads run more than ten times slower on this chip than
// atomics on lines that only atomics touch.  So a level with a wide frontier
// probes one copy, read-only for the whole level, and sends its atomics to the
// other ("split"); the copies swap at the next level.  A level with a narrow
// frontier probes and updates one copy, which keeps the atomic next to the
// probed line and the level short.  At the start of a level the probed copy is
// complete.  A split level folds its frontier's own vertices (the previous
// level's discoveries / improvements) into the copy it updates, which then
// lacks exactly those; SSSP folds at every level, so the unprobed array always
// lacks just the frontier's improvements.  A one-copy BFS level skips the fold
// and marks the other bitmap stale (it only ever holds visited vertices); the
// next split level then folds every non-zero word of the probed bitmap.
// BFS: buffer i is the bitmap visit + i * vwords.  SSSP: buffer 0 is the
// output distance array, buffer 1 the workspace one; both hold the result at
// the end (the last level improves nothing, so its fold leaves them equal).
struct Vis {
  const uint32_t* probe;  // read with plain loads
  uint32_t* claim;        // the level's claims / atomicMin
  uint32_t* fold;         // receives the frontier's vertices / distances
  bool split;
  uint32_t* own;          // BFS with per-XCD copies: this XCD's copy (= probe)
};

// BFS with per-XCD copies (Args::hint): bitmap 0 is the visited set.  On a
// wide level (split) it does not change until the harvest kernel, and each XCD
// (workgroup % 8) probes its own bitmap, which holds bitmap 0 as of the
// level's start plus the vertices this XCD has found since, kept with plain
// loads and stores that stay in its L2; a narrow level probes and claims
// bitmap 0 with atomics and appends in place.
template <int P>
__device__ __forceinline__ Vis vis_of(const Args& a, uint32_t c, bool split) {
  if (P == PROB_BFS && a.hint) {
    if (!split) return Vis{a.visit, a.visit, nullptr, false, nullptr};
    uint32_t* own = a.visit + (size_t)(2u + (blockIdx.x & (NHINT - 1))) * (uint32_t)a.vwords;
    return Vis{own, a.visit, nullptr, false, own};
  }
  uint32_t* b0 = P == PROB_BFS ? a.visit : a.dist;
  uint32_t* b1 = P == PROB_BFS ? a.visit + a.vwords : a.dist2;
  uint32_t* pb = c ? b1 : b0;
  uint32_t* ob = c ? b0 : b1;
  return Vis{pb, split ? ob : pb, ob, split, nullptr};
}

__device__ __forceinline__ uint32_t coherent_load(const uint32_t* p) {
  return __hip_atomic_load(p, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
}

// Child body for U neighbours per lane (v < 0: none), all probes issued before
// any atomic so that the U round trips overlap.  BFS: probe, then claim the
// unvisited ones and write their level (per-XCD copies: record them as found).
// SSSP: relax (atomicMin) the edges that improve on the probed distance; an
// improved vertex joins the next frontier once per level (iteration stamp
// exchanged atomically, or a found byte that the harvest kernel reads).
// out[u] is the slot to append to the next frontier, or -1.
template <int P, int U>
__device__ __forceinline__ void visit_batch(const Args& a, const Vis& vis, const int32_t (&v)[U],
                                            const uint32_t (&w)[U], const Elem (&c)[U],
                                            uint32_t L, int32_t (&out)[U]) {
  int32_t sl[U];
#pragma unroll
  for (int u = 0; u < U; ++u) {
    sl[u] = -1;
    if (v[u] >= 0) {
      const int32_t loc = v[u] - c[u].vbase;
      if ((uint32_t)loc >= (uint32_t)c[u].n) set_error(a.st, ERR_ARG);
      else sl[u] = v[u] + c[u].sbase;
    }
    out[u] = -1;
  }
  if (P == PROB_BFS) {
    const uint32_t* pb = vis.probe;
    uint32_t* cb = vis.claim;
    uint32_t word[U];
#pragma unroll
    for (int u = 0; u < U; ++u) word[u] = sl[u] >= 0 ? pb[(uint32_t)sl[u] >> 5] : ~0u;
    // Per-XCD copies (wide level): a candidate records itself in its XCD's
    // copy and in the found bytes, both plain stores, and nothing else: no
    // atomic, no level, no append.  The harvest kernel after the level takes
    // every found vertex that bitmap 0 (visited before the level) lacks, so
    // the level's discoveries cost no device atomics, which the chip runs at
    // a few tens of G/s for random addresses.  A set bit in the copy means a
    // lane of this XCD found the vertex at this level, or it was visited
    // before; a stale or lost bit only lets a second found store through.
    if (vis.own) {
#pragma unroll
      for (int u = 0; u < U; ++u) {
        const uint32_t bit = 1u << (sl[u] & 31);
        if (sl[u] >= 0 && !(word[u] & bit)) {
          vis.own[(uint32_t)sl[u] >> 5] = word[u] | bit;
          a.found[sl[u]] = 1;
        }
      }
      return;
    }
    // Two shared copies (split level): vertices found earlier in this level
    // are still clear in the probed bitmap; a batch with many candidates reads
    // the claim words with coherent loads first, with few that round trip
    // would only add latency.
    bool filter = false;
    if (vis.split) {
      uint32_t ncand = 0;
#pragma unroll
      for (int u = 0; u < U; ++u)
        ncand += (uint32_t)__popcll(__ballot(sl[u] >= 0 && !(word[u] & (1u << (sl[u] & 31)))));
      filter = ncand > PRECHECK_MIN;
    }
    if (filter) {
#pragma unroll
      for (int u = 0; u < U; ++u)
        if (sl[u] >= 0 && !(word[u] & (1u << (sl[u] & 31))))
          word[u] = coherent_load(&cb[(uint32_t)sl[u] >> 5]);
    }
#pragma unroll
    for (int u = 0; u < U; ++u) {
      const uint32_t bit = 1u << (sl[u] & 31);
      if (sl[u] >= 0 && !(word[u] & bit)) word[u] = atomicOr(&cb[(uint32_t)sl[u] >> 5], bit);
      else word[u] = ~0u;
    }
#pragma unroll
    for (int u = 0; u < U; ++u) {
      if (!(word[u] & (1u << (sl[u] & 31)))) {
        a.level[sl[u]] = c[u].lv;
        out[u] = sl[u];
      }
    }
  } else {
    const uint32_t* dp = vis.probe;
    uint32_t* dl = vis.claim;
    uint32_t nd[U], cur[U];
#pragma unroll
    for (int u = 0; u < U; ++u) {
      // saturating: a walk of 2^32 - 1 or more never improves a distance, so
      // no wrapped sum can undercut the true one
      const uint32_t sum = c[u].du + w[u];
      nd[u] = sum < c[u].du ? 0xFFFFFFFFu : sum;
      cur[u] = sl[u] >= 0 ? dp[sl[u]] : 0u;
    }
    uint32_t ncand = 0;
    if (vis.split) {
#pragma unroll
      for (int u = 0; u < U; ++u) ncand += (uint32_t)__popcll(__ballot(sl[u] >= 0 && nd[u] < cur[u]));
    }
    const bool pre = ncand > PRECHECK_MIN;
    if (pre) {
#pragma unroll
      for (int u = 0; u < U; ++u)
        if (sl[u] >= 0 && nd[u] < cur[u]) cur[u] = coherent_load(&dl[sl[u]]);
    }
#pragma unroll
    for (int u = 0; u < U; ++u) {
      if (sl[u] >= 0 && nd[u] < cur[u]) cur[u] = atomicMin(&dl[sl[u]], nd[u]);
      else cur[u] = 0u;
    }
    // Found bytes (Args::hint): an improved vertex is recorded with a plain
    // byte store and queued once by the harvest kernel after the level, so an
    // improving lane waits for no atomic after its atomicMin.
    if (a.hint) {
#pragma unroll
      for (int u = 0; u < U; ++u)
        if (nd[u] < cur[u]) a.found[sl[u]] = 1;
      return;
    }
    const uint32_t it = L + 1;
    uint32_t stamp[U];
#pragma unroll
    for (int u = 0; u < U; ++u) stamp[u] = (pre && nd[u] < cur[u]) ? coherent_load(&a.visit[sl[u]]) : 0u;
#pragma unroll
    for (int u = 0; u < U; ++u) {
      if (nd[u] < cur[u] && stamp[u] != it) stamp[u] = atomicExch(&a.visit[sl[u]], it);
      else stamp[u] = it;
    }
#pragma unroll
    for (int u = 0; u < U; ++u)
      if (stamp[u] != it) out[u] = sl[u];
  }
}

struct Counters {
  uint32_t front, serial, rec, child, eser, echild, desc;
};

// Per-workgroup counters: one row per workgroup, summed on the host.
__device__ __forceinline__ void add_stats(const Args& a, unsigned long long* s_stats,
                                          const Counters& c, int tid) {
  if (!a.count_stats) return;
  if (c.front) atomicAdd(&s_stats[S_FRONT], (unsigned long long)c.front);
  if (c.serial) atomicAdd(&s_stats[S_SERIAL], (unsigned long long)c.serial);
  if (c.rec) atomicAdd(&s_stats[S_REC], (unsigned long long)c.rec);
  if (c.child) atomicAdd(&s_stats[S_CHILD], (unsigned long long)c.child);
  if (c.eser) atomicAdd(&s_stats[S_ESER], (unsigned long long)c.eser);
  if (c.echild) atomicAdd(&s_stats[S_ECHILD], (unsigned long long)c.echild);
  if (c.desc) atomicAdd(&s_stats[S_DESC], (unsigned long long)c.desc);
  __syncthreads();
  if (tid < NSTAT && blockIdx.x < MAX_GRID) a.stats[blockIdx.x * NSTAT + tid] += s_stats[tid];
}

// Phase clock of one wave, for the timed instantiations (ON = false: empty).
// mark(p) charges the shader-clock cycles since the previous mark to phase p,
// after the wave's outstanding memory operations have completed, so each
// phase pays for the loads and stores it issued.  Marks sit only at points
// that every lane of the wave reaches together, so the clock values stay
// wave-uniform.
template <bool ON>
struct PhaseClock {
  uint64_t last = 0;
  uint64_t acc[TP_N] = {0, 0, 0, 0, 0};
  __device__ __forceinline__ void start() {
    if (ON) last = __builtin_amdgcn_s_memtime();
  }
  __device__ __forceinline__ void mark(int p) {
    if (!ON) return;
    __builtin_amdgcn_sched_barrier(0);
    __builtin_amdgcn_s_waitcnt(0);
    const uint64_t now = __builtin_amdgcn_s_memtime();
    acc[p] += now - last;
    last = now;
    __builtin_amdgcn_sched_barrier(0);
  }
};

__device__ __forceinline__ uint64_t realtime() { return __builtin_amdgcn_s_memrealtime(); }

// Timed instantiations: the workgroup's row (entry / exit realtime, cycles per
// phase summed over its waves, the busiest wave's total).  Block-uniform call.
template <bool ON>
__device__ __forceinline__ void tm_write(const Args& a, const PhaseClock<ON>& pc, int kind,
                                         uint32_t L, uint64_t t_entry, int tid) {
  if (!ON) return;
  __shared__ unsigned long long s_tm[NW][TP_N];
  const int lane = tid & 63, wave = tid >> 6;
  if (lane == 0)
    for (int p = 0; p < TP_N; ++p) s_tm[wave][p] = pc.acc[p];
  __syncthreads();
  if (tid == 0 && L < (uint32_t)TM_LEVELS && blockIdx.x < (uint32_t)MAX_GRID) {
    unsigned long long sum[TP_N] = {0, 0, 0, 0, 0}, mx = 0;
    for (int w = 0; w < NW; ++w) {
      unsigned long long t = 0;
      for (int p = 0; p < TP_N; ++p) {
        sum[p] += s_tm[w][p];
        t += s_tm[w][p];
      }
      mx = t > mx ? t : mx;
    }
    unsigned long long* row =
        a.tm + ((size_t)(L * TM_KINDS + (uint32_t)kind) * MAX_GRID + blockIdx.x) * TM_ROW;
    row[0] = t_entry;
    row[1] = realtime();
    for (int p = 0; p < TP_N; ++p) row[2 + p] = sum[p];
    row[7] = mx;
  }
}

// Append one aggregated grid to descriptor queue q (one lane).
__device__ __forceinline__ void publish(const Args& a, LevelSet* ls, uint32_t q, uint32_t rec_base,
                                        uint32_t nrec, uint32_t total) {
  const unsigned long long old =
      atomicAdd(&ls->qctr[q], ((unsigned long long)1 << 32) | (unsigned long long)total);
  const uint32_t d = (uint32_t)(old >> 32);
  if (d >= (uint32_t)a.desc_cap) {
    set_error(a.st, ERR_CAPACITY);
    return;
  }
  a.desc[(size_t)q * a.desc_cap + d] = make_int4((int32_t)rec_base, (int32_t)nrec, (int32_t)old, 0);
}

// Launch record `r` of the level: the parent's row, child count, scanned
// offset of its coarsened grid and distance; its query; for SSSP its slot.
template <int P>
__device__ __forceinline__ void put_record(const Args& a, uint32_t r, int32_t start, int32_t deg,
                                           uint32_t off, uint32_t du, int32_t q, int32_t slot) {
  a.rec[r] = make_int4(start, deg, (int32_t)off, (int32_t)du);
  a.rec_q[r] = q;
  if (P == PROB_SSSP) a.rec_slot[r] = slot;
}

// Frontier entry i of level L: queue q with s_fpre[q] <= i < s_fpre[q + 1].
__device__ __forceinline__ int32_t frontier_at(const Args& a, const int32_t* fin,
                                               const uint32_t* s_fpre, uint32_t i) {
  uint32_t lo = 0, hi = NQF + 1;
  while (hi - lo > 1) {
    const uint32_t mid = (lo + hi) >> 1;
    if (s_fpre[mid] <= i) lo = mid; else hi = mid;
  }
  return fin[(size_t)lo * a.fcap + (i - s_fpre[lo])];
}


// One parent thread: its query, vertex, row and parameters.
struct Parent {
  int32_t start, deg, T, CF, slot;
  uint32_t q;
  Elem e;
};

template <int P>
__device__ __forceinline__ Parent load_parent(const Args& a, const int32_t* fin,
                                              const uint32_t* s_fpre, uint32_t i, uint32_t L) {
  Parent p;
  p.slot = frontier_at(a, fin, s_fpre, i);
  p.q = (uint32_t)a.qmap[(uint32_t)p.slot >> 5];
  const Query Q = a.q[p.q];
  const int32_t vg = Q.vbase + (p.slot - Q.slot0);
  p.start = a.rp[vg];
  p.deg = a.rp[vg + 1] - p.start;
  p.T = Q.T;
  p.CF = Q.CF;
  p.e.vbase = Q.vbase;
  p.e.n = Q.n;
  p.e.sbase = Q.slot0 - Q.vbase;
  p.e.lv = (int32_t)(L + 1) - Q.lstart;
  p.e.du = 0;
  return p;
}

// ------------------------------------------------------------ parent kernel
// Pass 1 reads each frontier entry once, decides it (threshold), aggregates
// the launching ones and writes their records (block barriers) and lists the
// thresholded ones; pass 2 runs the listed parents' serial children with no
// barrier, so waves do not wait on each other.
//
// PH = PH_BOTH runs both passes.  PH_LIST runs pass 1 only and leaves the
// workgroup's list length in a.sercnt; PH_SERIAL, launched after the level's
// child kernel on the same grid, runs pass 2 over that list (SSSP: its parents
// are then checked against every improvement the launched children made).
template <int P, int G, int PH, bool TM>
__global__ __launch_bounds__(PB) void parent_kernel(Args a, uint32_t step) {
  __shared__ int32_t s_stage[NW][STAGE];
  __shared__ uint32_t s_fpre[NQF + 2];
  __shared__ uint32_t s_scan[2 * NW];
  __shared__ uint32_t s_bc[NW + 8];
  __shared__ unsigned long long s_stats[NSTAT];
  __shared__ uint32_t s_live[MAX_QUERIES / 32];  // queries seen at this level
  __shared__ uint32_t s_ser[2];                  // serial list: length, next entry
  __shared__ uint32_t s_soff[NW][64];            // per wave: scanned child sizes of a group
  __shared__ uint32_t s_lpre[PH == PH_SERIAL ? MAX_GRID + 1 : 1];  // prefix of list lengths

  const int tid = threadIdx.x, lane = tid & 63, wave = tid >> 6;
  State* st = a.st;
  uint64_t t_entry = 0;
  if (TM) t_entry = realtime();
  PhaseClock<TM> pc;
  pc.start();
  if (st->done || st->error) return;
  const uint32_t L = st->base + step;
  LevelSet* prv = &st->set[(L + 2) % 3];  // fills of frontier L
  LevelSet* cur = &st->set[L % 3];        // this level: next-frontier fills, queues, groups
  const int32_t* fin = (L & 1) ? a.front1 : a.front0;
  int32_t* fout = (L & 1) ? a.front0 : a.front1;

  // frontier L = queues 0..NQF-1 then overflow; prefix of their fills
  if (wave == 0) {
    const uint32_t c = min(prv->fcnt[lane], (uint32_t)a.fcap);
    const uint32_t incl = wave_incl_scan(c, lane);
    s_fpre[lane + 1] = incl;
    if (lane == 0) s_fpre[0] = 0;
    if (lane == 63) s_fpre[NQF + 1] = incl + prv->fcnt[NQF];
  }
  if (tid < NSTAT) s_stats[tid] = 0;
  for (int i = tid; i < (a.nq + 31) / 32; i += PB) s_live[i] = 0;
  __syncthreads();
  const uint32_t F = s_fpre[NQF + 1];
  if (F == 0) {
    if (PH != PH_SERIAL && blockIdx.x == 0 && tid == 0) st->done = 1;
    return;
  }
  // Each vertex enters a frontier at most once per level (the claim atomic,
  // the SSSP stamp, the harvest of found bytes), and the launch records,
  // serial lists and group counters of a level are sized for that; a larger
  // frontier is an error, never an index past them.
  if (F > (uint32_t)a.slots) {
    if (tid == 0) set_error(st, ERR_CAPACITY);
    return;
  }
  // visited copies of this level (every workgroup derives the same choice)
  const uint32_t vc = st->vsel[L & 1];
  const bool split = F >= (uint32_t)a.split_min;
  const bool stale = st->vstale[L & 1] != 0;
  const Vis vis = vis_of<P>(a, vc, split);
  if (PH != PH_SERIAL && blockIdx.x == 0) {
    LevelSet* z = &st->set[(L + 1) % 3];  // idle until level L + 1
    if (tid <= NQF) z->fcnt[tid] = 0;
    if (tid < NQD) z->qctr[tid] = 0;
    if (tid < NQD) z->cclaim[tid][0] = 0;
    if (tid == 0) {
      st->levels_run = L + 1;
      cur->vmode = vc | (split ? 2u : 0u);  // for this level's child kernel
      st->vsel[(L + 1) & 1] = vc ^ (split ? 1u : 0u);
      st->vstale[(L + 1) & 1] = (P == PROB_BFS && !split) ? 1u : 0u;
    }
  }
  if (G == AGG_MULTI && PH != PH_SERIAL) {
    const uint32_t nz = (L + 1) % 3;
    for (int i = blockIdx.x * PB + tid; i < a.ngroups_cap; i += gridDim.x * PB) {
      a.grp_packed[nz * a.ngroups_cap + i] = 0;
      a.grp_done[nz * a.ngroups_cap + i] = 0;
    }
  }

  Stage s{s_stage[wave], 0u};
  Counters cn{0, 0, 0, 0, 0, 0, 0};
  const uint32_t nvb = ceil_div(F, PB);
  // thresholded parents listed by this workgroup
  if (tid == 0) s_ser[0] = PH == PH_SERIAL ? a.sercnt[blockIdx.x] : 0u;
  __syncthreads();

  // Fold into the copy not probed at this level: one atomic per frontier
  // entry, or, for BFS after a one-copy level or with more frontier entries
  // than bitmap words, one per non-zero word of the probed bitmap.  BFS with
  // per-XCD copies: a wide level starts by copying bitmap 0 into every XCD's
  // copy (each XCD's workgroups write their own copy), before pass 1 so that
  // pass 2 mostly probes complete copies; narrow levels keep no copy up to
  // date, which is why the next wide level copies it whole.
  const bool own = P == PROB_BFS && a.hint;
  const bool word_fold =
      !own && PH != PH_SERIAL && P == PROB_BFS && split && (stale || F > (uint32_t)a.vwords);
  const bool entry_fold = P == PROB_SSSP || (!own && split && !word_fold);
  if (own && split && PH != PH_SERIAL) {
    const bool local = gridDim.x % NHINT == 0;
    const uint32_t x0 = local ? blockIdx.x % NHINT : 0u, nx = local ? 1u : (uint32_t)NHINT;
    const uint32_t k = local ? blockIdx.x / NHINT : blockIdx.x;
    const uint32_t nk = local ? gridDim.x / NHINT : gridDim.x;
    for (uint32_t w = k * PB + tid; w < (uint32_t)a.vwords; w += nk * PB) {
      const uint32_t cw = a.visit[w];
      if (cw)
        for (uint32_t x = x0; x < x0 + nx; ++x) a.visit[(size_t)(2 + x) * a.vwords + w] = cw;
    }
  }
  // a workgroup with at most one virtual block keeps its thresholded parents
  // in registers (narrow levels are latency-bound)
  const bool in_regs = PH == PH_BOTH && nvb <= gridDim.x;
  int32_t e = 0, end = 0;     // this lane's serial child: edges [e, end)
  Elem ctx{0, 0, 0, 0, 0u};

  // ---- pass 1: every frontier entry once.  Threshold, coarsened grid size,
  // aggregation and launch records; thresholded parents go to this
  // workgroup's serial list for pass 2.
  for (uint32_t vb = blockIdx.x; vb < (PH == PH_SERIAL ? 0u : nvb); vb += gridDim.x) {
    const uint32_t i = vb * PB + tid;
    int32_t start = 0, deg = 0, q = 0, slot = 0;
    uint32_t du = 0, cg = 0;
    bool launch = false, ser = false;
    if (i < F) {
      const Parent p = load_parent<P>(a, fin, s_fpre, i, L);
      start = p.start;
      deg = p.deg;
      q = (int32_t)p.q;
      slot = p.slot;
      ++cn.front;
      atomicOr(&s_live[p.q >> 5], 1u << (p.q & 31));
      if (P == PROB_SSSP) {
        du = vis.probe[slot];
        // PH_LIST runs before any relaxation of its level, so this is the
        // entry's only writer and du is never above the value it replaces
        // (the copy lacks just the frontier's improvements): a plain store
        if (PH == PH_LIST) vis.fold[slot] = du;
        else atomicMin(&vis.fold[slot], du);
      } else if (entry_fold) {
        atomicOr(&vis.fold[(uint32_t)slot >> 5], 1u << (slot & 31));
      }
      launch = G != AGG_FLAT && deg > 0 && deg >= p.T;
      ser = deg > 0 && !launch;
      if (launch) {
        // coarsened grid size (Sec. IV-B)
        cg = ceil_div(ceil_div((uint32_t)deg, (uint32_t)a.CB), (uint32_t)p.CF);
      }
      if (ser) {
        ++cn.serial;
        if (in_regs) {
          e = start;
          end = start + deg;
          ctx = p.e;
          ctx.du = du;
        }
      }
    }
    if (!in_regs) {
      // entry k of the list sits in this workgroup's own virtual blocks
      const unsigned long long m = __ballot(ser);
      uint32_t base = 0;
      if (lane == 0 && m) base = atomicAdd(&s_ser[0], (uint32_t)__popcll(m));
      base = __shfl(base, 0, 64);
      if (ser) {
        const uint32_t k = base + lane_rank(m);
        a.ser[(size_t)(blockIdx.x + (k / PB) * gridDim.x) * PB + k % PB] =
            make_int4(start, deg, slot, (int32_t)du);
      }
    }
    pc.mark(TP_PARENT);
    if (G != AGG_FLAT) {
      if (launch) ++cn.rec;

      if (G == AGG_NONE) {
        // every launching parent publishes its own grid; its record sits at
        // its frontier index
        if (TM) {
          if (launch) put_record<P>(a, i, start, deg, 0u, du, q, slot);
          pc.mark(TP_AGG);
        }
        if (launch) {
          if (!TM) put_record<P>(a, i, start, deg, 0u, du, q, slot);
          publish(a, cur, vb % NQD, i, 1u, cg);
          ++cn.desc;
        }
        pc.mark(TP_LAUNCH);
      } else if (G == AGG_WAVE) {
        const unsigned long long m = __ballot(launch);
        const uint32_t nrec = (uint32_t)__popcll(m);
        const uint32_t seg = vb * PB + wave * 64;
        if (m && nrec < (uint32_t)a.agg_threshold) {
          // too few participants (Sec. V-B): each parent launches its own grid
          if (launch) put_record<P>(a, seg + lane_rank(m), start, deg, 0u, du, q, slot);
          pc.mark(TP_AGG);
          if (launch) {
            publish(a, cur, vb % NQD, seg + lane_rank(m), 1u, cg);
            ++cn.desc;
          }
          pc.mark(TP_LAUNCH);
        } else if (m) {  // wave-uniform
          const uint32_t incl = wave_incl_scan(cg, lane);
          const uint32_t total = __shfl(incl, 63, 64);
          if (launch) {
            put_record<P>(a, seg + lane_rank(m), start, deg, incl - cg, du, q, slot);
          }
          pc.mark(TP_AGG);
          if (lane == 0) {
            publish(a, cur, vb % NQD, seg, nrec, total);
            ++cn.desc;
          }
          pc.mark(TP_LAUNCH);
        }
      } else {
        // block-level scan of (launch, cg): wave scans, then across waves in LDS
        const unsigned long long m = __ballot(launch);
        const uint32_t incl = wave_incl_scan(cg, lane);
        if (lane == 63) {
          s_scan[wave] = (uint32_t)__popcll(m);
          s_scan[NW + wave] = incl;
        }
        __syncthreads();
        uint32_t roff = 0, coff = 0, nrec_b = 0, total_b = 0;
#pragma unroll
        for (int w = 0; w < NW; ++w) {
          if (w < wave) { roff += s_scan[w]; coff += s_scan[NW + w]; }
          nrec_b += s_scan[w];
          total_b += s_scan[NW + w];
        }
        if (G == AGG_BLOCK) {
          const uint32_t seg = vb * PB;
          if (nrec_b < (uint32_t)a.agg_threshold) {
            // too few participants (Sec. V-B): each parent launches its own grid
            const uint32_t r = seg + roff + lane_rank(m);
            if (launch) put_record<P>(a, r, start, deg, 0u, du, q, slot);
            pc.mark(TP_AGG);
            if (launch) {
              publish(a, cur, vb % NQD, r, 1u, cg);
              ++cn.desc;
            }
            pc.mark(TP_LAUNCH);
          } else {
            if (launch) {
              put_record<P>(a, seg + roff + lane_rank(m), start, deg, coff + incl - cg, du, q, slot);
            }
            pc.mark(TP_AGG);
            if (tid == 0 && nrec_b) {
              publish(a, cur, vb % NQD, seg, nrec_b, total_b);
              ++cn.desc;
            }
            pc.mark(TP_LAUNCH);
          }
          __syncthreads();  // s_scan reuse
        } else {  // AGG_MULTI: group of k consecutive virtual blocks (Sec. V-A)
          const uint32_t g = vb / (uint32_t)a.k;
          const uint32_t seg = g * (uint32_t)a.k * PB;
          unsigned long long* gp = &a.grp_packed[(L % 3) * a.ngroups_cap + g];
          uint32_t* gd = &a.grp_done[(L % 3) * a.ngroups_cap + g];
          if (tid == 0) {
            unsigned long long old = 0;
            if (nrec_b)
              old = atomicAdd(gp, ((unsigned long long)nrec_b << 32) | (unsigned long long)total_b);
            s_bc[0] = (uint32_t)(old >> 32);
            s_bc[1] = (uint32_t)old;
          }
          __syncthreads();
          const uint32_t slot0 = s_bc[0], off0 = s_bc[1];
          if (launch) {
            put_record<P>(a, seg + slot0 + roff + lane_rank(m), start, deg, off0 + coff + incl - cg,
                          du, q, slot);
          }
          // the group's last block to finish "launches" the aggregated grid;
          // its packed-counter add returned before this increment was issued
          bool last_block = false;
          if (tid == 0) {
            const uint32_t in_group = min((uint32_t)a.k, nvb - g * (uint32_t)a.k);
            last_block = atomicAdd(gd, 1u) == in_group - 1;
          }
          pc.mark(TP_AGG);
          if (last_block) {
            const unsigned long long tot = atomicAdd(gp, 0ull);
            const uint32_t nrec_g = (uint32_t)(tot >> 32);
            if (nrec_g) {
              publish(a, cur, g % NQD, seg, nrec_g, (uint32_t)tot);
              ++cn.desc;
            }
          }
          pc.mark(TP_LAUNCH);
          __syncthreads();  // s_scan / s_bc reuse
        }
      }
      pc.mark(TP_AGG);
    }
  }

  // ---- pass 2: the thresholded children (Sec. III-B: no launch; the parent's
  // own threads run the child work).
  __syncthreads();
  if (PH == PH_LIST && tid == 0) a.sercnt[blockIdx.x] = s_ser[0];
  if (PH != PH_LIST) {
    const uint32_t nser = s_ser[0];
    // This workgroup's list entries [r0, r1).  PH_SERIAL: the lists are
    // complete, and the workgroups split their concatenation evenly (a block
    // scan of the list lengths), so each runs the same number of thresholded
    // parents however many its own list holds.
    uint32_t r0 = 0, r1 = nser, nl = 0;
    if (PH == PH_SERIAL && G != AGG_FLAT && a.serial_wave) {
      nl = min(gridDim.x, nvb);
      constexpr int PER = MAX_GRID / PB;
      uint32_t vals[PER], sum = 0;
#pragma unroll
      for (int j = 0; j < PER; ++j) {
        const uint32_t l = (uint32_t)tid * PER + j;
        vals[j] = l < nl ? a.sercnt[l] : 0u;
        sum += vals[j];
      }
      const uint32_t incl = wave_incl_scan(sum, lane);
      if (lane == 63) s_scan[wave] = incl;
      __syncthreads();
      uint32_t run = incl - sum, tot = 0;
#pragma unroll
      for (int w2 = 0; w2 < NW; ++w2) {
        if (w2 < wave) run += s_scan[w2];
        tot += s_scan[w2];
      }
#pragma unroll
      for (int j = 0; j < PER; ++j) {
        const uint32_t l = (uint32_t)tid * PER + j;
        if (l < nl) s_lpre[l] = run;
        run += vals[j];
      }
      if (tid == 0) s_lpre[nl] = tot;
      r0 = (uint32_t)((uint64_t)blockIdx.x * tot / gridDim.x);
      r1 = (uint32_t)((uint64_t)(blockIdx.x + 1) * tot / gridDim.x);
    }
    if (tid == 0) s_ser[1] = r0;  // next list entry
    __syncthreads();
    constexpr int U = 8;
    if (G != AGG_FLAT && a.serial_wave) {
      // The wave runs the children of up to 64 parents together: their edges
      // are concatenated (a wave scan of the degrees) and taken 64 at a time,
      // each lane finding its parent by a search of the scanned offsets, so
      // lanes read consecutive edges and none idles while a long child runs.
      uint32_t* off = s_soff[wave];
      bool first = true;
      while (true) {
        int32_t cs = 0, cd = 0;
        Elem cc{0, 0, 0, 0, 0u};
        if (in_regs) {  // the lanes' own parents from pass 1: one group
          if (!first) break;
          cs = e;
          cd = end - e;
          cc = ctx;
          cn.eser += (uint32_t)cd;
        } else {
          uint32_t base = 0, n = 64;
          int4 r = make_int4(0, 0, 0, 0);
          if (PH == PH_SERIAL) {
            // Claim the next entries of this workgroup's range whose children
            // total at most GROUP_EDGES edges (at least one entry): groups of
            // similar length, so no wave's last group holds up its workgroup.
            while (true) {
              if (lane == 0)
                base = __hip_atomic_load(&s_ser[1], __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_WORKGROUP);
              base = __shfl(base, 0, 64);
              if (base >= r1) break;
              uint32_t k = base + (uint32_t)lane;
              uint32_t dg = 0;
              if (k < r1) {
                // list holding entry k of the concatenation: the last list
                // whose prefix is <= k (empty lists share their successor's)
                uint32_t lo = 0, hi = nl;
                while (hi - lo > 1) {
                  const uint32_t mid = (lo + hi) >> 1;
                  if (s_lpre[mid] <= k) lo = mid; else hi = mid;
                }
                k -= s_lpre[lo];
                r = a.ser[(size_t)(lo + (k / PB) * gridDim.x) * PB + k % PB];
                dg = (uint32_t)r.y;
              }
              const uint32_t inc = wave_incl_scan(dg, lane);
              n = (uint32_t)__popcll(__ballot(base + (uint32_t)lane < r1 && inc <= GROUP_EDGES));
              n = max(n, 1u);
              uint32_t won = 0;
              if (lane == 0) won = atomicCAS(&s_ser[1], base, base + n) == base ? 1u : 0u;
              if (__shfl(won, 0, 64)) break;
            }
          } else {
            if (lane == 0) base = atomicAdd(&s_ser[1], 64u);
            base = __shfl(base, 0, 64);
            const uint32_t k = base + (uint32_t)lane;
            if (k < r1) r = a.ser[(size_t)(blockIdx.x + (k / PB) * gridDim.x) * PB + k % PB];
            n = base < r1 ? min(64u, r1 - base) : 0u;
          }
          if (base >= r1) break;
          if ((uint32_t)lane < n) {
            const Query Q = a.q[a.qmap[(uint32_t)r.z >> 5]];
            cs = r.x;
            cd = r.y;
            cc = Elem{Q.vbase, Q.n, Q.slot0 - Q.vbase, (int32_t)(L + 1) - Q.lstart, (uint32_t)r.w};
            // SSSP: a parent lowered again during this level expands at the next
            if (P == PROB_SSSP && coherent_load(&vis.claim[r.z]) < (uint32_t)r.w) cd = 0;
            cn.eser += (uint32_t)cd;
          }
        }
        first = false;
        const uint32_t incl = wave_incl_scan((uint32_t)cd, lane);
        const uint32_t excl = incl - (uint32_t)cd;
        const uint32_t total = __shfl(incl, 63, 64);
        wave_lds_sync();
        off[lane] = excl;
        wave_lds_sync();
        for (uint32_t x0 = 0; x0 < total; x0 += 64u * U) {
          int32_t v[U], out[U];
          uint32_t w[U];
          Elem c[U];
#pragma unroll
          for (int u = 0; u < U; ++u) {
            const uint32_t x = x0 + (uint32_t)u * 64u + (uint32_t)lane;
            const uint32_t xs = x < total ? x : total - 1;
            // parent of edge xs: the last lane whose offset is <= xs
            uint32_t pl = 0;
#pragma unroll
            for (uint32_t st = 32; st; st >>= 1)
              if (off[pl + st] <= xs) pl += st;
            const int32_t sp = __shfl(cs, (int)pl, 64);
            const uint32_t ep = (uint32_t)__shfl((int32_t)excl, (int)pl, 64);
            c[u] = Elem{__shfl(cc.vbase, (int)pl, 64), __shfl(cc.n, (int)pl, 64),
                        __shfl(cc.sbase, (int)pl, 64), __shfl(cc.lv, (int)pl, 64),
                        (uint32_t)__shfl((int32_t)cc.du, (int)pl, 64)};
            const int32_t ei = sp + (int32_t)(xs - ep);
            v[u] = x < total ? a.col[ei] : -1;
            w[u] = (P == PROB_SSSP && x < total) ? a.w[ei] : 0u;
          }
          visit_batch<P, U>(a, vis, v, w, c, L, out);
#pragma unroll
          for (int u = 0; u < U; ++u) stage_push(s, out[u] >= 0, out[u], a, cur, fout, lane);
        }
        wave_lds_sync();  // off[] is rewritten by the next group
      }
    } else {
      // Each child runs sequentially in one lane (the paper's form; always
      // used by the flat kernel).  A lane whose child is done takes the next
      // parent of the list, so lanes do not idle until the wave's largest
      // child finishes.
      uint32_t pnow = 0xFFFFFFFFu;  // SSSP: the lane's parent distance when taken
      while (true) {
        // SSSP: a parent lowered again during this level expands at the next
        // (checked one batch after the load was issued, so nothing waits)
        if (P == PROB_SSSP && pnow < ctx.du) end = e;
        const bool idle = e >= end;
        const unsigned long long m = __ballot(idle);
        uint32_t base = 0;
        if (m) {
          if (lane == __builtin_ctzll(m)) base = atomicAdd(&s_ser[1], (uint32_t)__popcll(m));
          base = __shfl(base, __builtin_ctzll(m), 64);
        }
        if (idle) {
          const uint32_t k = base + lane_rank(m);
          if (k < nser) {
            const int4 r = a.ser[(size_t)(blockIdx.x + (k / PB) * gridDim.x) * PB + k % PB];
            const Query Q = a.q[a.qmap[(uint32_t)r.z >> 5]];
            e = r.x;
            end = r.x + r.y;
            if (P == PROB_SSSP) pnow = coherent_load(&vis.claim[r.z]);
            ctx.vbase = Q.vbase;
            ctx.n = Q.n;
            ctx.sbase = Q.slot0 - Q.vbase;
            ctx.lv = (int32_t)(L + 1) - Q.lstart;
            ctx.du = (uint32_t)r.w;
          }
        }
        if (!__any(e < end)) break;
        int32_t v[U], out[U];
        uint32_t w[U];
        Elem c[U];
#pragma unroll
        for (int r = 0; r < U; ++r) {
          v[r] = (e + r < end) ? a.col[e + r] : -1;
          w[r] = (P == PROB_SSSP && e + r < end) ? a.w[e + r] : 0u;
          c[r] = ctx;
        }
        visit_batch<P, U>(a, vis, v, w, c, L, out);
#pragma unroll
        for (int r = 0; r < U; ++r) stage_push(s, out[r] >= 0, out[r], a, cur, fout, lane);
        const int32_t e2 = min(e + U, end);
        cn.eser += (uint32_t)(e2 - e);
        e = e2;
      }
    }
  }
  if (word_fold) {
    for (uint32_t w = blockIdx.x * PB + tid; w < (uint32_t)a.vwords; w += gridDim.x * PB) {
      const uint32_t x = vis.probe[w];
      if (x) atomicOr(&vis.fold[w], x);
    }
  }
  block_flush(s, a, cur, fout, tid, s_bc);
  // queries with frontier entries at this level are still running
  __syncthreads();
  if (PH != PH_SERIAL)
    for (int i = tid; i < a.nq; i += PB)
      if (s_live[i >> 5] & (1u << (i & 31))) a.q[i].last = (int32_t)L;
  add_stats(a, s_stats, cn, tid);
  pc.mark(TP_PARENT);
  tm_write<TM>(a, pc, PH == PH_SERIAL ? TK_SERIAL : TK_PARENT, L, t_entry, tid);
}

// ------------------------------------------------------------ child kernel
// Largest p in [0, n) with key(p) <= t, where key(0) <= t and keys increase:
// 64-ary wave search (each round narrows the range 64-fold).
template <typename KeyFn>
__device__ __forceinline__ uint32_t wave_upper_search(uint32_t n, uint32_t t, int lane, KeyFn key) {
  uint32_t lo = 0, hi = n;
  while (hi - lo > 1) {
    const uint32_t step = (hi - lo + 63) / 64;
    const uint32_t p = lo + (uint32_t)lane * step;
    const bool le = p < hi && key(p) <= t;
    const uint32_t k = (uint32_t)__popcll(__ballot(le));
    lo += (k - 1) * step;
    hi = min(lo + step, hi);
  }
  return lo;
}

// Lane k of a wave holds record r0 + k of the current descriptor, the fields
// of its query and its share of the wave's child blocks [t0, t1): blocks
// [lo, hi) of its coarsened grid, i.e. the edges [elo, ehi) of its row, cut
// into 64-lane slices.  Consecutive small records cost one wave-wide load.
struct Window {
  int32_t rs, elo, ehi;             // row start, edge range of the share
  uint32_t excl, nslices;           // exclusive scan of the slice counts, total
  int32_t vbase, n, sbase, lv;      // query fields (Elem)
  uint32_t du;
  int32_t ps;                       // SSSP: the parent's slot
  bool last;                        // the wave's range ends in this window
  bool bad;
};

// Window of the records base .. base + wn - 1.  SSSP: a parent whose distance
// was lowered again during this level is already queued for the next level,
// where it expands with the lower distance; every relaxation of its share here
// would be dominated then, so the share is dropped (claim: the distance copy
// this level's atomicMin updates).
template <int P>
__device__ __forceinline__ Window load_window(const Args& a, const uint32_t* claim, uint32_t base,
                                              uint32_t wn, uint32_t gbase, uint32_t t0, uint32_t t1,
                                              int lane, uint32_t L, uint32_t& blocks) {
  Window w{0, 0, 0, 0u, 0u, 0, 0, 0, 0, 0u, 0, false, false};
  uint32_t ns = 0;
  bool bad = false, ends = false;
  if ((uint32_t)lane < wn) {
    const int4 rec = a.rec[base + lane];
    const int32_t q = a.rec_q[base + lane];
    uint32_t pnow = 0xFFFFFFFFu;  // the parent's distance now (SSSP)
    if (P == PROB_SSSP) {
      w.ps = a.rec_slot[base + lane];
      if ((uint32_t)w.ps < (uint32_t)a.slots) pnow = coherent_load(&claim[w.ps]);
      else bad = true;
    }
    int32_t CF = 1;
    if ((uint32_t)q < (uint32_t)a.nq) {
      const Query Q = a.q[q];
      CF = max(Q.CF, 1);
      w.vbase = Q.vbase;
      w.n = Q.n;
      w.sbase = Q.slot0 - Q.vbase;
      w.lv = (int32_t)(L + 1) - Q.lstart;
    } else {
      bad = true;
    }
    const int32_t deg = rec.y;
    if (deg <= 0 || rec.x < 0 || (int64_t)rec.x + deg > (int64_t)a.m) bad = true;
    if (!bad) {
      // coarsened grid of the record (Sec. IV-B): ceil(ceil(deg / CB) / CF)
      // blocks of CF * CB edges, starting at global block G
      const uint32_t span = (uint32_t)CF * (uint32_t)a.CB;
      const uint32_t cgr = ceil_div((uint32_t)deg, span);
      const uint32_t G = gbase + (uint32_t)rec.z;
      const uint32_t lo = max(G, t0), hi = min(G + cgr, t1);
      ends = G + cgr >= t1;
      const bool superseded = P == PROB_SSSP && pnow < (uint32_t)rec.w;
      if (hi > lo && !superseded) {
        w.rs = rec.x;
        w.elo = (int32_t)((lo - G) * span);
        w.ehi = min(deg, (int32_t)((hi - G) * span));
        ns = ceil_div((uint32_t)(w.ehi - w.elo), 64u);
        blocks += hi - lo;
      }
      w.du = (uint32_t)rec.w;
    }
  }
  const uint32_t incl = wave_incl_scan(ns, lane);
  w.excl = incl - ns;
  w.nslices = __shfl(incl, 63, 64);
  w.last = __any(ends);
  w.bad = __any(bad);
  return w;
}

// One wave runs a contiguous share [t0, t1) of the level's aggregated child
// blocks: the parent of its first block is found by search (the
// disaggregation of Sec. V-A), then records are taken 64 at a time and their
// slices U at a time.
template <int P, bool TM, bool NT>
__global__ __launch_bounds__(PB) void child_kernel(Args a, uint32_t step) {
  __shared__ int32_t s_stage[NW][STAGE];
  __shared__ uint32_t s_bc[NW + 8];
  __shared__ uint32_t s_qpre[NQD + 1];
  __shared__ uint32_t s_qnd[NQD];
  __shared__ unsigned long long s_stats[NSTAT];

  const int tid = threadIdx.x, lane = tid & 63, wave = tid >> 6;
  State* st = a.st;
  uint64_t t_entry = 0;
  if (TM) t_entry = realtime();
  PhaseClock<TM> pc;
  pc.start();
  if (st->done || st->error) return;
  const uint32_t L = st->base + step;
  LevelSet* cur = &st->set[L % 3];
  int32_t* fout = (L & 1) ? a.front0 : a.front1;

  // aggregated child blocks of this level, queue by queue
  if (wave == 0) {
    const unsigned long long c = lane < NQD ? cur->qctr[lane] : 0ull;
    const uint32_t incl = wave_incl_scan((uint32_t)c, lane);
    if (lane < NQD) {
      s_qnd[lane] = (uint32_t)(c >> 32);
      s_qpre[lane + 1] = incl;
    }
    if (lane == 0) s_qpre[0] = 0;
  }
  if (tid < NSTAT) s_stats[tid] = 0;
  __syncthreads();
  const uint32_t B = s_qpre[NQD];
  if (B == 0) return;
  const uint32_t vm = cur->vmode;
  const Vis vis = vis_of<P>(a, vm & 1u, (vm & 2u) != 0);
  // Blocks of the level for this wave.  dyn_pct = 0: an even share of all B.
  // Otherwise the blocks are split into one range per XCD group (workgroups w
  // with the same w % 8, which run on the same XCD); a wave takes an even
  // share of (100 - dyn_pct)% of its group's range, then claims chunks of the
  // rest from its group's counter until none is left, as a hardware block
  // scheduler hands out the blocks of a grid.
  uint32_t t0, t1, dyn0 = 0, dyn1 = 0, csz = 1, xg = 0;
  if (a.dyn_pct == 0 || gridDim.x % NQD) {
    const uint32_t nwaves = gridDim.x * NW, gw = blockIdx.x * NW + wave;
    t0 = (uint32_t)((uint64_t)gw * B / nwaves);
    t1 = (uint32_t)((uint64_t)(gw + 1) * B / nwaves);
  } else {
    xg = blockIdx.x % NQD;
    const uint32_t nwx = (gridDim.x / NQD) * NW, k = (blockIdx.x / NQD) * NW + wave;
    const uint32_t r0 = (uint32_t)((uint64_t)xg * B / NQD);
    const uint32_t r1 = (uint32_t)((uint64_t)(xg + 1) * B / NQD);
    const uint32_t share = (uint32_t)((uint64_t)(r1 - r0) * (uint32_t)(100 - a.dyn_pct) / 100u) / nwx;
    t0 = r0 + k * share;
    t1 = t0 + share;
    dyn0 = r0 + nwx * share;
    dyn1 = r1;
    csz = max(1u, (dyn1 - dyn0) / (2u * nwx));  // about two chunks per wave
  }
  // wave-uniform by construction (scalar registers)
  t0 = __builtin_amdgcn_readfirstlane(t0);
  t1 = __builtin_amdgcn_readfirstlane(t1);
  dyn0 = __builtin_amdgcn_readfirstlane(dyn0);
  dyn1 = __builtin_amdgcn_readfirstlane(dyn1);
  csz = __builtin_amdgcn_readfirstlane(csz);
  Counters cn{0, 0, 0, 0, 0, 0, 0};
  Stage s{s_stage[wave], 0u};
  pc.mark(TP_LAUNCH);  // reading the level's published grids

  bool failed = false;
  while (true) {
    if (t0 < t1) {
      // disaggregation of the first block (Sec. V-A): queue, descriptor, record
      uint32_t q = 0;
      while (t0 >= s_qpre[q + 1]) ++q;
      const int4* dq = a.desc + (size_t)q * a.desc_cap;
      const uint32_t tq = t0 - s_qpre[q];
      uint32_t d = wave_upper_search(s_qnd[q], tq, lane, [&](uint32_t p) { return (uint32_t)dq[p].z; });
      int4 dd = dq[d];
      uint32_t r = wave_upper_search((uint32_t)dd.y, tq - (uint32_t)dd.z, lane,
                                     [&](uint32_t p) { return (uint32_t)a.rec[dd.x + p].z; });
      constexpr int U = 8;
      while (true) {
        const uint32_t wn = min(64u, (uint32_t)dd.y - r);
        const Window win = load_window<P>(a, vis.claim, (uint32_t)dd.x + r, wn,
                                          s_qpre[q] + (uint32_t)dd.z, t0, t1, lane, L, cn.child);
        pc.mark(TP_DISAGG);
        if (win.bad) {
          if (lane == 0) set_error(st, ERR_CAPACITY);
          failed = true;
          break;
        }
        // Coarsening loop (Sec. IV-B): a coarsened block covers original blocks
        // j*CF .. j*CF+CF-1 of CB lanes, the contiguous edges [j*CF*CB,
        // (j+1)*CF*CB) of its row, taken here 64 lanes at a time.
        // SSSP: the parents' distances are loaded again with each batch and
        // checked at the next one (by then the load has returned), so shares of
        // parents lowered while the wave runs them are cut short.
        uint32_t pnow = 0xFFFFFFFFu;
        for (uint32_t x0 = 0; x0 < win.nslices; x0 += U) {
          int32_t v[U], out[U];
          uint32_t w[U];
          Elem c[U];
          unsigned long long sup = 0ull;  // records whose parent was lowered
          if (P == PROB_SSSP) {
            sup = __ballot((uint32_t)lane < wn && pnow < win.du);
            if ((uint32_t)lane < wn) pnow = coherent_load(&vis.claim[win.ps]);
          }
  #pragma unroll
          for (int u = 0; u < U; ++u) {
            v[u] = -1;
            w[u] = 0u;
            c[u] = Elem{0, 0, 0, 0, 0u};
            const uint32_t x = x0 + u;
            if (x < win.nslices) {
              // record of slice x: the last lane whose scan start is <= x
              const uint32_t k =
                  (uint32_t)__popcll(__ballot((uint32_t)lane < wn && win.excl <= x)) - 1u;
              const int32_t rs = __builtin_amdgcn_readlane(win.rs, k);
              const int32_t e0 = rs + __builtin_amdgcn_readlane(win.elo, k) +
                                 (int32_t)((x - (uint32_t)__builtin_amdgcn_readlane((int32_t)win.excl, k)) * 64u);
              const int32_t e1 = rs + __builtin_amdgcn_readlane(win.ehi, k);
              c[u].vbase = __builtin_amdgcn_readlane(win.vbase, k);
              c[u].n = __builtin_amdgcn_readlane(win.n, k);
              c[u].sbase = __builtin_amdgcn_readlane(win.sbase, k);
              c[u].lv = __builtin_amdgcn_readlane(win.lv, k);
              c[u].du = (uint32_t)__builtin_amdgcn_readlane((int32_t)win.du, k);
              if (e0 + lane < e1 && !((sup >> k) & 1ull)) {
                // NT (with found bytes: single traversals, the serving
                // engine): the level's adjacency (and weights) are read once,
                // so their lines leave L2 first and the probed bitmaps or
                // distances and the found bytes stay.  A batch of many
                // traversals over few graphs reads each adjacency again.
                v[u] = NT ? __builtin_nontemporal_load(&a.col[e0 + lane]) : a.col[e0 + lane];
                if (P == PROB_SSSP)
                  w[u] = NT ? __builtin_nontemporal_load(&a.w[e0 + lane]) : a.w[e0 + lane];
              }
            }
          }
          if (a.count_stats) {  // edges run (lane 0 keeps the wave's count)
  #pragma unroll
            for (int u = 0; u < U; ++u) {
              const uint32_t nv = (uint32_t)__popcll(__ballot(v[u] >= 0));
              if (lane == 0) cn.echild += nv;
            }
          }
          visit_batch<P, U>(a, vis, v, w, c, L, out);
  #pragma unroll
          for (int u = 0; u < U; ++u) stage_push(s, out[u] >= 0, out[u], a, cur, fout, lane);
        }
        pc.mark(TP_CHILD);
        if (win.last) break;
        // next window: rest of this descriptor, else the next one (next queue
        // if need be)
        r += wn;
        if (r >= (uint32_t)dd.y) {
          r = 0;
          if (++d >= s_qnd[q]) {
            d = 0;
            do { ++q; } while (q < NQD && s_qnd[q] == 0);
            if (q >= NQD) {
              if (lane == 0) set_error(st, ERR_CAPACITY);
              failed = true;
              break;
            }
            dq = a.desc + (size_t)q * a.desc_cap;
          }
          dd = dq[d];
        }
      }
    }
    // next chunk of the group's dynamic part, if any is left
    if (failed || dyn0 >= dyn1) break;
    uint32_t j = 0;
    if (lane == 0) j = atomicAdd(&cur->cclaim[xg][0], 1u);
    j = __builtin_amdgcn_readfirstlane(j);
    const uint64_t c0 = (uint64_t)dyn0 + (uint64_t)j * csz;
    if (c0 >= dyn1) break;
    t0 = (uint32_t)c0;
    t1 = min(t0 + csz, dyn1);
    pc.mark(TP_LAUNCH);
  }
  block_flush(s, a, cur, fout, tid, s_bc);
  add_stats(a, s_stats, cn, tid);
  pc.mark(TP_CHILD);
  tm_write<TM>(a, pc, TK_CHILD, L, t_entry, tid);
}

// ------------------------------------------------------------ harvest kernel
// The last kernel of a level step with found bytes (Args::hint).  SSSP: every
// found vertex was improved at this level; it joins the next frontier once and
// its byte is cleared for the next level.  BFS with per-XCD copies, after a
// wide level: a found vertex that bitmap 0 lacks was discovered at this level.  It gets its level, its
// bit in bitmap 0 and a place in the next frontier (in slot order, which also
// makes the next level's row loads mostly consecutive).  One lane per slot: a
// run of 64 slots is 64 found bytes and the two bitmap words they map to, which
// the wave that reads them owns for the kernel.  Found bytes are never cleared within a
// traversal: one set at an earlier level belongs to a vertex that the harvest
// of that level put into bitmap 0.  Admission clears a query's found bytes,
// and a serving engine clears all of them when it is created
// (clear_found_kernel), so slots outside every admitted query hold none.  A
// narrow level claimed and appended in place, and its harvest returns at once.
template <int P, bool TM>
__global__ __launch_bounds__(PB) void harvest_kernel(Args a, uint32_t step) {
  __shared__ int32_t s_stage[NW][STAGE];
  __shared__ uint32_t s_bc[NW + 8];

  const int tid = threadIdx.x, lane = tid & 63, wave = tid >> 6;
  State* st = a.st;
  uint64_t t_entry = 0;
  if (TM) t_entry = realtime();
  PhaseClock<TM> pc;
  pc.start();
  if (st->done || st->error) return;
  const uint32_t L = st->base + step;
  LevelSet* cur = &st->set[L % 3];
  if (P == PROB_BFS && !(cur->vmode & 2u)) return;
  int32_t* fout = (L & 1) ? a.front0 : a.front1;
  Stage s{s_stage[wave], 0u};
  const uint32_t n = (uint32_t)a.slots;
  // BFS: a single traversal has one level value; with several queries it is
  // looked up per found vertex
  const int32_t lv1 = P == PROB_BFS ? (int32_t)(L + 1) - a.q[0].lstart : 0;
  // HU runs of 64 slots per wave and round, all their loads issued first
  constexpr int HU = HARVEST_RUNS;
  for (uint32_t b = (blockIdx.x * NW + wave) * (64u * HU); b < n; b += gridDim.x * PB * HU) {
    uint32_t c[HU];
    bool f[HU];
#pragma unroll
    for (int k = 0; k < HU; ++k) {
      const uint32_t v = b + (uint32_t)k * 64u + (uint32_t)lane;
      c[k] = (P == PROB_BFS && v < n) ? a.visit[v >> 5] : 0u;
      f[k] = v < n && a.found[v] != 0;
    }
#pragma unroll
    for (int k = 0; k < HU; ++k) {
      const uint32_t v = b + (uint32_t)k * 64u + (uint32_t)lane;
      if (P == PROB_SSSP) {
        if (f[k]) a.found[v] = 0;
        stage_push(s, f[k], (int32_t)v, a, cur, fout, lane);
        continue;
      }
      const bool nw = f[k] && !((c[k] >> (v & 31)) & 1u);
      const unsigned long long m = __ballot(nw);
      if (m) {  // wave-uniform
        if (nw) a.level[v] = a.nq == 1 ? lv1 : (int32_t)(L + 1) - a.q[a.qmap[v >> 5]].lstart;
        // lanes 0 and 32 own the words of the run's slots 0 .. 31 and 32 .. 63
        if ((lane & 31) == 0) {
          const uint32_t bits = (uint32_t)(m >> (lane & 32));
          if (bits) a.visit[v >> 5] = c[k] | bits;
        }
      }
      stage_push(s, nw, (int32_t)v, a, cur, fout, lane);
    }
  }
  block_flush(s, a, cur, fout, tid, s_bc);
  pc.mark(TP_CHILD);
  tm_write<TM>(a, pc, TK_HARVEST, L, t_entry, tid);
}

// ------------------------------------------------------------ init / admit / advance
// Traversal-set start: level sets and counters cleared.  Queries are
// started by admit_kernel.
__global__ __launch_bounds__(PB) void init_kernel(Args a) {
  const uint32_t gsz = gridDim.x * PB;
  const uint32_t gid = blockIdx.x * PB + threadIdx.x;
  for (uint32_t i = gid; i < 3u * (uint32_t)a.ngroups_cap; i += gsz) {
    a.grp_packed[i] = 0;
    a.grp_done[i] = 0;
  }
  for (uint32_t i = gid; i < (uint32_t)(MAX_GRID * NSTAT); i += gsz) a.stats[i] = 0;
  uint32_t* stw = (uint32_t*)a.st;
  for (uint32_t i = gid; i < sizeof(State) / 4; i += gsz) stw[i] = 0;
}

// Starts the queries list[0 .. count) at level index L = st->base: their
// outputs set to "unreached" except the source, their visit state cleared and
// their 32-slot chunks mapped to them.  Query list[k] is served by the
// workgroups [pre[k], pre[k + 1]) (pre = list + count, a host-built prefix of
// per-query workgroup counts proportional to n), so a batch of many small
// queries does not leave most of the grid idle.  `reset` (host-known: every
// earlier query has finished) also clears the level sets, whose fills are then
// stale.
template <int P>
__global__ __launch_bounds__(PB) void admit_kernel(Args a, const int32_t* list, int32_t count,
                                                   int32_t reset) {
  State* st = a.st;
  const int32_t* pre = list + count;
  // query of this workgroup: largest k with pre[k] <= blockIdx.x
  int32_t lo = 0, hi = count;
  while (hi - lo > 1) {
    const int32_t mid = (lo + hi) >> 1;
    if (pre[mid] <= (int32_t)blockIdx.x) lo = mid; else hi = mid;
  }
  const int32_t qi = list[lo];
  const uint32_t j = blockIdx.x - (uint32_t)pre[lo];
  const uint32_t stride = (uint32_t)(pre[lo + 1] - pre[lo]) * PB;
  const Query Q = a.q[qi];
  const uint32_t s0 = (uint32_t)Q.slot0, src = (uint32_t)Q.src;
  for (uint32_t v = j * PB + threadIdx.x; v < (uint32_t)Q.n; v += stride) {
    if (P == PROB_BFS) {
      a.level[s0 + v] = (v == src) ? 0 : -1;
    } else {
      const uint32_t d = (v == src) ? 0u : 0xFFFFFFFFu;
      a.dist[s0 + v] = d;
      a.dist2[s0 + v] = d;
      if (!a.hint) a.visit[s0 + v] = 0u;  // iteration stamps
    }
  }
  const uint32_t words = ((uint32_t)Q.n + 31) / 32;
  for (uint32_t i = j * PB + threadIdx.x; i < words; i += stride) {
    a.qmap[s0 / 32 + i] = qi;
    if (P == PROB_BFS) {
      const uint32_t x = (i == src >> 5) ? (1u << (src & 31)) : 0u;
      a.visit[s0 / 32 + i] = x;  // both bitmaps hold the source
      a.visit[(size_t)a.vwords + s0 / 32 + i] = x;
      if (a.hint) {  // the per-XCD copies hold the source too; nothing found yet
        for (uint32_t h = 0; h < (uint32_t)NHINT; ++h) a.visit[(size_t)(2 + h) * a.vwords + s0 / 32 + i] = x;
        uint32_t* f = (uint32_t*)(a.found + (size_t)(s0 / 32 + i) * 32);
        for (int k = 0; k < 8; ++k) f[k] = 0u;
      }
    } else if (a.hint) {  // SSSP: nothing found yet
      uint32_t* f = (uint32_t*)(a.found + (size_t)(s0 / 32 + i) * 32);
      for (int k = 0; k < 8; ++k) f[k] = 0u;
    }
  }
  if (reset) {
    const uint32_t gsz = gridDim.x * PB;
    const uint32_t gid = blockIdx.x * PB + threadIdx.x;
    uint32_t* sw = (uint32_t*)&st->set[0];
    for (uint32_t i = gid; i < 3 * sizeof(LevelSet) / 4; i += gsz) sw[i] = 0;
    for (uint32_t i = gid; i < 3u * (uint32_t)a.ngroups_cap; i += gsz) {
      a.grp_packed[i] = 0;
      a.grp_done[i] = 0;
    }
  }
}

// BFS with per-XCD copies: every found byte of the workspace cleared (a
// serving engine's output arena has slots that no query has been admitted to
// yet; the harvest kernel must see no found vertex there).
__global__ __launch_bounds__(PB) void clear_found_kernel(Args a) {
  uint32_t* f = (uint32_t*)a.found;
  const uint32_t nw = (uint32_t)a.vwords * 8u;
  for (uint32_t i = blockIdx.x * PB + threadIdx.x; i < nw; i += gridDim.x * PB) f[i] = 0u;
}

// Second half of admission (after admit_kernel): sources into frontier L.
__global__ void admit_sources_kernel(Args a, const int32_t* list, int32_t count) {
  State* st = a.st;
  const uint32_t L = st->base;
  LevelSet* ls = &st->set[(L + 2) % 3];  // fills of frontier L
  int32_t* fin = (L & 1) ? a.front1 : a.front0;
  const int32_t k = (int32_t)(blockIdx.x * blockDim.x + threadIdx.x);
  if (k < count) {
    Query* Q = &a.q[list[k]];
    Q->lstart = (int32_t)L;
    Q->last = (int32_t)L;
    const uint32_t pos = atomicAdd(&ls->fcnt[NQF], 1u);
    if (pos < (uint32_t)a.slots) fin[(size_t)NQF * a.fcap + pos] = Q->slot0 + Q->src;
    else set_error(st, ERR_CAPACITY);
  }
  if (k == 0) st->done = 0;
}

__global__ void advance_kernel(State* st, uint32_t steps) {
  if (threadIdx.x == 0 && blockIdx.x == 0) st->base += steps;
}

// ---------------------------------------------------------------- tables
template <int P, int PH, bool TM>
static const void* parent_for(int g) {
  switch (g) {
    case AGG_NONE: return (const void*)parent_kernel<P, AGG_NONE, PH, TM>;
    case AGG_WAVE: return (const void*)parent_kernel<P, AGG_WAVE, PH, TM>;
    case AGG_BLOCK: return (const void*)parent_kernel<P, AGG_BLOCK, PH, TM>;
    case AGG_MULTI: return (const void*)parent_kernel<P, AGG_MULTI, PH, TM>;
    default: return nullptr;
  }
}

template <bool TM>
static const void* parent_ptr(int problem, int gran) {
  if (gran == AGG_FLAT)
    return problem == PROB_BFS ? (const void*)parent_kernel<PROB_BFS, AGG_FLAT, PH_BOTH, TM>
                               : (const void*)parent_kernel<PROB_SSSP, AGG_FLAT, PH_BOTH, TM>;
  return problem == PROB_BFS ? parent_for<PROB_BFS, PH_BOTH, TM>(gran)
                             : parent_for<PROB_SSSP, PH_LIST, TM>(gran);
}

// BFS, and the flat kernel: both passes in one kernel.  SSSP with child
// kernels: pass 1, the child kernel, then pass 2 (serial_kernel_ptr).
const void* parent_kernel_ptr(int problem, int gran, bool timed) {
  return timed ? parent_ptr<true>(problem, gran) : parent_ptr<false>(problem, gran);
}

const void* serial_kernel_ptr(int problem, int gran, bool timed) {
  if (problem == PROB_BFS || gran == AGG_FLAT) return nullptr;
  return timed ? parent_for<PROB_SSSP, PH_SERIAL, true>(gran)
               : parent_for<PROB_SSSP, PH_SERIAL, false>(gran);
}

const void* harvest_kernel_ptr(int problem, bool timed) {
  if (problem == PROB_BFS)
    return timed ? (const void*)harvest_kernel<PROB_BFS, true>
                 : (const void*)harvest_kernel<PROB_BFS, false>;
  return timed ? (const void*)harvest_kernel<PROB_SSSP, true>
               : (const void*)harvest_kernel<PROB_SSSP, false>;
}

template <bool TM>
static const void* child_ptr(int problem, bool nt) {
  if (problem == PROB_BFS)
    return nt ? (const void*)child_kernel<PROB_BFS, TM, true>
              : (const void*)child_kernel<PROB_BFS, TM, false>;
  return nt ? (const void*)child_kernel<PROB_SSSP, TM, true>
            : (const void*)child_kernel<PROB_SSSP, TM, false>;
}

const void* child_kernel_ptr(int problem, bool timed, bool nt) {
  return timed ? child_ptr<true>(problem, nt) : child_ptr<false>(problem, nt);
}

const void* init_kernel_ptr(int) { return (const void*)init_kernel; }

const void* admit_kernel_ptr(int problem) {
  return problem == PROB_BFS ? (const void*)admit_kernel<PROB_BFS>
                             : (const void*)admit_kernel<PROB_SSSP>;
}

const void* admit_sources_kernel_ptr() { return (const void*)admit_sources_kernel; }

const void* clear_found_kernel_ptr() { return (const void*)clear_found_kernel; }

const void* advance_kernel_ptr() { return (const void*)advance_kernel; }

}  // namespace dpo
