// Device code: level-synchronous nested-parallel BFS / SSSP for gfx950.
//
// One level step is one persistent kernel.  Workgroups (256 lanes = 4 wave64)
// first claim virtual parent blocks of 256 frontier entries (the parent
// grid), then turn into consumers of the child grids those parents
// "launched".  Per parent thread u with child-thread count deg(u)
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
// counters as one integer), pre-aggregated per block, and the last block of
// the group (group-wide done counter) publishes the aggregated grid.
//
// HIP has no device-side launch.  "Publishing" appends a descriptor {record
// segment, record count, global child-block base} to a queue through a second
// packed 64-bit counter (hi = descriptors, lo = child blocks), so descriptor
// bases grow with the descriptor index.  Consumers take global child-block
// tickets, find the descriptor by a wave-parallel 64-ary search over the
// bases, then their parent record by the same search over the scanned
// offsets (the disaggregation of Sec. V-A), and run the coarsening loop over
// CF original blocks of CB lanes (Sec. IV-B) with coalesced col_idx reads.
//
// Child body: BFS claims v in a visited bitmap (an L2-resident n-bit array)
// and writes level[v] = L + 1; SSSP relaxes dist[v] with atomicMin and
// queues v once per iteration through an iteration stamp.  Discovered vertices
// are staged per wave in LDS and appended to the next frontier with one atomic
// per flush.
#include <hip/hip_runtime.h>
#include <stdint.h>

#include "dpo_internal.h"

namespace dpo {

#define AGENT __HIP_MEMORY_SCOPE_AGENT

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

__device__ __forceinline__ uint64_t now_ticks() { return __builtin_amdgcn_s_memrealtime(); }

// Per-wave LDS staging of next-frontier vertices.
struct Stage {
  int32_t* buf;  // STAGE slots in LDS owned by this wave
  uint32_t cnt;  // wave-uniform fill
};

__device__ __noinline__ void stage_flush(Stage& s, const Args& a, int32_t* fout,
                                         uint32_t* fcount, int lane) {
  if (s.cnt == 0) return;
  uint32_t base = 0;
  if (lane == 0) base = atomicAdd(fcount, s.cnt);
  base = __shfl(base, 0, 64);
  wave_lds_sync();
  if ((uint64_t)base + s.cnt > (uint64_t)a.n) {
    if (lane == 0) set_error(a.st, ERR_CAPACITY);
  } else {
    for (uint32_t i = lane; i < s.cnt; i += 64) fout[base + i] = s.buf[i];
  }
  wave_lds_sync();
  s.cnt = 0;
}

// Wave-uniform call: every lane of the wave must reach it.
__device__ __forceinline__ void stage_push(Stage& s, bool found, int32_t v, const Args& a,
                                           int32_t* fout, uint32_t* fcount, int lane) {
  unsigned long long m = __ballot(found);
  if (m == 0) return;
  uint32_t c = (uint32_t)__popcll(m);
  if (s.cnt + c > STAGE) stage_flush(s, a, fout, fcount, lane);
  if (found) s.buf[s.cnt + lane_rank(m)] = v;
  s.cnt += c;
}

// Child body for one neighbour (one original child thread).
template <int P>
__device__ __forceinline__ bool visit(const Args& a, int32_t v, uint32_t wgt, uint32_t du,
                                      uint32_t L) {
  if ((uint32_t)v >= (uint32_t)a.n) {
    set_error(a.st, ERR_ARG);
    return false;
  }
  if (P == PROB_BFS) {
    uint32_t word = (uint32_t)v >> 5, bit = 1u << (v & 31);
    if (a.visit[word] & bit) return false;
    uint32_t old = atomicOr(&a.visit[word], bit);
    if (old & bit) return false;
    a.level[v] = (int32_t)(L + 1);
    return true;
  } else {
    uint32_t nd = du + wgt;
    if (nd >= a.dist[v]) return false;
    uint32_t old = atomicMin(&a.dist[v], nd);
    if (nd >= old) return false;
    uint32_t it = L + 1;
    if (a.visit[v] == it) return false;
    return atomicExch(&a.visit[v], it) != it;
  }
}

// Serial version of the child (Sec. III-B): the parent lane walks its own
// neighbours.  Wave-uniform loop so that appends stay wave-aggregated.
template <int P>
__device__ __forceinline__ void serial_children(const Args& a, int32_t start, int32_t cnt,
                                                uint32_t du, uint32_t L, Stage& s, int32_t* fout,
                                                uint32_t* fcount, int lane) {
  constexpr int U = 4;
  int32_t e = start;
  const int32_t end = start + cnt;
  while (__any(e < end)) {
    int32_t v[U];
    uint32_t w[U];
#pragma unroll
    for (int r = 0; r < U; ++r) {
      v[r] = (e + r < end) ? a.col[e + r] : -1;
      w[r] = (P == PROB_SSSP && e + r < end) ? a.w[e + r] : 0u;
    }
#pragma unroll
    for (int r = 0; r < U; ++r) {
      bool f = false;
      if (v[r] >= 0) f = visit<P>(a, v[r], w[r], du, L);
      stage_push(s, f, v[r], a, fout, fcount, lane);
    }
    e += U;
  }
}

// Wait until descriptor p of this level is published; returns its child-block
// base, or UINT32_MAX after the watchdog fired.
__device__ __forceinline__ uint32_t desc_base(const Args& a, uint32_t p, uint32_t L) {
  unsigned long long b = __hip_atomic_load(&a.desc_b[p], __ATOMIC_ACQUIRE, AGENT);
  if ((uint32_t)(b >> 32) == L + 1) return (uint32_t)b;
  const uint64_t t0 = now_ticks();
  for (;;) {
    __builtin_amdgcn_s_sleep(1);
    b = __hip_atomic_load(&a.desc_b[p], __ATOMIC_ACQUIRE, AGENT);
    if ((uint32_t)(b >> 32) == L + 1) return (uint32_t)b;
    if (now_ticks() - t0 > a.watchdog_ticks) {
      set_error(a.st, ERR_TIMEOUT);
      return UINT32_MAX;
    }
  }
}

struct Claim {
  int32_t start, deg, j;
  uint32_t du;
  int32_t quit;
};

// Wave 0 of a consumer workgroup: take a child-block ticket, wait for it to be
// published, and disaggregate it (Sec. V-A: binary search of the scanned grid
// sizes), here as 64-ary wave searches over descriptors, then records.
template <int G, int CF>
__device__ Claim claim_child(const Args& a, Ctr* c, uint32_t L, uint32_t ngroups, int lane) {
  Claim r{0, 0, 0, 0u, 1};
  uint32_t t = 0;
  if (lane == 0) t = atomicAdd(&c->child_ticket, 1u);
  t = __shfl(t, 0, 64);
  unsigned long long dc = __hip_atomic_load(&c->desc_ctr, __ATOMIC_RELAXED, AGENT);
  if (t >= (uint32_t)dc) {
    const uint64_t t0 = now_ticks();
    for (;;) {
      uint32_t gf = __hip_atomic_load(&c->groups_finished, __ATOMIC_ACQUIRE, AGENT);
      dc = __hip_atomic_load(&c->desc_ctr, __ATOMIC_RELAXED, AGENT);
      if (t < (uint32_t)dc) break;
      if (gf >= ngroups) return r;  // every group finished and t is past the end
      if (now_ticks() - t0 > a.watchdog_ticks) {
        set_error(a.st, ERR_TIMEOUT);
        return r;
      }
      __builtin_amdgcn_s_sleep(2);
    }
  }
  // descriptor search: largest d with base(d) <= t; bases grow with d
  const uint32_t ndesc = (uint32_t)(dc >> 32);
  uint32_t lo = 0, hi = ndesc;
  while (hi - lo > 1) {
    const uint32_t step = (hi - lo + 63) / 64;
    const uint32_t p = lo + (uint32_t)lane * step;
    const uint32_t b = (p < hi) ? desc_base(a, p, L) : 0u;
    if (__any(p < hi && b == UINT32_MAX)) return r;  // watchdog fired
    const bool le = p < hi && b <= t;
    const uint32_t k = (uint32_t)__popcll(__ballot(le));
    lo += (k - 1) * step;
    hi = min(lo + step, hi);
  }
  const uint32_t d = lo;
  const uint32_t base = desc_base(a, d, L);
  if (base == UINT32_MAX || d >= (uint32_t)a.desc_cap) return r;
  const unsigned long long da = a.desc_a[d];
  const uint32_t rec_base = (uint32_t)da, nrec = (uint32_t)(da >> 32);
  const uint32_t tt = t - base;
  if (nrec == 0 || (uint64_t)rec_base + nrec > (uint64_t)a.n) {
    if (lane == 0) set_error(a.st, ERR_CAPACITY);
    return r;
  }
  // record search: largest q with off(q) <= tt; offsets strictly increase
  lo = 0;
  hi = nrec;
  while (hi - lo > 1) {
    const uint32_t step = (hi - lo + 63) / 64;
    const uint32_t p = lo + (uint32_t)lane * step;
    bool le = false;
    if (p < hi) le = (uint32_t)a.rec[rec_base + p].z <= tt;
    const uint32_t k = (uint32_t)__popcll(__ballot(le));
    lo += (k - 1) * step;
    hi = min(lo + step, hi);
  }
  const int4 rc = a.rec[rec_base + lo];
  r.start = rc.x;
  r.deg = rc.y;
  r.j = (int32_t)(tt - (uint32_t)rc.z);
  r.du = (uint32_t)rc.w;
  const int32_t gdim = (rc.y + a.CB - 1) / a.CB;
  if (rc.y <= 0 || rc.x < 0 || (int64_t)rc.x + rc.y > (int64_t)a.m || r.j < 0 ||
      r.j >= (gdim + CF - 1) / CF) {
    if (lane == 0) set_error(a.st, ERR_CAPACITY);
    return r;
  }
  r.quit = 0;
  return r;
}

// Publish one aggregated child grid: records [rec_base, rec_base + nrec) with
// `total` coarsened child blocks.  Called by one lane.
__device__ __forceinline__ void publish(const Args& a, Ctr* c, uint32_t rec_base, uint32_t nrec,
                                        uint32_t total, uint32_t L) {
  const unsigned long long old =
      atomicAdd(&c->desc_ctr, ((unsigned long long)1 << 32) | (unsigned long long)total);
  const uint32_t d = (uint32_t)(old >> 32), base = (uint32_t)old;
  if (d >= (uint32_t)a.desc_cap) {
    set_error(a.st, ERR_CAPACITY);
    return;
  }
  a.desc_a[d] = ((unsigned long long)nrec << 32) | rec_base;
  __hip_atomic_store(&a.desc_b[d], ((unsigned long long)(L + 1) << 32) | base, __ATOMIC_RELEASE,
                     AGENT);
}

enum { S_FRONT = 0, S_SERIAL, S_REC, S_CHILD, S_ESER, S_ECHILD, S_DESC, S_N };

template <int P, int G, int CF>
__global__ __launch_bounds__(PB) void step_kernel(Args a) {
  __shared__ int32_t s_stage[NW][STAGE];
  __shared__ uint32_t s_scan[2 * NW];
  __shared__ uint32_t s_bc[4];
  __shared__ Claim s_claim;
  __shared__ unsigned long long s_stats[S_N];

  const int tid = threadIdx.x, lane = tid & 63, wave = tid >> 6;
  State* st = a.st;
  if (st->done || st->error) return;
  const uint32_t L = st->level;
  const uint32_t F = st->fcount[L % 3];
  if (F == 0) return;
  const uint32_t cur = L % 3, nxt = (L + 1) % 3, nn = (L + 2) % 3;
  Ctr* c = &st->ctr[cur];
  const int32_t* fin = (L & 1) ? a.front1 : a.front0;
  int32_t* fout = (L & 1) ? a.front0 : a.front1;
  uint32_t* fcount = &st->fcount[nxt];

  // Counters of the following step are idle now: clear them here.
  if (blockIdx.x == 0 && tid == 0) {
    Ctr* z = &st->ctr[nxt];
    z->parent_claim = 0;
    z->child_ticket = 0;
    z->groups_finished = 0;
    z->exit_count = 0;
    z->desc_ctr = 0;
    st->fcount[nn] = 0;
  }
  if (G == AGG_MULTI) {
    for (int i = blockIdx.x * PB + tid; i < a.ngroups_cap; i += gridDim.x * PB) {
      a.grp_packed[nxt * a.ngroups_cap + i] = 0;
      a.grp_done[nxt * a.ngroups_cap + i] = 0;
    }
  }
  if (tid < S_N) s_stats[tid] = 0;
  __syncthreads();

  Stage s{s_stage[wave], 0u};
  uint32_t n_front = 0, n_serial = 0, n_rec = 0, n_desc = 0, n_child = 0;
  uint64_t e_serial = 0, e_child = 0;

  const uint32_t nvb = (F + PB - 1) / PB;
  if (G == AGG_FLAT) {
    // No nesting: thread per frontier vertex, serial neighbour loop.
    for (uint32_t i0 = blockIdx.x * PB; i0 < F; i0 += gridDim.x * PB) {
      const uint32_t i = i0 + tid;
      int32_t start = 0, deg = 0;
      uint32_t du = 0;
      if (i < F) {
        const int32_t u = fin[i];
        start = a.rp[u];
        deg = a.rp[u + 1] - start;
        if (P == PROB_SSSP) du = a.dist[u];
        ++n_front;
        if (deg > 0) { ++n_serial; e_serial += deg; }
      }
      serial_children<P>(a, start, deg, du, L, s, fout, fcount, lane);
    }
  } else {
    const uint32_t ngroups = (G == AGG_MULTI) ? (nvb + a.k - 1) / a.k : nvb;
    // ---------------- parent phase: claim virtual parent blocks
    for (;;) {
      if (tid == 0) s_bc[0] = atomicAdd(&c->parent_claim, 1u);
      __syncthreads();
      const uint32_t vb = s_bc[0];
      __syncthreads();
      if (vb >= nvb) break;
      const uint32_t i = vb * PB + tid;
      int32_t start = 0, deg = 0;
      uint32_t du = 0;
      if (i < F) {
        const int32_t u = fin[i];
        start = a.rp[u];
        deg = a.rp[u + 1] - start;
        if (P == PROB_SSSP) du = a.dist[u];
        ++n_front;
      }
      const bool launch = deg > 0 && deg >= a.T;
      const bool ser = deg > 0 && !launch;
      if (ser) { ++n_serial; e_serial += deg; }
      // thresholded children run in the parent (Sec. III-B)
      serial_children<P>(a, start, ser ? deg : 0, du, L, s, fout, fcount, lane);
      // coarsened grid size (Sec. IV-B)
      const uint32_t gdim = launch ? (uint32_t)((deg + a.CB - 1) / a.CB) : 0u;
      const uint32_t cg = (gdim + CF - 1) / CF;
      if (launch) ++n_rec;

      if (G == AGG_NONE) {
        // one grid per launching parent
        if (launch) {
          const unsigned long long old =
              atomicAdd(&c->desc_ctr, ((unsigned long long)1 << 32) | (unsigned long long)cg);
          const uint32_t d = (uint32_t)(old >> 32), base = (uint32_t)old;
          if (d < (uint32_t)a.desc_cap) {
            a.rec[d] = make_int4(start, deg, 0, (int32_t)du);
            a.desc_a[d] = ((unsigned long long)1 << 32) | d;
            __hip_atomic_store(&a.desc_b[d], ((unsigned long long)(L + 1) << 32) | base,
                               __ATOMIC_RELEASE, AGENT);
            ++n_desc;
          } else {
            set_error(st, ERR_CAPACITY);
          }
        }
        __syncthreads();
        if (tid == 0) __hip_atomic_fetch_add(&c->groups_finished, 1u, __ATOMIC_RELEASE, AGENT);
      } else if (G == AGG_WAVE) {
        const unsigned long long m = __ballot(launch);
        if (m) {
          const uint32_t nrec = (uint32_t)__popcll(m);
          const uint32_t incl = wave_incl_scan(launch ? cg : 0u, lane);
          const uint32_t total = __shfl(incl, 63, 64);
          const uint32_t seg = vb * PB + wave * 64;
          if (launch)
            a.rec[seg + lane_rank(m)] = make_int4(start, deg, (int32_t)(incl - cg), (int32_t)du);
          __builtin_amdgcn_fence(__ATOMIC_RELEASE, "agent");
          if (lane == 0) { publish(a, c, seg, nrec, total, L); ++n_desc; }
        }
        __syncthreads();
        if (tid == 0) __hip_atomic_fetch_add(&c->groups_finished, 1u, __ATOMIC_RELEASE, AGENT);
      } else {
        // block-level scan of (launch, cg): wave scans, then across waves in LDS
        const unsigned long long m = __ballot(launch);
        const uint32_t incl = wave_incl_scan(launch ? cg : 0u, lane);
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
          if (launch)
            a.rec[seg + roff + lane_rank(m)] =
                make_int4(start, deg, (int32_t)(coff + incl - cg), (int32_t)du);
          __builtin_amdgcn_fence(__ATOMIC_RELEASE, "agent");
          __syncthreads();
          if (tid == 0) {
            if (nrec_b) { publish(a, c, seg, nrec_b, total_b, L); ++n_desc; }
            __hip_atomic_fetch_add(&c->groups_finished, 1u, __ATOMIC_RELEASE, AGENT);
          }
        } else {  // AGG_MULTI: group of k virtual blocks (Sec. V-A)
          const uint32_t g = vb / (uint32_t)a.k;
          const uint32_t seg = g * (uint32_t)a.k * PB;
          unsigned long long* gp = &a.grp_packed[cur * a.ngroups_cap + g];
          uint32_t* gd = &a.grp_done[cur * a.ngroups_cap + g];
          if (tid == 0) {
            unsigned long long old = 0;
            if (nrec_b)
              old = atomicAdd(gp, ((unsigned long long)nrec_b << 32) | (unsigned long long)total_b);
            s_bc[1] = (uint32_t)(old >> 32);
            s_bc[2] = (uint32_t)old;
          }
          __syncthreads();
          const uint32_t slot0 = s_bc[1], off0 = s_bc[2];
          if (launch)
            a.rec[seg + slot0 + roff + lane_rank(m)] =
                make_int4(start, deg, (int32_t)(off0 + coff + incl - cg), (int32_t)du);
          __builtin_amdgcn_fence(__ATOMIC_RELEASE, "agent");
          __syncthreads();
          if (tid == 0) {
            const uint32_t in_group = min((uint32_t)a.k, nvb - g * (uint32_t)a.k);
            const uint32_t done = __hip_atomic_fetch_add(gd, 1u, __ATOMIC_ACQ_REL, AGENT);
            if (done == in_group - 1) {
              const unsigned long long tot = __hip_atomic_load(gp, __ATOMIC_RELAXED, AGENT);
              const uint32_t nrec_g = (uint32_t)(tot >> 32);
              if (nrec_g) { publish(a, c, seg, nrec_g, (uint32_t)tot, L); ++n_desc; }
              __hip_atomic_fetch_add(&c->groups_finished, 1u, __ATOMIC_RELEASE, AGENT);
            }
          }
        }
      }
    }

    // ---------------- child phase: consume aggregated child grids
    for (;;) {
      if (wave == 0) {
        Claim cl = claim_child<G, CF>(a, c, L, ngroups, lane);
        if (lane == 0) s_claim = cl;
      }
      __syncthreads();
      const Claim cl = s_claim;
      __syncthreads();
      if (cl.quit) break;
      if (tid == 0) ++n_child;
      // coarsening loop (Sec. IV-B): original blocks j*CF .. j*CF+CF-1 of CB
      // lanes cover the contiguous edge range [j*CF*CB, (j+1)*CF*CB)
      const int32_t base_idx = cl.j * CF * a.CB;
      const int32_t lim = min(cl.deg - base_idx, CF * a.CB);
      const int32_t e0 = cl.start + base_idx;
      int32_t v[CF];
      uint32_t w[CF];
#pragma unroll
      for (int r = 0; r < CF; ++r) {
        const int32_t x = tid + r * PB;
        v[r] = (x < lim) ? a.col[e0 + x] : -1;
        w[r] = (P == PROB_SSSP && x < lim) ? a.w[e0 + x] : 0u;
      }
#pragma unroll
      for (int r = 0; r < CF; ++r) {
        if (r * PB < lim) {  // uniform across the workgroup
          bool f = false;
          if (v[r] >= 0) {
            ++e_child;
            f = visit<P>(a, v[r], w[r], cl.du, L);
          }
          stage_push(s, f, v[r], a, fout, fcount, lane);
        }
      }
    }
  }

  // ---------------- step end
  stage_flush(s, a, fout, fcount, lane);
  if (a.count_stats) {
    atomicAdd(&s_stats[S_FRONT], (unsigned long long)n_front);
    atomicAdd(&s_stats[S_SERIAL], (unsigned long long)n_serial);
    atomicAdd(&s_stats[S_REC], (unsigned long long)n_rec);
    atomicAdd(&s_stats[S_CHILD], (unsigned long long)n_child);
    atomicAdd(&s_stats[S_ESER], (unsigned long long)e_serial);
    atomicAdd(&s_stats[S_ECHILD], (unsigned long long)e_child);
    atomicAdd(&s_stats[S_DESC], (unsigned long long)n_desc);
  }
  __syncthreads();
  if (a.count_stats && tid < S_N && s_stats[tid]) atomicAdd(&st->stats[tid], s_stats[tid]);
  if (tid == 0) {
    const uint32_t old = __hip_atomic_fetch_add(&c->exit_count, 1u, __ATOMIC_ACQ_REL, AGENT);
    if (old == gridDim.x - 1) {
      const uint32_t nf = __hip_atomic_load(fcount, __ATOMIC_RELAXED, AGENT);
      st->levels_run = L + 1;
      st->level = L + 1;
      if (nf == 0) st->done = 1;
    }
  }
}

// Traversal start: outputs to "unreached", visit words cleared, descriptor
// flags cleared, counters zeroed, the source placed in frontier 0.
template <int P>
__global__ __launch_bounds__(PB) void init_kernel(Args a, int32_t src) {
  const uint32_t gsz = gridDim.x * PB;
  const uint32_t gid = blockIdx.x * PB + threadIdx.x;
  for (uint32_t v = gid; v < (uint32_t)a.n; v += gsz) {
    if (P == PROB_BFS) {
      a.level[v] = (v == (uint32_t)src) ? 0 : -1;
    } else {
      a.dist[v] = (v == (uint32_t)src) ? 0u : 0xFFFFFFFFu;
      a.visit[v] = 0u;
    }
  }
  if (P == PROB_BFS) {
    const uint32_t words = ((uint32_t)a.n + 31) / 32;
    for (uint32_t i = gid; i < words; i += gsz)
      a.visit[i] = (i == (uint32_t)src >> 5) ? (1u << (src & 31)) : 0u;
  }
  for (uint32_t i = gid; i < (uint32_t)a.desc_cap; i += gsz) a.desc_b[i] = 0;
  for (uint32_t i = gid; i < 3u * (uint32_t)a.ngroups_cap; i += gsz) {
    a.grp_packed[i] = 0;
    a.grp_done[i] = 0;
  }
  if (gid == 0) {
    State* st = a.st;
    st->level = 0;
    st->done = 0;
    st->error = 0;
    st->levels_run = 0;
    st->fcount[0] = 1;
    st->fcount[1] = 0;
    st->fcount[2] = 0;
    st->fcount[3] = 0;
    for (int k = 0; k < 3; ++k) {
      st->ctr[k].parent_claim = 0;
      st->ctr[k].child_ticket = 0;
      st->ctr[k].groups_finished = 0;
      st->ctr[k].exit_count = 0;
      st->ctr[k].desc_ctr = 0;
    }
    for (int k = 0; k < 8; ++k) st->stats[k] = 0;
    a.front0[0] = src;
  }
}

// ---------------------------------------------------------------- tables
template <int P, int G>
static const void* step_for_cf(int cf) {
  switch (cf) {
    case 1: return (const void*)step_kernel<P, G, 1>;
    case 2: return (const void*)step_kernel<P, G, 2>;
    case 4: return (const void*)step_kernel<P, G, 4>;
    case 8: return (const void*)step_kernel<P, G, 8>;
    case 16: return (const void*)step_kernel<P, G, 16>;
    default: return nullptr;
  }
}

template <int P>
static const void* step_for(int g, int cf) {
  switch (g) {
    case AGG_NONE: return step_for_cf<P, AGG_NONE>(cf);
    case AGG_WAVE: return step_for_cf<P, AGG_WAVE>(cf);
    case AGG_BLOCK: return step_for_cf<P, AGG_BLOCK>(cf);
    case AGG_MULTI: return step_for_cf<P, AGG_MULTI>(cf);
    case AGG_FLAT: return (const void*)step_kernel<P, AGG_FLAT, 1>;
    default: return nullptr;
  }
}

const void* step_kernel_ptr(int problem, int gran, int cf) {
  return problem == PROB_BFS ? step_for<PROB_BFS>(gran, cf) : step_for<PROB_SSSP>(gran, cf);
}

const void* init_kernel_ptr(int problem) {
  return problem == PROB_BFS ? (const void*)init_kernel<PROB_BFS>
                             : (const void*)init_kernel<PROB_SSSP>;
}

}  // namespace dpo
