// Shared declarations of the HIP library (device kernels and host driver).
#pragma once
#include <stddef.h>
#include <stdint.h>

namespace dpo {

constexpr int PB = 256;          // parent workgroup: 256 frontier entries per virtual block
constexpr int NW = PB / 64;      // wave64s per workgroup
constexpr int STAGE = 512;       // LDS slots per wave for next-frontier staging
constexpr int NQD = 8;           // descriptor queues (one per XCD: queue = virtual block % 8)
constexpr int NQF = 64;          // frontier queues (queue = workgroup % 64), plus one overflow
constexpr int MAX_GRID = 4096;   // persistent grid cap (rows of the per-workgroup counters)
constexpr int NSTAT = 8;
// parent kernel phases
constexpr int PH_BOTH = 0;    // pass 1 and pass 2
constexpr int PH_LIST = 1;    // pass 1; thresholded parents listed for PH_SERIAL
constexpr int PH_SERIAL = 2;  // pass 2 of the listed parents (after the child kernel)
constexpr uint32_t GROUP_EDGES = 1024;  // wave-run serial children: edges per group (about)
constexpr int MAX_QUERIES = 4096;  // per-query tables are staged in LDS
constexpr int ADMIT_CHUNK = 4096;  // output slots initialised per admit workgroup
constexpr int PRECHECK_MIN = 32;   // claim candidates per 512-lane batch above which
                                   // a coherent load precedes the atomics
constexpr int NHINT = 8;           // BFS per-XCD visited copies (Args::hint), one per XCD
constexpr int HARVEST_RUNS = 4;    // harvest kernel: 64-slot runs per wave and round
constexpr int HINT_AUTO_MIN_DEGREE = 8;  // DPO_HINT_AUTO: per-XCD copies from this average
                                         // degree (m / n) up

enum { PROB_BFS = 0, PROB_SSSP = 1 };
enum { AGG_NONE = 0, AGG_WAVE = 1, AGG_BLOCK = 2, AGG_MULTI = 3, AGG_FLAT = 4 };
// device error codes (stored as the negated dpo_status)
enum { ERR_ARG = 1, ERR_CAPACITY = 4, ERR_TIMEOUT = 5 };
enum { S_FRONT = 0, S_SERIAL, S_REC, S_CHILD, S_ESER, S_ECHILD, S_DESC };

// Phase timing (the timed instantiations of the level kernels only).  Each
// workgroup of each level kernel writes one row of TM_ROW words at
// tm[((level * TM_KINDS + kind) * MAX_GRID + workgroup) * TM_ROW]:
//   [0] realtime clock at entry, [1] at exit (constant-rate counter),
//   [2 + p] shader-clock cycles its waves spent in phase p (summed over the
//   workgroup's waves), [7] the largest total of one wave.
// Rows of levels >= TM_LEVELS are not written.
constexpr int TM_LEVELS = 64;
constexpr int TM_KINDS = 4;  // parent kernel, child kernel, thresholded children, harvest
constexpr int TM_ROW = 8;
enum { TK_PARENT = 0, TK_CHILD = 1, TK_SERIAL = 2, TK_HARVEST = 3 };
enum { TP_PARENT = 0, TP_AGG, TP_LAUNCH, TP_DISAGG, TP_CHILD, TP_N };

// Counters of one level; three sets rotate by level % 3 so that the parent
// kernel of level L can clear the set of level L + 1 while nobody uses it.
struct LevelSet {
  uint32_t fcnt[NQF + 1];              // next-frontier queue fills (+ overflow)
  uint32_t vmode;                      // visited copies of this level: bit 0 probed
                                       // buffer, bit 1 split (claims in the other one)
  uint32_t pad0[14];
  unsigned long long qctr[NQD];        // descriptor queues: hi32 count, lo32 child blocks
  uint32_t cclaim[NQD][32];            // child kernel: chunks claimed per XCD group (one
                                       // 128-byte line each)
};

struct State {
  uint32_t base;        // level index of step 0 of the current graph replay
  uint32_t done;        // set when a level starts with an empty frontier
  uint32_t error;       // first device error code, 0 = none
  uint32_t levels_run;  // index of the last non-empty level + 1
  uint32_t vsel[2];     // probed visited buffer of levels with parity 0 / 1
  uint32_t vstale[2];   // BFS: the other bitmap missed folds (a one-copy level ran)
  uint32_t pad[56];
  LevelSet set[3];
};

// One traversal ("query") of a batch.  Its outputs occupy the slots
// [slot0, slot0 + n) of the output arena; slot s is vertex s - slot0 + vbase of
// the CSR arena.
struct Query {
  int32_t slot0;   // first output slot
  int32_t n;       // vertices of its graph
  int32_t vbase;   // global id of its graph's vertex 0 in the CSR arena
  int32_t lstart;  // level index at which it started (its source is at level lstart)
  int32_t T;       // threshold of its size bucket
  int32_t CF;      // coarsening factor of its size bucket
  int32_t last;    // last level index with frontier entries (written by the kernels)
  int32_t src;     // source (local id)
};

// Kernel arguments (by value).  All pointers are device pointers.
struct Args {
  const int32_t* rp;
  const int32_t* col;
  const uint32_t* w;
  int32_t* level;                  // [slots] BFS output
  uint32_t* dist;                  // [slots] SSSP output (distance array 0)
  uint32_t* dist2;                 // [slots] SSSP distance array 1 (equal to dist at the end)
  State* st;
  Query* q;                        // [nq]
  unsigned long long* grp_packed;  // [3][ngroups_cap]: hi32 records, lo32 child blocks
  uint32_t* grp_done;              // [3][ngroups_cap]: blocks of the group finished
  int32_t* front0;                 // [NQF * fcap + slots]
  int32_t* front1;
  uint32_t* visit;                 // BFS: two bitmaps of vwords words, then NHINT per-XCD
                                   // copies; SSSP: stamps [slots]
  uint8_t* found;                  // [vwords * 32] bytes (Args::hint), set for the vertices
                                   // a level's child bodies find (BFS: wide levels) or
                                   // improve (SSSP); read by the harvest kernel
  int4* rec;                       // [slots] launch records {row start, deg, offset, parent dist}
  int32_t* rec_q;                  // [slots] query of each record
  int32_t* rec_slot;               // [slots] SSSP: slot of each record's parent
  int4* ser;                       // [slots rounded up to PB] thresholded parents
                                   // {row start, deg, slot, parent distance}
  int32_t* qmap;                   // [slots / 32] query owning each 32-slot chunk
  int4* desc;                      // [NQD][desc_cap] {record base, records, block base, -}
  unsigned long long* stats;       // [MAX_GRID][NSTAT], one row per workgroup
  uint32_t* sercnt;                // [MAX_GRID] listed thresholded parents per workgroup
  unsigned long long* tm;          // phase-timing rows (timed kernels only)
  int32_t slots;                   // total output slots (sum of the queries' n)
  int32_t m;                       // CSR arena entries
  int32_t nq;
  int32_t CB;
  int32_t k;
  int32_t ngroups_cap;
  int32_t desc_cap;                // per descriptor queue
  int32_t fcap;                    // per frontier queue
  int32_t count_stats;
  int32_t agg_threshold;           // wave / block granularity: fewer launching parents
                                   // than this launch individually (Sec. V-B)
  int32_t vwords;                  // words of one BFS bitmap (slots / 32)
  int32_t split_min;               // frontier size from which a level probes one
                                   // visited copy and updates the other
  int32_t serial_wave;             // thresholded children: run by the wave together
                                   // (1) or each in its parent's lane (0)
  int32_t dyn_pct;                 // child kernel: percent of each XCD group's blocks
                                   // that its waves claim in chunks (0 = even split)
  int32_t hint;                    // found bytes and the harvest kernel in use.  BFS:
                                   // per-XCD visited copies on wide levels (probed by the
                                   // XCD's workgroups, at visit + (2 + x) * vwords, x =
                                   // XCD), discoveries taken into bitmap 0 by the harvest;
                                   // SSSP: improvements queued by the harvest instead of
                                   // iteration stamps
};

// timed: the instantiation that stamps its phases into Args::tm
const void* parent_kernel_ptr(int problem, int gran, bool timed = false);
// nt: the child kernel's adjacency (and weight) loads are non-temporal (used
// with found bytes, Args::hint)
const void* child_kernel_ptr(int problem, bool timed = false, bool nt = false);
const void* serial_kernel_ptr(int problem, int gran, bool timed = false);
const void* harvest_kernel_ptr(int problem, bool timed = false);
const void* init_kernel_ptr(int problem);
const void* admit_kernel_ptr(int problem);
const void* admit_sources_kernel_ptr();
const void* clear_found_kernel_ptr();
const void* advance_kernel_ptr();

}  // namespace dpo
