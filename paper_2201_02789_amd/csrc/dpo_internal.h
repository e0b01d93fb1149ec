// Shared declarations of the HIP library (device kernels and host driver).
#pragma once
#include <stddef.h>
#include <stdint.h>

namespace dpo {

constexpr int PB = 256;        // parent workgroup: 256 frontier entries per virtual block
constexpr int NW = PB / 64;    // wave64s per workgroup
constexpr int STAGE = 512;     // LDS slots per wave for next-frontier staging
constexpr int NQD = 8;         // descriptor queues (one per XCD: queue = virtual block % 8)
constexpr int NQF = 64;        // frontier queues (queue = workgroup % 64), plus one overflow
constexpr int MAX_GRID = 4096; // persistent grid cap (rows of the per-workgroup counters)
constexpr int NSTAT = 8;

enum { PROB_BFS = 0, PROB_SSSP = 1 };
enum { AGG_NONE = 0, AGG_WAVE = 1, AGG_BLOCK = 2, AGG_MULTI = 3, AGG_FLAT = 4 };
// device error codes (stored as the negated dpo_status)
enum { ERR_ARG = 1, ERR_CAPACITY = 4, ERR_TIMEOUT = 5 };
enum { S_FRONT = 0, S_SERIAL, S_REC, S_CHILD, S_ESER, S_ECHILD, S_DESC };

// Counters of one level; three sets rotate by level % 3 so that the parent
// kernel of level L can clear the set of level L + 1 while nobody uses it.
struct LevelSet {
  uint32_t fcnt[NQF + 1];              // next-frontier queue fills (+ overflow)
  uint32_t pad0[15];
  unsigned long long qctr[NQD];        // descriptor queues: hi32 count, lo32 child blocks
};

struct State {
  uint32_t base;        // level index of step 0 of the current graph replay
  uint32_t done;        // set when a level starts with an empty frontier
  uint32_t error;       // first device error code, 0 = none
  uint32_t levels_run;  // non-empty levels
  uint32_t pad[60];
  LevelSet set[3];
};

// Kernel arguments (by value).  All pointers are device pointers.
struct Args {
  const int32_t* rp;
  const int32_t* col;
  const uint32_t* w;
  int32_t* level;
  uint32_t* dist;
  State* st;
  unsigned long long* grp_packed;  // [3][ngroups_cap]: hi32 records, lo32 child blocks
  uint32_t* grp_done;              // [3][ngroups_cap]: blocks of the group finished
  int32_t* front0;                 // [NQF * fcap + n]
  int32_t* front1;
  uint32_t* visit;                 // BFS bitmap words / SSSP stamps
  int4* rec;                       // [n] launch records {row start, deg, offset, parent value}
  int4* desc;                      // [NQD][desc_cap] {record base, records, block base, -}
  unsigned long long* stats;       // [MAX_GRID][NSTAT], one row per workgroup
  int32_t n;
  int32_t m;
  int32_t T;
  int32_t CB;
  int32_t CF;
  int32_t k;
  int32_t ngroups_cap;
  int32_t desc_cap;                // per descriptor queue
  int32_t fcap;                    // per frontier queue
  int32_t count_stats;
};

const void* parent_kernel_ptr(int problem, int gran);
const void* child_kernel_ptr(int problem, int cf);
const void* init_kernel_ptr(int problem);
const void* advance_kernel_ptr();

}  // namespace dpo
