// Shared declarations of the HIP library (device kernels and host driver).
#pragma once
#include <stddef.h>
#include <stdint.h>

namespace dpo {

constexpr int PB = 256;        // parent workgroup: 256 frontier entries per virtual block
constexpr int NW = PB / 64;    // wave64s per workgroup
constexpr int STAGE = 512;     // LDS slots per wave for next-frontier staging

enum { PROB_BFS = 0, PROB_SSSP = 1 };
enum { AGG_NONE = 0, AGG_WAVE = 1, AGG_BLOCK = 2, AGG_MULTI = 3, AGG_FLAT = 4 };
// device error codes (stored as the negated dpo_status)
enum { ERR_ARG = 1, ERR_CAPACITY = 4, ERR_TIMEOUT = 5 };

// Counters of one level step; three sets rotate by level % 3 so that step L
// can clear the set of step L + 1 while nobody uses it.
struct Ctr {
  uint32_t parent_claim;         // next virtual parent block
  uint32_t child_ticket;         // next global child-block ticket
  uint32_t groups_finished;      // aggregation groups whose parents all finished
  uint32_t exit_count;           // workgroups that left the step
  unsigned long long desc_ctr;   // hi32: descriptors reserved, lo32: child blocks reserved
  uint32_t pad[2];
};

struct State {
  uint32_t level;       // index of the next level step
  uint32_t done;        // set when a step leaves an empty next frontier
  uint32_t error;       // first device error code, 0 = none
  uint32_t levels_run;  // non-empty steps run
  uint32_t fcount[4];   // frontier sizes by level % 3
  Ctr ctr[3];
  unsigned long long stats[8];
};

// Kernel arguments (by value).  All pointers are device pointers.
struct Args {
  const int32_t* rp;
  const int32_t* col;
  const uint32_t* w;
  int32_t* level;
  uint32_t* dist;
  State* st;
  unsigned long long* grp_packed;  // [3][ngroups_cap]
  uint32_t* grp_done;              // [3][ngroups_cap]
  int32_t* front0;
  int32_t* front1;
  uint32_t* visit;                 // BFS bitmap words / SSSP stamps
  int4* rec;                       // launch records {row start, deg, offset, parent value}
  unsigned long long* desc_a;      // (nrec << 32) | record base
  unsigned long long* desc_b;      // (level + 1) << 32 | child-block base
  int32_t n;
  int32_t m;
  int32_t T;
  int32_t CB;
  int32_t k;
  int32_t ngroups_cap;
  int32_t desc_cap;
  int32_t count_stats;
  uint64_t watchdog_ticks;         // s_memrealtime ticks (100 MHz) a wait may last
};

const void* step_kernel_ptr(int problem, int gran, int cf);
const void* init_kernel_ptr(int problem);

}  // namespace dpo
