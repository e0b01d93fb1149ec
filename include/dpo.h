/*
 * dpo — nested-parallel BFS and SSSP on MI355X (gfx950) with thresholding,
 * coarsening and multi-block-granularity aggregation.
 *
 * Method: "A Compiler Framework for Optimizing Dynamic Parallelism on GPUs"
 * (arXiv 2201.02789).  A parent thread per frontier vertex owns the child
 * work of its neighbours (Sec. II-A).  The three transformations of the paper
 * are applied by hand in the kernels:
 *   thresholding (Sec. III-B): a parent whose child-thread count (its degree,
 *     Sec. III-D) is below T runs the child work serially itself;
 *   coarsening (Sec. IV-B): one child block runs CF original child blocks;
 *   aggregation (Sec. II-B, V-A): the child grids of a wave, a block or a
 *     group of k blocks are fused into one grid whose blocks find their parent
 *     by a binary search of the scanned grid sizes.
 * HIP has no device-side grid launch, so a "launch" is a device-resident
 * launch record plus a published descriptor; the aggregated child grids of a
 * level run in the child kernel that follows the level's parent kernel on the
 * same stream.
 *
 * Conventions for every call below
 *   - Graph arrays, outputs and the workspace are DEVICE pointers owned by the
 *     caller; the library never allocates device memory at run time (its one
 *     static device array serves dpo_bfs_noalloc) and never frees the caller's
 *     memory.  `stream` is a hipStream_t (NULL = default stream).
 *   - The CSR graph must be symmetric for the results to be shortest paths of
 *     an undirected graph; the kernels follow out-edges only.
 *   - Work is enqueued on `stream`.  The traversal calls synchronise `stream`
 *     once per `steps_per_replay` level steps to read the done flag, so they
 *     return only when the traversal has finished and outputs are final.
 *   - Errors are return codes, never exceptions.  Argument errors are found on
 *     the host before anything is enqueued.  Device-detected errors (queue
 *     capacity, a vertex id out of range) are read back at the end of the
 *     call.
 *   - Not thread-safe for concurrent calls that share a workspace.
 */
#ifndef DPO_H
#define DPO_H

#include <stddef.h>
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

typedef enum {
  DPO_OK = 0,
  DPO_ERR_ARG = -1,         /* null pointer, bad size or bad option             */
  DPO_ERR_SOURCE = -2,      /* source outside [0, n)                             */
  DPO_ERR_WORKSPACE = -3,   /* ws_bytes < dpo_workspace_bytes(...)               */
  DPO_ERR_CAPACITY = -4,    /* a device queue would have overflowed              */
  DPO_ERR_TIMEOUT = -5,     /* more level steps than the traversal can need      */
  DPO_ERR_HIP = -6,         /* a HIP runtime call failed                         */
  DPO_ERR_UNSUPPORTED = -7  /* option combination not built into the library    */
} dpo_status;

typedef enum {
  DPO_MODE_NESTED = 0, /* parent thread per frontier vertex + child work (T/C/A)   */
  DPO_MODE_FLAT = 1    /* no nesting: each parent walks its neighbours serially
                          (the paper's "No CDP" version, Sec. VII)              */
} dpo_mode;

typedef enum {
  DPO_AGG_NONE = 0,       /* every launching parent publishes its own child grid
                             (the paper's "CDP" version when T = 0, CF = 1)     */
  DPO_AGG_WAVE = 1,       /* aggregation over the 64 parents of a wave
                             (the paper's warp granularity, Sec. II-B)          */
  DPO_AGG_BLOCK = 2,      /* over the 256 parents of a workgroup (Sec. II-B)    */
  DPO_AGG_MULTIBLOCK = 3, /* over groups of agg_blocks workgroups (Sec. V-A)    */
  DPO_AGG_GRID = 4        /* over the whole parent grid of a level (Sec. II-B):
                             one aggregated grid per level                      */
} dpo_agg;

typedef struct {
  int32_t mode;             /* dpo_mode                                             */
  int32_t threshold;        /* T >= 0.  A parent of degree d, 0 < d < T, runs its
                               children serially; d >= max(T, 1) launches
                               (Sec. III-B).  T = 0 disables thresholding.         */
  int32_t coarsen;          /* CF in {1, 2, 4, 8, 16}: one child block runs CF
                               original child blocks (Sec. IV-B).                 */
  int32_t agg;              /* dpo_agg (Sec. II-B, V-A)                             */
  int32_t agg_blocks;       /* k >= 2 for DPO_AGG_MULTIBLOCK (e.g. 4 or 16)         */
  int32_t child_block;      /* original child block size bDim in {64, 128, 256}    */
  int32_t steps_per_replay; /* level steps per HIP-graph replay; 0 = 16            */
  int32_t agg_threshold;    /* aggregation threshold (Sec. V-B), wave and block
                               granularity only: when fewer than this many parents
                               of the wave / block launch, each launches its own
                               grid instead of joining an aggregated one; 0 = off */
  int32_t split_min;        /* >= 0.  A level whose frontier has at least this
                               many entries probes one copy of the visited state
                               and sends its atomics to a second copy; narrower
                               levels use one copy.  Affects speed only.  Default
                               65536; 0 = always two copies.  BFS with
                               claim_hint: the levels that use the per-XCD
                               copies.                                          */
  int32_t serial_wave;      /* 1 (default): the thresholded children of a wave's
                               parents run together, their edges 64 at a time
                               (no launch, as Sec. III-B asks, but every lane
                               busy); 0: each runs sequentially in its parent's
                               lane, the paper's literal form.  The flat mode
                               always uses the literal form.  Speed only.        */
  int32_t dyn_share;        /* 0..100, default 0.  How the child kernel's waves
                               share a level's aggregated child blocks.  0: each
                               wave runs an even share.  Otherwise each XCD's
                               workgroups (workgroup % 8) take that XCD's eighth
                               of the blocks, each wave an even share of
                               (100 - dyn_share)% of it, and then claim chunks of
                               the rest from a counter of their XCD until none is
                               left (as a hardware block scheduler hands out
                               blocks), so waves whose blocks run slow do fewer.
                               Speed only.                                      */
  int32_t claim_hint;       /* dpo_claim_hint, default DPO_HINT_AUTO.  Found bytes
                               and a harvest kernel after the level.  BFS levels
                               with at least split_min frontier entries: each
                               XCD (workgroup % 8) probes a visited bitmap of its
                               own, kept with plain loads and stores, and a lane
                               records a new vertex there and as a found byte,
                               with no atomic; the harvest gives every found
                               vertex not visited before it its level and a
                               place in the next frontier.  When off, such a
                               level probes a frozen copy while claiming with
                               atomics in a second one.  Narrower levels probe
                               and claim one bitmap.  SSSP, every level: a lane
                               whose atomicMin improved a distance records the
                               vertex as found, and the harvest queues it once;
                               when off, an iteration stamp exchanged
                               atomically does.  Speed only.                    */
} dpo_options;

typedef enum {
  DPO_HINT_AUTO = 0,  /* on for single traversals (dpo_bfs, dpo_sssp and
                         their variants) and the serving engines when the graph
                         (the arena for an engine) has at least 8 directed
                         entries per vertex; off for the batch calls and
                         sparser graphs, where many narrow levels would each
                         pay the extra kernel launch                           */
  DPO_HINT_ON = 1,
  DPO_HINT_OFF = 2
} dpo_claim_hint;

typedef struct {
  int32_t n;                /* vertices, >= 1                                      */
  int32_t m;                /* directed CSR entries, >= 0                          */
  const int32_t* row_ptr;   /* device, int32[n + 1], row_ptr[0] = 0, row_ptr[n] = m */
  const int32_t* col_idx;   /* device, int32[m], each in [0, n)                     */
  const uint32_t* weights;  /* device, uint32[m] (SSSP only; NULL for BFS)          */
} dpo_csr;

/* Per-traversal counters (host struct).  Requesting them makes the kernels
 * count and adds one synchronising read at the end of the call. */
typedef struct {
  int32_t levels;           /* level steps with a non-empty frontier               */
  int32_t reserved;
  int64_t frontier_total;   /* parent threads run (sum of frontier sizes)          */
  int64_t serial_parents;   /* parents that ran their children serially (T)        */
  int64_t records;          /* parents that launched (launch records written)      */
  int64_t child_blocks;     /* coarsened child blocks started                      */
  int64_t edges_serial;     /* neighbour visits done inside parents                */
  int64_t edges_child;      /* neighbour visits done by child blocks; SSSP counts
                               neither kind for a parent whose distance dropped
                               again in its level (its work is dropped)         */
  int64_t descriptors;      /* aggregated grids published ("launches")             */
} dpo_stats;

/* Fills *o with the defaults: nested, T = 128, CF = 8, 4-block aggregation,
 * child block 256, 16 steps per replay, no aggregation threshold, two visited
 * copies from 65,536 frontier entries, wave-run thresholded children, even
 * child shares, claim_hint automatic. */
void dpo_default_options(dpo_options* o);

/* Device workspace bytes needed by dpo_bfs / dpo_sssp on a graph with g->n
 * vertices under options o (the same buffer serves both); about 72 bytes per
 * vertex for large graphs.  0 on bad args.
 * Layout, all inside the caller's buffer: traversal state and counters, two
 * frontier buffers (64 sharded queues plus an overflow queue), a per-vertex
 * visit word (for BFS two visited bitmaps, one per XCD and a found byte per
 * vertex, for SSSP iteration stamps or found bytes), a second distance array
 * (SSSP), launch records of 24 bytes per
 * vertex, a list
 * of thresholded parents of 16 bytes per vertex, 8 descriptor queues of 16
 * bytes per possible aggregated grid and per-workgroup counters. */
size_t dpo_workspace_bytes(const dpo_csr* g, const dpo_options* o);

/* Breadth-first search (Table I, BFS) from `source`.
 * levels: device int32[g->n]; on return levels[v] = hop distance from the
 * source, -1 if unreachable.  Bit-identical for every option combination.
 * ws: device buffer of at least dpo_workspace_bytes(g, o) bytes, contents on
 * entry irrelevant.  st: optional host pointer (NULL = no counters). */
dpo_status dpo_bfs(const dpo_csr* g, int32_t source, const dpo_options* o, int32_t* levels,
                   void* ws, size_t ws_bytes, void* stream, dpo_stats* st);

/* Single-source shortest paths (Table I, SSSP) by frontier Bellman-Ford with
 * atomicMin relaxations.  g->weights required, any uint32 values (0 allowed).
 * Path sums saturate at 0xFFFFFFFF instead of wrapping.
 * dist: device uint32[g->n]; on return the exact shortest distances,
 * 0xFFFFFFFF if unreachable (and for a vertex whose shortest distance is
 * 0xFFFFFFFF or more).  Other arguments as for dpo_bfs. */
dpo_status dpo_sssp(const dpo_csr* g, int32_t source, const dpo_options* o, uint32_t* dist,
                    void* ws, size_t ws_bytes, void* stream, dpo_stats* st);

/* ------------------------------------------------------------ no allocation
 * For callers that cannot allocate device memory: code that must not call
 * hipMalloc (tight serving loops, harnesses that forbid it) or that cannot
 * hand the library a workspace.  dpo_bfs_noalloc is dpo_bfs with its
 * workspace taken from a static device array of DPO_NOALLOC_SCRATCH_BYTES
 * that the library holds on every GPU it runs on until the process ends.  The
 * call allocates nothing (no hipMalloc, hipFree, pinned host memory or HIP
 * graph instantiation: its level steps are plain kernel launches).
 *   - Graphs whose dpo_workspace_bytes(g, o) exceed DPO_NOALLOC_SCRATCH_BYTES
 *     are rejected with DPO_ERR_WORKSPACE before anything is enqueued (up to
 *     about 925,000 vertices at the default options, 757,000 with
 *     DPO_AGG_NONE; the size grows with n only).
 *   - Every call on one GPU shares that GPU's array, which keeps the last
 *     call's contents; each call clears what it reads before reading it.
 *     Calls that overlap in time on one GPU (other threads, other streams)
 *     race on the array and give undefined results: serialise them.
 *   - Same arguments, results and errors as dpo_bfs otherwise; no counters. */
#define DPO_NOALLOC_SCRATCH_BYTES (64u << 20)

dpo_status dpo_bfs_noalloc(const dpo_csr* g, int32_t source, const dpo_options* o, int32_t* levels,
                           void* stream);

/* ------------------------------------------------------------ phase timing
 * Execution-time breakdown of one traversal (Sec. VIII-B splits time into
 * parent work, aggregation, launch, disaggregation and child work).  Runs
 * dpo_bfs (kind 0) or dpo_sssp (kind 1) with timed instantiations of the
 * level kernels, with the same results, on the product kernels' grids (a
 * timed kernel that needs more registers, and so fits fewer workgroups per
 * compute unit, runs on the grid resident at its own occupancy).
 * Each wave stamps a shader-clock counter at phase boundaries, after waiting
 * for its own outstanding memory operations (so the timed traversal is
 * slower than the product one), and each workgroup of each level kernel
 * writes one row of 8 uint64 words to `timing` (device, caller-owned, at
 * least DPO_TIMING_BYTES, zeroed by the call) at index
 *   ((level * 4 + kernel) * 4096 + workgroup) * 8,
 * kernel 0 = parent kernel, 1 = child kernel, 2 = SSSP's thresholded-children
 * kernel, 3 = the harvest kernel (found bytes, claim_hint); words: [0] a constant-rate (100 MHz) clock at the workgroup's entry,
 * [1] at its exit, [2..6] the cycles its waves spent in parent work,
 * aggregation, launch (publishing a grid; reading the level's published
 * grids), disaggregation (finding records, loading record windows) and child
 * work, summed over its waves, [7] the largest total of one wave.  A row of
 * zeros: the workgroup did not run (or the level index is 64 or more).
 * Counters are not collected.  Otherwise as dpo_bfs / dpo_sssp;
 * DPO_ERR_ARG if kind, timing or timing_bytes are invalid. */
#define DPO_TIMING_BYTES (64u * 4u * 4096u * 8u * 8u)

dpo_status dpo_traverse_timed(int32_t kind, const dpo_csr* g, int32_t source, const dpo_options* o,
                              void* out, void* ws, size_t ws_bytes, void* stream, void* timing,
                              size_t timing_bytes);

/* ------------------------------------------------------------------ batches
 * Many traversals in one launch sequence (the parent and child kernels of a
 * level serve every traversal of the batch; frontier entries carry their
 * traversal).  Graphs are packed in one CSR arena: graph g owns the arena
 * vertices [graph_vbase[g], graph_vbase[g + 1]), its rows list arena vertex
 * ids, and no edge leaves a graph. */
typedef struct {
  int32_t ngraphs;             /* >= 1                                              */
  const int32_t* graph_vbase;  /* HOST int32[ngraphs + 1], graph_vbase[0] = 0,
                                  graph_vbase[ngraphs] = csr.n, strictly increasing  */
  dpo_csr csr;                 /* the arena (device arrays, as for dpo_bfs)          */
} dpo_arena;

typedef struct {
  int32_t graph;   /* graph index in the arena                                  */
  int32_t source;  /* vertex id local to that graph                             */
  int32_t bucket;  /* options entry whose threshold and coarsen this query uses */
} dpo_query;

/* Output layout of a batch: query i writes its graph's n_g results at
 * [slot0[i], slot0[i] + n_g), slot0[i] = sum over j < i of round_up(n_g(j), 32).
 * Returns the total number of slots (the output length) and, if slot0 is not
 * NULL, fills the HOST array slot0[nq + 1].  -1 on bad arguments. */
int64_t dpo_batch_slots(const dpo_arena* arena, const dpo_query* queries, int32_t nq,
                        int64_t* slot0);

/* Device workspace bytes for dpo_bfs_batch / dpo_sssp_batch (0 on bad args). */
size_t dpo_batch_workspace_bytes(const dpo_arena* arena, const dpo_query* queries, int32_t nq,
                                 const dpo_options* o);

/* nq (<= 4096) traversals at once.  bucket_opts[b] supplies threshold and
 * coarsen for the queries of bucket b (per-size-bucket tuning); mode, agg,
 * agg_blocks, child_block and steps_per_replay come from bucket_opts[0].
 * levels / dist: device arrays of dpo_batch_slots(...) entries, laid out as
 * above; every query's results are bit-identical to a single dpo_bfs /
 * dpo_sssp call on its graph.  Returns when all queries have finished. */
dpo_status dpo_bfs_batch(const dpo_arena* arena, const dpo_query* queries, int32_t nq,
                         const dpo_options* bucket_opts, int32_t nbuckets, int32_t* levels,
                         void* ws, size_t ws_bytes, void* stream, dpo_stats* st);
dpo_status dpo_sssp_batch(const dpo_arena* arena, const dpo_query* queries, int32_t nq,
                          const dpo_options* bucket_opts, int32_t nbuckets, uint32_t* dist,
                          void* ws, size_t ws_bytes, void* stream, dpo_stats* st);

/* ------------------------------------------------------------------ serving
 * Continuous batching over resident graphs.  Queries are submitted at any
 * time; each dpo_engine_step() waits for the replay in flight (if any),
 * retires the queries that finished (their results are copied to the
 * caller's `out` before their tickets are reported), admits waiting queries
 * in arrival order while a query-table entry and round_up(n_g, 32) free output
 * slots are available (admission by footprint: a query that does not fit
 * waits, and so do the ones behind it), and launches the next replay of
 * steps_per_replay level steps without waiting for it.  Admitted queries join
 * the running ones at the next level step; every result is bit-identical to a
 * single dpo_bfs / dpo_sssp call.  One engine serves one kind (BFS or SSSP);
 * engines on different streams overlap on the device. */
typedef struct dpo_engine dpo_engine;

/* Device workspace bytes for an engine (0 on bad args). */
size_t dpo_engine_workspace_bytes(const dpo_options* o, int32_t max_queries, int64_t max_slots);

/* kind: 0 = BFS, 1 = SSSP.  bucket_opts / nbuckets as for the batch calls;
 * graph_bucket: HOST int32[arena->ngraphs] bucket of each graph (NULL = 0).
 * max_queries <= 4096 running at once; max_slots: output slots shared by the
 * running queries (the footprint pool).  ws: device, dpo_engine_workspace_bytes;
 * out_arena: device int32/uint32[round_up(max_slots, 32)] engine-owned
 * scratch for running queries' outputs.  The arena, ws and out_arena must
 * outlive the engine; ws may hold anything (the call initialises what the
 * kernels read before any admission, on `stream`, and waits for it).  The
 * engine keeps a copy of graph_vbase. */
dpo_status dpo_engine_create(const dpo_arena* arena, int32_t kind, const dpo_options* bucket_opts,
                             int32_t nbuckets, const int32_t* graph_bucket, int32_t max_queries,
                             int64_t max_slots, void* ws, size_t ws_bytes, void* out_arena,
                             void* stream, dpo_engine** engine);

/* Queue a query: `out` is a device array of n_g entries written before the
 * ticket is reported by dpo_engine_poll.  DPO_ERR_CAPACITY if the graph can
 * never fit in max_slots. */
dpo_status dpo_engine_submit(dpo_engine* e, int32_t graph, int32_t source, void* out,
                             uint64_t* ticket);

/* One scheduling step (see above); running / pending: optional host outputs. */
dpo_status dpo_engine_step(dpo_engine* e, int32_t* running, int32_t* pending);

/* Moves up to cap completed tickets into tickets[]; returns how many. */
int32_t dpo_engine_poll(dpo_engine* e, uint64_t* tickets, int32_t cap);

/* Waits for the replay in flight and releases the engine's host resources. */
void dpo_engine_destroy(dpo_engine* e);

/* Static string for a dpo_status value. */
const char* dpo_strerror(int32_t status);

#ifdef __cplusplus
}
#endif

#endif /* DPO_H */
