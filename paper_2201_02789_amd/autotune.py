"""Tuning of threshold, coarsening and aggregation granularity for batched
traversals.

Sec. VIII-C of the paper reports that the best threshold is usually the one
that leaves about 6,000-8,000 child-grid launches, that performance is not
sensitive to the coarsening factor once it is large enough, that warp
granularity is never the best, and that a handful of runs finds a point close
to the best.  The tuner follows that in three stages:

1. per size bucket, threshold and coarsening: start from the threshold whose
   launch count (parents of degree >= T, summed over the bucket's queries) is
   closest to the 6,000-8,000 band, then take greedy steps through a small
   (T, CF) grid, timing the batch restricted to that bucket, until no
   neighbour is faster or after `max_runs` timed points;
2. aggregation granularity, for the whole launch: block, 4-block, 16-block
   and grid (wave is skipped, as the paper finds it never best), timing the
   whole batch with every bucket at its stage-1 point, then the other
   original child block sizes (64, 128, 256 lanes) at the fastest
   granularity;
3. a check on the whole batch: each bucket in turn goes back to the base
   (T, CF) and keeps it when the whole batch is faster that way (a bucket's
   best point timed alone need not be best beside the others, and stage-1
   differences can be within timing noise).

Granularity is a property of the launch, not of a bucket: the parent
workgroups' frontier entries mix queries of every bucket, and aggregation
groups are formed over those entries; so is the child block size, which fixes
the child kernel's slice arithmetic.  The result can be saved as JSON and
reloaded, so a tuned table is reused across runs.
"""
from __future__ import annotations

import json
import time
from dataclasses import asdict, replace

import numpy as np

from . import dpo

T_GRID = (0, 8, 32, 128, 512, 2048)
CF_GRID = (1, 2, 4, 8)
LAUNCH_BAND = (6000, 8000)


def heuristic_threshold(graphs, queries) -> int:
    """T in T_GRID whose launch count over the queries' graphs is nearest the band.

    Every reached vertex is a parent once per traversal; parents of degree
    >= T launch.  Reachability is not known before running, so all vertices of
    a query's graph are counted (an upper bound; the graphs are one component
    plus isolated vertices, which have degree 0 and never launch)."""
    target = sum(LAUNCH_BAND) / 2
    counts = {}
    for T in T_GRID:
        c = 0
        for g, _s in queries:
            d = graphs[g].degrees()
            c += int(np.count_nonzero(d >= max(T, 1)))
        counts[T] = c
    return min(T_GRID, key=lambda T: abs(np.log((counts[T] + 1) / target)))


CHILD_BLOCKS = (64, 128, 256)
GRANULARITIES = ((dpo.DPO_AGG_BLOCK, 4, "block"), (dpo.DPO_AGG_MULTIBLOCK, 4, "4-block"),
                 (dpo.DPO_AGG_MULTIBLOCK, 16, "16-block"), (dpo.DPO_AGG_GRID, 4, "grid"))


def _time_batch(kind, arena, queries, opts, reps=2):
    """Best of `reps` wall times of one batch call; `opts` is one Options (every
    query in bucket 0) or a per-bucket list."""
    import torch
    bopts = opts if isinstance(opts, (list, tuple)) else [opts]
    tot, _ = dpo.dpo_batch_slots(arena, queries)
    out = torch.empty(tot, dtype=torch.int32, device="cuda")
    ws = torch.empty(dpo.dpo_batch_workspace_bytes(arena, queries, bopts[0]), dtype=torch.uint8,
                     device="cuda")
    f = dpo.dpo_bfs_batch if kind == "bfs" else dpo.dpo_sssp_batch
    f(arena, queries, bopts, out, ws)  # warm-up (also instantiates the graph)
    torch.cuda.synchronize()
    best = float("inf")
    for _ in range(reps):
        t0 = time.perf_counter()
        f(arena, queries, bopts, out, ws)
        torch.cuda.synchronize()
        best = min(best, time.perf_counter() - t0)
    return best


def with_granularity(o: dpo.Options, agg: int, k: int) -> dpo.Options:
    return dpo.Options(**{**asdict(o), "agg": agg, "agg_blocks": k})


def tune_granularity(kind, arena, queries, bucket_opts, log=None, reps=3):
    """Stage 2: times the whole batch (queries with their buckets) at each
    granularity, every bucket keeping its threshold and coarsening.  Returns
    (per-bucket Options at the fastest granularity, [(label, seconds)])."""
    trace = []
    for agg, k, name in GRANULARITIES:
        cand = [with_granularity(o, agg, k) for o in bucket_opts]
        t = _time_batch(kind, arena, queries, cand, reps)
        trace.append((name, t, cand))
        if log:
            log(f"[tune] {kind} granularity {name}: {t * 1e3:.3f} ms")
    name, t, best = min(trace, key=lambda x: x[1])
    # the original child block size at that granularity (also per launch: it
    # fixes the child kernel's slice arithmetic)
    for cb in CHILD_BLOCKS:
        if cb == best[0].child_block:
            continue
        cand = [replace(o, child_block=cb) for o in best]
        tc = _time_batch(kind, arena, queries, cand, reps)
        trace.append((f"{name}-CB{cb}", tc, cand))
        if log:
            log(f"[tune] {kind} granularity {name}, child block {cb}: {tc * 1e3:.3f} ms")
    name, t, best = min(trace, key=lambda x: x[1])
    return best, [(n, v) for n, v, _ in trace]


def tune_bucket(kind, arena, graphs, queries, base: dpo.Options, max_runs: int = 10, log=None):
    """Returns (best Options, [(label, seconds)]) for one bucket's queries."""
    qs = [(g, s, 0) for g, s in queries]
    T0 = heuristic_threshold(graphs, queries)
    ti, ci = T_GRID.index(T0), CF_GRID.index(1)
    seen = {}

    def measure(i, j):
        if (i, j) not in seen:
            o = dpo.Options(**{**asdict(base), "threshold": T_GRID[i], "coarsen": CF_GRID[j]})
            seen[(i, j)] = _time_batch(kind, arena, qs, o)
            if log:
                log(f"[tune] {kind} bucket T={T_GRID[i]} CF={CF_GRID[j]}: {seen[(i, j)] * 1e3:.3f} ms")
        return seen[(i, j)]

    cur = measure(ti, ci)
    while len(seen) < max_runs:
        nbrs = [(ti + di, ci + dj) for di, dj in ((-1, 0), (1, 0), (0, -1), (0, 1))
                if 0 <= ti + di < len(T_GRID) and 0 <= ci + dj < len(CF_GRID)]
        nbrs = [p for p in nbrs if p not in seen][: max_runs - len(seen)]
        if not nbrs:
            break
        times = [(measure(*p), p) for p in nbrs]
        t, p = min(times)
        if t >= cur:
            break
        cur, (ti, ci) = t, p
    best = dpo.Options(**{**asdict(base), "threshold": T_GRID[ti], "coarsen": CF_GRID[ci]})
    trace = [(f"T{T_GRID[i]}-CF{CF_GRID[j]}", v) for (i, j), v in seen.items()]
    return best, trace


def tune(kind, arena, graphs, queries, bucket_of_graph, nbuckets, base: dpo.Options,
         max_runs: int = 10, log=None):
    """Tunes every bucket's threshold and coarsening (stage 1), then the
    launch's aggregation granularity (stage 2).  Returns the per-bucket Options
    list, the per-bucket (T, CF) traces and the granularity trace."""
    opts, traces = [], []
    for b in range(nbuckets):
        qb = [(g, s) for g, s in queries if bucket_of_graph[g] == b]
        if not qb:
            opts.append(base)
            traces.append([])
            continue
        o, tr = tune_bucket(kind, arena, graphs, qb, base, max_runs, log)
        opts.append(o)
        traces.append(tr)
    qs = [(g, s, bucket_of_graph[g]) for g, s in queries]
    opts, gtrace = tune_granularity(kind, arena, qs, opts, log)
    opts, ctrace = check_against_base(kind, arena, qs, opts, base, log)
    return opts, traces, gtrace + ctrace


def check_against_base(kind, arena, queries, bucket_opts, base: dpo.Options, log=None, reps=3):
    """Stage 3: per bucket, the whole batch with that bucket back at the base
    threshold and coarsening; kept when faster.  Returns (Options, trace)."""
    cur = list(bucket_opts)
    best = _time_batch(kind, arena, queries, cur, reps)
    trace = [("tuned", best)]
    for b, o in enumerate(cur):
        if (o.threshold, o.coarsen) == (base.threshold, base.coarsen):
            continue
        cand = list(cur)
        cand[b] = dpo.Options(**{**asdict(o), "threshold": base.threshold, "coarsen": base.coarsen})
        t = _time_batch(kind, arena, queries, cand, reps)
        trace.append((f"bucket{b}-base", t))
        if log:
            log(f"[tune] {kind} bucket {b} at the base point: {t * 1e3:.3f} ms (tuned {best * 1e3:.3f})")
        if t < best:
            cur, best = cand, t
    return cur, trace


def save(path, opts, meta=None):
    with open(path, "w") as f:
        json.dump({"buckets": [asdict(o) for o in opts], "meta": meta or {}}, f, indent=1)


def load(path):
    with open(path) as f:
        d = json.load(f)
    return [dpo.Options(**o) for o in d["buckets"]]
