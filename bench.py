#!/usr/bin/env python3
"""Benchmark: GTEPS of nested-parallel BFS on R-MAT scale 22 (edgefactor 16,
16 sources) with thresholding + coarsening + aggregation, beside the flat
(no nesting) and naive (one child grid per parent) kernels on the same GPU,
the HBM roofline of the level-step kernel, and the CPU oracle on host cores.

A step is one pass of the whole hot path over the batch: one BFS from each of
the 16 sources.  Prints ONE JSON line.

  python bench.py [--steps K] [--warmup W] [--workload bfs22|sssp21|batch|serve]
                  [--sweep] [--no-cpu] [--no-baselines] [--no-extras]

The default run prints the s22 BFS line with two extra objects: "batched"
(512 BFS over 64 R-MAT graphs of scales 10..18 in one launch sequence,
per-bucket tuned) and "serving" (Poisson BFS/SSSP stream against 8 resident
graphs, p50/p99 latency per offered rate).
"""
import argparse
import json
import os
import sys
import time

import numpy as np

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

HBM_PEAK_GBS = 8000.0  # MI355X HBM3E


def parse():
    p = argparse.ArgumentParser()
    p.add_argument("--gpus", type=int, default=1)
    p.add_argument("--steps", type=int, default=5)
    p.add_argument("--warmup", type=int, default=2)
    p.add_argument("--workload", default="bfs22",
                   choices=["bfs22", "bfs25", "er22", "sssp21", "bfs12", "batch", "serve", "road"])
    p.add_argument("--no-extras", action="store_true", help="skip the batched and serving legs")
    p.add_argument("--serve-seconds", type=float, default=10.0,
                   help="arrivals per offered rate (capped at 25,000 queries)")
    p.add_argument("--cpu-serve-queries", type=int, default=600,
                   help="arrivals of the lowest-rate trace that the oracle pool serves")
    p.add_argument("--rates", default="1000,2000,5000,10000,20000,50000")
    p.add_argument("--threshold", type=int, default=None)
    p.add_argument("--coarsen", type=int, default=None)
    p.add_argument("--split-min", type=int, default=None,
                   help="frontier size from which a level uses two visited copies")
    p.add_argument("--agg", default=None, help="none|wave|block|<k>-block")
    p.add_argument("--serial-wave", type=int, default=None, choices=[0, 1])
    p.add_argument("--child-block", type=int, default=None, choices=[64, 128, 256])
    p.add_argument("--dyn-share", type=int, default=None,
                   help="percent of the child blocks claimed in chunks (0 = even split)")
    p.add_argument("--claim-hint", type=int, default=None, choices=[0, 1, 2],
                   help="BFS per-XCD visited copies: 0 auto, 1 on, 2 off (also for the serving engines)")
    p.add_argument("--breakdown", action="store_true",
                   help="execution-time breakdown (Sec. VIII-B) of bfs22 or sssp21 at CF 1..8")
    p.add_argument("--sweep", action="store_true",
                   help="threshold x coarsening x granularity sweep of the workload instead")
    p.add_argument("--no-cpu", action="store_true")
    p.add_argument("--no-baselines", action="store_true")
    p.add_argument("--cpu-seconds", type=float, default=10.0,
                   help="minimum oracle time of the cpu_baseline sample")
    p.add_argument("--calibrate-primitives", action="store_true",
                   help="only run the memory-primitive microbenchmarks and write "
                        "profiles/primitives.md")
    p.add_argument("--calibrate-copy", action="store_true",
                   help="only run a plain 512 MiB device copy (counter calibration)")
    p.add_argument("--simulate-bands", action="store_true",
                   help="host simulation of a near-far band split of the s21 SSSP levels; "
                        "writes profiles/sssp21_bands.md (no GPU)")
    p.add_argument("--summarize-counters", metavar="DIR", default=None,
                   help="write profiles/<workload>_counters.md from the counter passes under DIR")
    p.add_argument("--summarize-profiles", metavar="DIR", default=None,
                   help="write profiles/<workload>_kernels.md and _traffic.json from the "
                        "rocprofv3 CSV output under DIR (trace/, fetch/, write/, "
                        "copy_fetch/, copy_write/; trace/out.json = the traced bench line)")
    return p.parse_args()


def log(*a):
    print(*a, file=sys.stderr, flush=True)


def agg_of(s):
    from paper_2201_02789_amd import dpo
    if s is None:
        return None
    if s == "none":
        return (dpo.DPO_AGG_NONE, 4)
    if s == "wave":
        return (dpo.DPO_AGG_WAVE, 4)
    if s == "block":
        return (dpo.DPO_AGG_BLOCK, 4)
    return (dpo.DPO_AGG_MULTIBLOCK, int(s.split("-")[0]))


# Best point of each workload's sweep (threshold x coarsening x granularity,
# and the one-copy threshold for SSSP) on MI355X; overridable from the command
# line.  The original child block size (the untransformed program's child
# blockDim, which the naive baseline shares) is 128 lanes on the large
# workloads: the child kernel splits a level's blocks evenly over its waves,
# and smaller blocks make equal block counts closer to equal edge counts.
TUNED = {"bfs22": dict(threshold=64, coarsen=1, agg=3, agg_blocks=4, child_block=128, dyn_share=25,
                       split_min=4096),
         # above the maximum degree (62): nothing launches, the waves run every
         # child together; wave granularity keeps pass 1 free of block barriers
         "er22": dict(threshold=128, coarsen=1, agg=1, child_block=128, split_min=4096),
         "bfs25": dict(threshold=64, coarsen=1, agg=3, agg_blocks=4, child_block=128),
         "bfs12": dict(threshold=32, coarsen=8, agg=3, agg_blocks=4),
         "sssp21": dict(threshold=512, coarsen=1, agg=3, agg_blocks=4, split_min=262144,
                        child_block=128, dyn_share=50)}


SERVE_T = {"bfs": 64, "sssp": 512}  # thresholds of the serving engines
SERVE_DYN = {"bfs": 0, "sssp": 50}  # percent of child blocks claimed in chunks
SERVE_CB = {"bfs": 128, "sssp": 128}  # original child block sizes of the serving engines


class Workload:
    def __init__(self, name):
        from paper_2201_02789_amd import graphgen as gg
        self.name = name
        t0 = time.time()
        if name == "bfs22":
            self.g = gg.rmat(22, 16, 22, perm_seed=24)
            self.sources = gg.sample_sources(self.g, 16, 1)
            self.kind = "bfs"
            self.desc = "BFS, R-MAT scale 22, edgefactor 16, a/b/c/d .57/.19/.19/.05, permuted, 16 sources"
        elif name == "bfs25":
            # the largest R-MAT whose directed entry count fits int32 CSR indices
            self.g = gg.rmat(25, 16, 25, perm_seed=26)
            self.sources = gg.sample_sources(self.g, 4, 1)
            self.kind = "bfs"
            self.desc = "BFS, R-MAT scale 25, edgefactor 16, permuted, 4 sources"
        elif name == "er22":
            # Erdos-Renyi control: same n and the same number of undirected edges as
            # the s22 R-MAT graph, Poisson degrees instead of a power law
            r = gg.rmat(22, 16, 22, perm_seed=24)
            self.g = gg.erdos_renyi(r.n, r.m // 2, 23)
            del r
            self.sources = gg.sample_sources(self.g, 16, 1)
            self.kind = "bfs"
            self.desc = ("BFS, Erdos-Renyi G(n, M) with the s22 R-MAT graph's n and undirected "
                         "edge count, 16 sources")
        elif name == "bfs12":
            self.g = gg.rmat(12, 16, 1)
            self.sources = np.array([0], dtype=np.int32)
            self.kind = "bfs"
            self.desc = "BFS, R-MAT scale 12, edgefactor 16, unpermuted, source 0"
        else:
            self.g = gg.add_weights(gg.rmat(21, 16, 21, perm_seed=24), 31)
            self.sources = np.array([gg.max_degree_vertex(self.g)], dtype=np.int32)
            self.kind = "sssp"
            self.desc = "SSSP, R-MAT scale 21, edgefactor 16, weights U[1,255], max-degree source"
        log(f"[bench] graph {name}: n={self.g.n} m={self.g.m} ({time.time() - t0:.1f}s)")


def run_one(dpo, dg, kind, src, opts, out, ws):
    if kind == "bfs":
        return dpo.dpo_bfs(dg, int(src), opts, out, ws)
    return dpo.dpo_sssp(dg, int(src), opts, out, ws)


def measure(dpo, torch, wl, dg, opts, steps, warmup, sources=None):
    """Times `steps` passes over the sources; returns per-call event times (ms)."""
    sources = wl.sources if sources is None else sources
    out = torch.empty(dg.n, dtype=torch.int32, device="cuda")
    ws = dpo.alloc_workspace(dg, opts)
    stream = torch.cuda.current_stream()
    for _ in range(warmup):
        for s in sources:
            run_one(dpo, dg, wl.kind, s, opts, out, ws)
    torch.cuda.synchronize()
    ev = [(torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True))
          for _ in range(steps * len(sources))]
    t0 = time.perf_counter()
    i = 0
    for _ in range(steps):
        for s in sources:
            ev[i][0].record(stream)
            run_one(dpo, dg, wl.kind, s, opts, out, ws)
            ev[i][1].record(stream)
            i += 1
    torch.cuda.synchronize()
    wall = time.perf_counter() - t0
    per_call = np.array([a.elapsed_time(b) for a, b in ev]).reshape(steps, len(sources))
    return per_call, wall


class Certifier:
    """Edge certificates of a traversal result, computed with torch's own
    gather / scatter kernels on the device (independent of the HIP path, no
    oracle): BFS (i) level[s] = 0, (ii) every reached v != s has an
    in-neighbour one level lower, (iii) every edge from a reached u reaches v
    with level[v] <= level[u] + 1; SSSP the same with dist and w (>= 1).
    Together they fix levels / distances exactly."""

    def __init__(self, torch, dg):
        self.torch = torch
        deg = (dg.row_ptr[1:] - dg.row_ptr[:-1]).to(torch.int64)
        self.u = torch.repeat_interleave(torch.arange(dg.n, device=deg.device), deg)
        self.v = dg.col_idx.to(torch.int64)
        self.w = None if dg.weights is None else dg.weights.to(torch.int64) & 0xFFFFFFFF
        self.n = dg.n

    def __call__(self, kind, src, out):
        torch = self.torch
        if kind == "bfs":
            x = out.to(torch.int64)
            unreached, step = -1, 1
        else:
            x = out.to(torch.int64) & 0xFFFFFFFF
            unreached, step = 0xFFFFFFFF, self.w
        if int(x[src]) != 0:
            return False
        xu, xv = x[self.u], x[self.v]
        ru = xu != unreached
        bound = xu + step
        if bool(torch.any(ru & ((xv == unreached) | (xv > bound)))):
            return False
        tight = torch.zeros(self.n, dtype=torch.bool, device=x.device)
        tight[self.v[ru & (xv == bound)]] = True
        need = x != unreached
        need[src] = False
        return bool(torch.all(tight[need]))


def reached_stats(dpo, torch, wl, dg, opts):
    """(m_r, n_r, stats) per source from one untimed run with counters, and
    how many sources' results pass their edge certificates."""
    out = torch.empty(dg.n, dtype=torch.int32, device="cuda")
    ws = dpo.alloc_workspace(dg, opts)
    deg = torch.diff(dg.row_ptr).to(torch.int64)
    cert = Certifier(torch, dg)
    res, passed = [], 0
    for s in wl.sources:
        if wl.kind == "bfs":
            st = dpo.dpo_bfs(dg, int(s), opts, out, ws, stats=True)
            reached = out >= 0
        else:
            st = dpo.dpo_sssp(dg, int(s), opts, out, ws, stats=True)
            reached = out != -1  # 0xFFFFFFFF as int32
        passed += int(cert(wl.kind, int(s), out))
        res.append((int(deg[reached].sum()), int(reached.sum()), st))
    del cert
    return res, passed


# the kernels of a level step (SSSP runs parent_kernel twice; single
# traversals add the harvest)
LEVEL_KERNELS = ("parent_kernel", "child_kernel", "harvest_kernel")
KERNEL_SOURCES = ["paper_2201_02789_amd/csrc/dpo_kernels.hip",
                  "paper_2201_02789_amd/csrc/dpo_host.hip",
                  "paper_2201_02789_amd/csrc/dpo_internal.h"]


def kernel_sources_sha():
    import hashlib
    h = hashlib.sha256()
    for f in KERNEL_SOURCES:
        with open(os.path.join(ROOT, f), "rb") as fh:
            h.update(fh.read())
    return h.hexdigest()


def measured_traffic(workload, options_label, key="hbm_bytes_per_launch"):
    """HBM bytes per launch (or another field) from the committed counter
    summary (profiles/<workload>_traffic.json: FETCH_SIZE and WRITE_SIZE per
    traversal, scaled by a plain copy of known size), or None when the kernels
    changed since the counters were taken or the options differ."""
    path = os.path.join(ROOT, "profiles", f"{workload}_traffic.json")
    if not os.path.exists(path):
        return None
    with open(path) as f:
        t = json.load(f)
    if t.get("kernel_sources_sha256") != kernel_sources_sha() or t.get("options") != options_label:
        return None
    return t.get(key)


def algorithmic_bytes(kind, m_r, n_r):
    # BFS: col_idx + level probe per edge, row_ptr pair + level write + frontier
    # write/read per reached vertex.  SSSP: col + weight + dist probe per edge.
    return (8 * m_r + 20 * n_r) if kind == "bfs" else (12 * m_r + 24 * n_r)


def host_cpu():
    """CPU model and the cores this process may use."""
    model = "unknown"
    try:
        with open("/proc/cpuinfo") as f:
            for ln in f:
                if ln.startswith("model name"):
                    model = ln.split(":", 1)[1].strip()
                    break
    except OSError:
        pass
    return f"{model}, {len(os.sched_getaffinity(0))} usable cores"


def cpu_baseline(wl, min_seconds=10.0, max_seconds=30.0):
    """The oracle on this host, single thread, over the workload's sources in
    order (repeated if need be) until at least min_seconds of work."""
    import oracle
    t0 = time.perf_counter()
    edges, runs, dt = 0, 0, 0.0
    while dt < min_seconds:
        s = wl.sources[runs % len(wl.sources)]
        if wl.kind == "bfs":
            lv, _ = oracle.bfs(wl.g, int(s))
            reached = lv >= 0
        else:
            d = oracle.dijkstra(wl.g, int(s))
            reached = d != 0xFFFFFFFF
        edges += int(np.diff(wl.g.row_ptr)[reached].sum())
        runs += 1
        dt = time.perf_counter() - t0
        if dt * (runs + 1) / runs > max_seconds:
            break
    return {"value": round(edges / 2 / dt / 1e9, 4), "unit": "GTEPS", "cores": 1,
            "kind": "oracle", "host": host_cpu(),
            "sample": f"{runs} traversals over the workload's {len(wl.sources)} source(s) in order, "
                      f"one full {'queue BFS' if wl.kind == 'bfs' else 'binary-heap Dijkstra'} each, "
                      f"single thread, {dt:.1f} s"}


# ---------------------------------------------------------------- calibration
_calib = None


def calib_lib():
    """libdpo_calib.so: the primitive microbenchmarks (measurement only)."""
    global _calib
    if _calib is None:
        import ctypes
        path = os.path.join(ROOT, "paper_2201_02789_amd", "libdpo_calib.so")
        if not os.path.exists(path):
            raise RuntimeError(f"{path} is missing: build it with __graft_entry__.build()")
        L = ctypes.CDLL(path)
        vp, u32, i32 = ctypes.c_void_p, ctypes.c_uint32, ctypes.c_int
        L.dpo_calib_random_loads.argtypes = [vp, u32, u32, i32, vp, vp]
        L.dpo_calib_stream.argtypes = [vp, u32, i32, i32, vp, vp]
        L.dpo_calib_stream_probe.argtypes = [vp, u32, vp, u32, i32, vp, vp]
        L.dpo_calib_random_atomic_or.argtypes = [vp, u32, u32, i32, vp]
        L.dpo_calib_workgroup_atomics.argtypes = [vp, u32, u32, i32, vp]
        L.dpo_calib_workgroup_placement.argtypes = [i32, i32, vp, vp]
        L.dpo_calib_random_coherent_loads.argtypes = [vp, u32, u32, i32, vp, vp]
        L.dpo_calib_random_atomic_or_ret.argtypes = [vp, u32, u32, i32, vp, vp]
        L.dpo_calib_random_stores.argtypes = [vp, u32, u32, i32, vp]
        L.dpo_calib_loads_and_atomics.argtypes = [vp, vp, u32, u32, u32, u32, i32, vp, vp]
        _calib = L
    return _calib


def _timed(torch, fn, reps=3):
    """Best of reps: ms of fn(stream_ptr) between two events on torch's stream."""
    stream = torch.cuda.current_stream()
    best = float("inf")
    for _ in range(reps + 1):  # the first run warms up
        e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
        e0.record(stream)
        if fn(stream.cuda_stream) != 0:
            raise RuntimeError("calibration launch failed")
        e1.record(stream)
        torch.cuda.synchronize()
        best = min(best, e0.elapsed_time(e1))
    return best


def random_load_rate(torch, table_bytes, grid=2048, iters=32):
    """Random 4-byte loads per second from a table of table_bytes (a power of
    two), 8 independent loads in flight per lane."""
    L = calib_lib()
    words = table_bytes // 4
    table = torch.ones(words, dtype=torch.int32, device="cuda")
    out = torch.empty(grid * 256, dtype=torch.int32, device="cuda")
    ms = _timed(torch, lambda st: L.dpo_calib_random_loads(table.data_ptr(), words, iters, grid,
                                                           out.data_ptr(), st))
    return grid * 256 * iters * 8 / (ms * 1e-3)


def calibrate_primitives(torch):
    """Rates of the memory primitives the level kernels are built from."""
    L = calib_lib()
    grid = 2048
    out = torch.empty(grid * 256, dtype=torch.int32, device="cuda")
    res = {}
    for kb in (512, 8 << 10, 16 << 10, 256 << 10):
        res[f"random_load_{kb}KiB_G_per_s"] = round(random_load_rate(torch, kb << 10) / 1e9, 1)
    for kb in (512, 8 << 10):
        words = (kb << 10) // 4
        t = torch.ones(words, dtype=torch.int32, device="cuda")
        ms = _timed(torch, lambda st: L.dpo_calib_random_coherent_loads(t.data_ptr(), words, 32, grid,
                                                                        out.data_ptr(), st))
        res[f"random_coherent_load_{kb}KiB_G_per_s"] = round(grid * 256 * 32 * 8 / (ms * 1e-3) / 1e9, 1)
    n = 128 << 20  # 512 MiB of int32
    a = torch.ones(n, dtype=torch.int32, device="cuda")
    ms = _timed(torch, lambda st: L.dpo_calib_stream(a.data_ptr(), n, 0, grid, out.data_ptr(), st))
    res["stream_int32_GB_per_s"] = round(n * 4 / (ms * 1e-3) / 1e9, 1)
    ms = _timed(torch, lambda st: L.dpo_calib_stream(a.data_ptr(), n // 4, 1, grid, out.data_ptr(), st))
    res["stream_int4_GB_per_s"] = round(n * 4 / (ms * 1e-3) / 1e9, 1)
    col = torch.randint(0, 1 << 22, (n,), dtype=torch.int32, device="cuda")
    table = torch.ones(1 << 17, dtype=torch.int32, device="cuda")  # 512 KiB
    ms = _timed(torch, lambda st: L.dpo_calib_stream_probe(col.data_ptr(), n, table.data_ptr(), 1 << 17,
                                                           grid, out.data_ptr(), st))
    res["stream_probe_512KiB_G_elems_per_s"] = round(n / (ms * 1e-3) / 1e9, 1)
    del col, a
    for kb in (512, 64 << 10):
        words = (kb << 10) // 4
        t = torch.zeros(words, dtype=torch.int32, device="cuda")
        ms = _timed(torch, lambda st: L.dpo_calib_random_atomic_or(t.data_ptr(), words, 8, grid, st))
        res[f"random_atomic_or_{kb}KiB_G_per_s"] = round(grid * 256 * 8 * 8 / (ms * 1e-3) / 1e9, 2)
    for kb in (512, 16 << 10):
        words = (kb << 10) // 4
        t = torch.zeros(words, dtype=torch.int32, device="cuda")
        ms = _timed(torch, lambda st: L.dpo_calib_random_atomic_or_ret(t.data_ptr(), words, 8, grid,
                                                                       out.data_ptr(), st))
        res[f"random_atomic_or_returning_{kb}KiB_G_per_s"] = round(grid * 256 * 8 * 8 / (ms * 1e-3) / 1e9, 2)
        ms = _timed(torch, lambda st: L.dpo_calib_random_stores(t.data_ptr(), words, 16, grid, st))
        res[f"random_store_{kb}KiB_G_per_s"] = round(grid * 256 * 16 * 8 / (ms * 1e-3) / 1e9, 1)
    # loads of a 512 KiB table by 15 of every 16 workgroups, while the 16th
    # run returning atomics on the same table or on a second one
    words, every, it = 1 << 17, 16, 16
    lt = torch.zeros(words, dtype=torch.int32, device="cuda")
    at = torch.zeros(words, dtype=torch.int32, device="cuda")
    loads = (grid - (grid + every - 1) // every) * 256 * it * 8
    for key, tbl, mode in (("loads_alone", lt, 1), ("atomics_alone", lt, 2),
                           ("loads_with_atomics_same_table", lt, 3),
                           ("loads_with_atomics_other_table", at, 3)):
        ms = _timed(torch, lambda st: L.dpo_calib_loads_and_atomics(lt.data_ptr(), tbl.data_ptr(), words,
                                                                    it, every, mode, grid,
                                                                    out.data_ptr(), st))
        res[f"mixed_512KiB_{key}_ms"] = round(ms, 4)
        if mode != 2:
            res[f"mixed_512KiB_{key}_load_G_per_s"] = round(loads / (ms * 1e-3) / 1e9, 1)
    # where workgroups run: the XCC id each one reads from its hardware
    # register, against workgroup % 8 (round-robin placement over the XCDs)
    for g in (2048, 4096):
        pl = torch.zeros(2 * g, dtype=torch.int32, device="cuda")
        if L.dpo_calib_workgroup_placement(g, 256, pl.data_ptr(),
                                           torch.cuda.current_stream().cuda_stream) != 0:
            raise RuntimeError("placement probe failed")
        torch.cuda.synchronize()
        xcc = pl.cpu().numpy()[0::2] & 0xF
        res[f"placement_{g}_wg_xcc_equals_wg_mod_8"] = round(float(np.mean(xcc == np.arange(g) % 8)), 4)
        res[f"placement_{g}_wg_per_xcc"] = np.bincount(xcc, minlength=8).tolist()
    ctr = torch.zeros(8 * 32, dtype=torch.int32, device="cuda")
    for naddr in (1, 8):
        ms = _timed(torch, lambda st: L.dpo_calib_workgroup_atomics(ctr.data_ptr(), naddr, 16, grid, st))
        res[f"workgroup_atomic_{naddr}_address_ns_per_op"] = round(ms * 1e6 / (grid * 16), 3)
    return res


# ---------------------------------------------------------------- profiles
COPY_BYTES = 512 << 20  # --calibrate-copy: bytes read and written per copy
COPY_REPS = 3


def _csv(dirpath, suffix):
    import csv
    import glob
    files = sorted(glob.glob(os.path.join(dirpath, "**", f"*{suffix}"), recursive=True))
    if not files:
        raise SystemExit(f"no *{suffix} under {dirpath}")
    with open(files[0]) as f:
        return list(csv.DictReader(f))


def _short(name):
    return name.split("(")[0].replace("void ", "").replace("dpo::", "")


# counter passes of --summarize-counters (each within the per-block limits of
# one rocprofv3 --pmc run: at most 8 SQ, 4 TCP, 2 TA and 2 GRBM counters)
COUNTER_PASSES = [
    "SQ_WAVES SQ_WAVE_CYCLES SQ_BUSY_CYCLES SQ_WAIT_INST_ANY SQ_WAIT_ANY SQ_ACTIVE_INST_VALU "
    "SQ_ACTIVE_INST_VMEM SQ_ACTIVE_INST_ANY GRBM_GUI_ACTIVE",
    "SQ_INSTS_VALU SQ_INSTS_SALU SQ_INSTS_VMEM_RD SQ_INSTS_VMEM_WR SQ_INSTS_LDS SQ_INSTS_SMEM "
    "SQ_INSTS_BRANCH SQ_INST_LEVEL_VMEM",
    "TA_BUSY_avr TA_ADDR_STALLED_BY_TC_CYCLES_sum TCP_PENDING_STALL_CYCLES_sum TCP_TCC_READ_REQ_sum "
    "TCP_TCC_READ_REQ_LATENCY_sum TCP_TCR_TCP_STALL_CYCLES_sum GRBM_GUI_ACTIVE GRBM_TA_BUSY",
    "TCP_UTCL1_STALL_INFLIGHT_MAX_sum TCP_READ_TAGCONFLICT_STALL_CYCLES_sum "
    "TCP_TCC_ATOMIC_WITH_RET_REQ_sum TCP_TD_TCP_STALL_CYCLES_sum TA_DATA_STALLED_BY_TC_CYCLES_sum "
    "TA_TA_BUSY_sum"]


def simulate_bands(deltas=(32, 64, 128, 256, 512)):
    """Host simulation (numpy, no GPU) of synchronous frontier Bellman-Ford on
    the s21 SSSP graph, plain and with a near-far band split of width delta:
    an improved vertex whose distance is at or above the current band's upper
    bound is not expanded; when no frontier is left, the next band's vertices
    are selected by a scan of all distances.  Counts the edges relaxed and the
    levels (scan levels included), the quantities that decide whether deferral
    could pay on this graph.  Writes profiles/sssp21_bands.md."""
    from paper_2201_02789_amd import graphgen as gg
    g = gg.add_weights(gg.rmat(21, 16, 21, perm_seed=24), 31)
    rp = g.row_ptr.astype(np.int64)
    col = g.col_idx.astype(np.int64)
    w = g.weights.astype(np.int64)
    n, src, inf = g.n, int(gg.max_degree_vertex(g)), np.int64(1) << 40

    def run(delta):
        d = np.full(n, inf)
        d[src] = 0
        front, bound = np.array([src], np.int64), (delta or inf)
        relaxed = levels = scans = deferred = 0
        while True:
            levels += 1
            if len(front) == 0:
                if not delta:
                    break
                lo, bound = bound, bound + delta  # every finite d >= lo is pending
                scans += 1
                front = np.nonzero((d >= lo) & (d < bound))[0]
                if len(front) == 0 and not np.any((d >= bound) & (d < inf)):
                    break
                continue
            near = d[front] < bound
            deferred += int(np.count_nonzero(~near))
            fr = front[near]
            deg = rp[fr + 1] - rp[fr]
            relaxed += int(deg.sum())
            e = np.repeat(rp[fr] - (np.cumsum(deg) - deg), deg) + np.arange(int(deg.sum()))
            old = d.copy()
            np.minimum.at(d, col[e], np.repeat(d[fr], deg) + w[e])
            front = np.nonzero(d < old)[0]
        return relaxed, levels, scans, deferred, d

    base = run(0)
    reached = base[4] < inf
    m_reached = int((rp[1:] - rp[:-1])[reached].sum())
    rows = [("plain", base)] + [(str(dl), run(dl)) for dl in deltas]
    for _, r in rows:
        assert np.array_equal(r[4], base[4])
    md = ["# sssp21: synchronous frontier Bellman-Ford with a near-far band split (host simulation)",
          "", "Command (repository root): `python3 bench.py --simulate-bands` (numpy, no GPU).", "",
          f"Graph: R-MAT scale 21, edgefactor 16, weights U[1,255], max-degree source; "
          f"{m_reached / 1e6:.1f} M edges out of reached vertices, largest distance "
          f"{int(base[4][reached].max())}.  Every row reaches the same distances.", "",
          "| band width | edges relaxed (M) | per reached edge | levels | scan levels | deferred entries (M) |",
          "|---|---|---|---|---|---|"]
    md += [f"| {k} | {r[0] / 1e6:.1f} | {r[0] / m_reached:.2f} | {r[1]} | {r[2]} | {r[3] / 1e6:.2f} |"
           for k, r in rows]
    with open(os.path.join(ROOT, "profiles", "sssp21_bands.md"), "w") as f:
        f.write("\n".join(md) + "\n")
    return {k: {"relaxed": r[0], "levels": r[1], "scans": r[2]} for k, r in rows}


def summarize_counters(args, d):
    """Where the level kernels' waves spend their time, from the counter passes
    under d (<workload>_p1 .. _p4, one rocprofv3 --pmc run each): issue and
    wait shares of wave time, wave instructions per edge run, average L2 read
    latency, texture-addresser busy share."""
    import csv
    import glob
    name = args.workload
    extra = "" if name == "bfs22" else f" --workload {name}"
    agg, trav = {}, {}
    for i in range(1, len(COUNTER_PASSES) + 1):
        files = glob.glob(os.path.join(d, f"{name}_p{i}", "**", "*counter_collection.csv"), recursive=True)
        if not files:
            raise SystemExit(f"no counter CSV for pass {i} under {d}")
        ncnt = len(COUNTER_PASSES[i - 1].split())
        inits = 0
        for r in csv.DictReader(open(files[0])):
            n = _short(r["Kernel_Name"])
            if n == "init_kernel":
                inits += 1
            if n.startswith(LEVEL_KERNELS):
                c = agg.setdefault(n, {})
                c[r["Counter_Name"]] = c.get(r["Counter_Name"], 0.0) + float(r["Counter_Value"])
        trav[i] = inits / ncnt  # one row per counter per dispatch
    # edges run per traversal: the bench line that the first pass's run printed
    with open(os.path.join(d, f"{name}_p1.out")) as f:
        line = json.loads([ln for ln in f if ln.startswith("{")][-1])
    edges = line["roofline_probe"]["probes_per_traversal"]
    md = [f"# {name}: where the level kernels' waves spend their time (rocprofv3 counters)", "",
          "Commands (MI355X, repository root, after `export TMPDIR=/tmp`), one run per pass:", "", "```"]
    md += [f"rocprofv3 --pmc {p} --output-format csv -d {d}/{name}_p{i + 1} -o c -- python3 bench.py"
           f"{extra} --no-cpu --no-extras --no-baselines --steps 1 --warmup 1 > {d}/{name}_p{i + 1}.out"
           for i, p in enumerate(COUNTER_PASSES)]
    md += [f"python3 bench.py{extra} --summarize-counters {d}", "```", "",
           f"Traversals per run: {trav[1]:.0f}; edges run per traversal {edges:.0f}.  Shares are of "
           "SQ_WAVE_CYCLES (the waves' resident time); per-edge counts are wave instructions "
           "(one per 64 lanes).", "",
           "| kernel | issuing any / VALU | waiting on memory (WAIT_INST_ANY) | waiting on anything (WAIT_ANY) | "
           "VALU / SALU / VMEM-read / LDS / branch per edge | L2 read latency (cycles) | TA busy |",
           "|---|---|---|---|---|---|---|"]
    for n, c in sorted(agg.items()):
        wc = max(c.get("SQ_WAVE_CYCLES", 0.0), 1.0)
        per = edges * trav[2]
        md.append(f"| {n} | {c['SQ_ACTIVE_INST_ANY'] / wc:.3f} / {c['SQ_ACTIVE_INST_VALU'] / wc:.3f} | "
                  f"{c['SQ_WAIT_INST_ANY'] / wc:.3f} | {c['SQ_WAIT_ANY'] / wc:.3f} | "
                  f"{c['SQ_INSTS_VALU'] / per:.2f} / {c['SQ_INSTS_SALU'] / per:.2f} / "
                  f"{c['SQ_INSTS_VMEM_RD'] / per:.3f} / {c['SQ_INSTS_LDS'] / per:.3f} / "
                  f"{c['SQ_INSTS_BRANCH'] / per:.3f} | "
                  f"{c['TCP_TCC_READ_REQ_LATENCY_sum'] / max(c['TCP_TCC_READ_REQ_sum'], 1):.0f} | "
                  f"{c['TA_BUSY_avr'] / max(c['GRBM_GUI_ACTIVE'], 1):.3f} |")
    md += ["", "Raw sums over the run's dispatches:", "", "| kernel | counter | value |", "|---|---|---|"]
    for n, c in sorted(agg.items()):
        md += [f"| {n} | {k} | {v:.4g} |" for k, v in sorted(c.items())]
    out = os.path.join(ROOT, "profiles", f"{name}_counters.md")
    with open(out, "w") as f:
        f.write("\n".join(md) + "\n")
    print(json.dumps({"wrote": out}))


def summarize_profiles(args, d):
    """Level-step kernel time from a kernel trace and HBM bytes from FETCH_SIZE
    / WRITE_SIZE counter runs, each counter scaled by what it reads for a plain
    copy of known size."""
    with open(os.path.join(d, "trace", "out.json")) as f:
        line = json.loads([ln for ln in f if ln.startswith("{")][-1])
    label, launches_per = line["config"]["options"], line["roofline"]["launches_per_traversal"]
    step = LEVEL_KERNELS

    trace = _csv(os.path.join(d, "trace"), "kernel_trace.csv")
    rows = [(int(r["Start_Timestamp"]), int(r["End_Timestamp"]), _short(r["Kernel_Name"])) for r in trace]
    stats = {}
    for t0, t1, n in rows:
        c, tot = stats.get(n, (0, 0))
        stats[n] = (c + 1, tot + (t1 - t0))
    traversals = sum(1 for _, _, n in rows if n == "init_kernel")
    step_ns = sum(t1 - t0 for t0, t1, n in rows if n.startswith(step))
    launches = traversals * launches_per
    kernel_us = step_ns / launches / 1e3

    def per_dispatch(sub, counter):
        return [(_short(r["Kernel_Name"]), float(r["Counter_Value"]))
                for r in _csv(os.path.join(d, sub), "counter_collection.csv")
                if r["Counter_Name"] == counter]

    def copy_scale(sub, counter):
        # every dispatch of the device copies (however the runtime splits them)
        vals = [v for n, v in per_dispatch(sub, counter) if "copy" in n.lower()]
        return COPY_REPS * COPY_BYTES / (sum(vals) * 1024)

    sf, sw = copy_scale("copy_fetch", "FETCH_SIZE"), copy_scale("copy_write", "WRITE_SIZE")
    fetch = [(n, v) for n, v in per_dispatch("fetch", "FETCH_SIZE") if n.startswith(step)]
    write = [(n, v) for n, v in per_dispatch("write", "WRITE_SIZE") if n.startswith(step)]
    trav_pmc = sum(1 for n, _ in per_dispatch("fetch", "FETCH_SIZE") if n == "init_kernel")
    launches_pmc = trav_pmc * launches_per
    fetch_b = sum(v for _, v in fetch) * 1024 * sf / launches_pmc
    write_b = sum(v for _, v in write) * 1024 * sw / launches_pmc
    traffic = {"workload": args.workload, "options": label,
               "kernel_sources_sha256": kernel_sources_sha(),
               "hbm_bytes_per_launch": round(fetch_b + write_b),
               "fetch_bytes_per_launch": round(fetch_b), "write_bytes_per_launch": round(write_b),
               "fetch_scale": round(sf, 4), "write_scale": round(sw, 4),
               "traversals": trav_pmc, "launches_per_traversal": launches_per}

    alg = line["roofline"]["algorithmic_bytes_per_launch"]
    # the library's kernels (torch's kernels of the untimed result certificates
    # and the calibration kernel of the probe roofline are left out)
    ours = LEVEL_KERNELS + ("init_kernel", "admit", "advance", "clear_found", "__amd_rocclr")
    top = sorted(((n, v) for n, v in stats.items() if n.startswith(ours)), key=lambda kv: -kv[1][1])[:8]
    md = [f"# {args.workload}: kernel time and HBM traffic ({label})", "",
          "Commands (MI355X, from the repository root, after `export TMPDIR=/tmp`):", "",
          "```"] + [ln.rstrip() for ln in open(os.path.join(d, "commands.txt"))] + ["```", "",
          "## Kernel trace (`rocprofv3 --kernel-trace --stats`)", "",
          "The library's kernels; the trace also holds torch's kernels of the untimed result "
          "certificates and the probe-ceiling calibration kernel, which are not listed.", "",
          "| kernel | calls | total ms | mean us |", "|---|---|---|---|"]
    md += [f"| {n} | {c} | {t / 1e6:.3f} | {t / c / 1e3:.2f} |" for n, (c, t) in top]
    md += ["", f"Traversals traced: {traversals}; level-step launches per traversal "
               f"{launches_per:.4g} (levels + 1).",
           f"Level step (parent_kernel + child_kernel"
           f" + harvest_kernel{'; the parent kernel runs as two kernels, pass 1 before and pass 2 after the child kernel' if args.workload.startswith('sssp') else ''}"
           f") kernel time per launch: **{kernel_us:.2f} us** "
           f"(bench line of the traced run: mean_launch_us {line['roofline']['mean_launch_us']}, "
           f"which also holds the gaps between graph nodes).", "",
           "## HBM traffic (`rocprofv3 --pmc FETCH_SIZE`, then `--pmc WRITE_SIZE`)", "",
           f"Copy calibration (`bench.py --calibrate-copy`, {COPY_BYTES >> 20} MiB read + written): "
           f"bytes = counter KiB x 1024 x {sf:.4f} (fetch), x {sw:.4f} (write).", "",
           f"Per level-step launch over {trav_pmc} traversals: fetch {fetch_b / 1e6:.2f} MB, "
           f"write {write_b / 1e6:.2f} MB, total **{(fetch_b + write_b) / 1e6:.2f} MB** "
           f"vs algorithmic {alg / 1e6:.2f} MB ({(fetch_b + write_b) / alg:.2f}x).", "",
           f"kernel_sources_sha256 `{traffic['kernel_sources_sha256']}`", ""]
    # the same counters per level kernel (FETCH / WRITE per traversal)
    md += ["### Per kernel (per traversal)", "", "| kernel | fetch MB | write MB |", "|---|---|---|"]
    per_k = {}
    for n, v in fetch:
        per_k.setdefault(n, [0.0, 0.0])[0] += v * 1024 * sf / trav_pmc
    for n, v in write:
        per_k.setdefault(n, [0.0, 0.0])[1] += v * 1024 * sw / trav_pmc
    md += [f"| {n} | {f / 1e6:.1f} | {w / 1e6:.1f} |" for n, (f, w) in sorted(per_k.items())]
    md += [""]
    traffic["per_kernel_bytes_per_traversal"] = {n: [round(f), round(w)] for n, (f, w) in per_k.items()}
    l2 = os.path.join(d, "l2")
    if os.path.isdir(l2):
        # L2 requests of the child kernel (counter run of its own; TCC_* summed
        # over the 16 channels of each XCD and over the XCDs)
        rows = _csv(l2, "counter_collection.csv")
        disp = {}
        for r in rows:
            n = _short(r["Kernel_Name"])
            if not n.startswith("child_kernel"):
                continue
            e = disp.setdefault(r["Dispatch_Id"], {"ns": int(r["End_Timestamp"]) - int(r["Start_Timestamp"])})
            e[r["Counter_Name"]] = float(r["Counter_Value"])
        big = sorted(disp.values(), key=lambda e: -e["ns"])[:max(1, len(disp) // 16)]
        req = sum(e.get("TCC_REQ_sum", 0) for e in big)
        hit = sum(e.get("TCC_HIT_sum", 0) for e in big)
        miss = sum(e.get("TCC_MISS_sum", 0) for e in big)
        ns = sum(e["ns"] for e in big)
        md += ["## L2 requests of the child kernel (`rocprofv3 --pmc TCC_REQ_sum TCC_HIT_sum "
               "TCC_MISS_sum`)", "",
               f"Longest {len(big)} of {len(disp)} child dispatches: {req / 1e6:.1f} M L2 requests, "
               f"hit rate {hit / max(hit + miss, 1):.3f}, over {ns / 1e6:.3f} ms (durations "
               f"of the counter run): **{req / ns:.1f} G requests/s**, against about 265 G/s measured "
               f"for random 4-byte loads from a 512 KB table (one request per L2 channel "
               f"and clock).", ""]
        traffic["l2_requests_per_s"] = round(req / ns * 1e9)
        # every level kernel: L2 requests, hit rate and request rate over all its dispatches
        allk = {}
        for r in rows:
            n = _short(r["Kernel_Name"])
            if not n.startswith(step):
                continue
            e = allk.setdefault(n, {}).setdefault(
                r["Dispatch_Id"], {"ns": int(r["End_Timestamp"]) - int(r["Start_Timestamp"])})
            e[r["Counter_Name"]] = float(r["Counter_Value"])
        md += ["| kernel | dispatches | L2 requests (M) | hit rate | G requests/s |", "|---|---|---|---|---|"]
        for n, dd in sorted(allk.items()):
            q = sum(e.get("TCC_REQ_sum", 0) for e in dd.values())
            h = sum(e.get("TCC_HIT_sum", 0) for e in dd.values())
            mi = sum(e.get("TCC_MISS_sum", 0) for e in dd.values())
            t = sum(e["ns"] for e in dd.values())
            md.append(f"| {n} | {len(dd)} | {q / 1e6:.1f} | {h / max(h + mi, 1):.3f} | {q / max(t, 1):.1f} |")
        md.append("")
    out_json = os.path.join(ROOT, "profiles", f"{args.workload}_traffic.json")
    with open(out_json, "w") as f:
        json.dump(traffic, f, indent=1)
        f.write("\n")
    out_md = os.path.join(ROOT, "profiles", f"{args.workload}_kernels.md")
    with open(out_md, "w") as f:
        f.write("\n".join(md))
    print(json.dumps({"wrote": [out_md, out_json], "kernel_us_per_launch": round(kernel_us, 2),
                      "traffic": traffic}))


def workload_line(args, dpo, torch, name, steps, warmup, with_cpu, with_baselines, overrides=True):
    """Measures one traversal workload; returns its JSON line (None for --sweep).
    `overrides`: apply the command line's threshold / coarsening / granularity."""
    wl = Workload(name)
    dg = dpo.DeviceGraph.from_host(wl.g)
    tuned = dict(TUNED[name])
    if overrides and args.threshold is not None:
        tuned["threshold"] = args.threshold
    if overrides and args.coarsen is not None:
        tuned["coarsen"] = args.coarsen
    if overrides and args.split_min is not None:
        tuned["split_min"] = args.split_min
    if overrides and args.serial_wave is not None:
        tuned["serial_wave"] = args.serial_wave
    if overrides and args.dyn_share is not None:
        tuned["dyn_share"] = args.dyn_share
    if overrides and args.child_block is not None:
        tuned["child_block"] = args.child_block
    if overrides and args.claim_hint is not None:
        tuned["claim_hint"] = args.claim_hint
    a = agg_of(args.agg) if overrides else None
    if a:
        tuned["agg"], tuned["agg_blocks"] = a
    opts = dpo.Options(**tuned)

    if args.sweep:
        sweep(dpo, torch, wl, dg, "python3 bench.py " + " ".join(sys.argv[1:]))
        return None

    # untimed run with counters: edges reached and level count per source
    rs, certified = reached_stats(dpo, torch, wl, dg, opts)
    if certified != len(wl.sources):
        log(f"[bench] ERROR: {len(wl.sources) - certified} of {len(wl.sources)} results fail "
            f"their edge certificates")
    levels = max(r[2]["levels"] for r in rs)
    opts.steps_per_replay = levels + 1  # one replay covers a traversal
    m_r = np.array([r[0] for r in rs], dtype=np.float64)
    n_r = np.array([r[1] for r in rs], dtype=np.float64)
    log(f"[bench] options {opts.label()} steps/replay {opts.steps_per_replay}; "
        f"m_r mean {m_r.mean():.0f}, n_r mean {n_r.mean():.0f}")

    per_call, wall = measure(dpo, torch, wl, dg, opts, steps, warmup)
    t_step_ms = per_call.sum(axis=1)  # ms per step (all sources)
    total_ms = float(per_call.sum())
    edges_step = float((m_r / 2).sum())
    gteps = steps * edges_step / (total_ms * 1e-3) / 1e9
    log(f"[bench] T+C+A: {gteps:.2f} GTEPS, {t_step_ms.mean():.3f} ms/step, wall {wall:.3f}s")

    # roofline of the level-step kernel: algorithmic bytes per launch / mean
    # launch duration, both per traversal divided by its launch count
    launches = np.array([r[2]["levels"] + 1 for r in rs], dtype=np.float64)
    bytes_call = algorithmic_bytes(wl.kind, m_r, n_r)
    mean_call_ms = per_call.mean(axis=0)
    achieved = float((bytes_call.sum() / launches.sum()) /
                     ((mean_call_ms.sum() * 1e-3) / launches.sum()) / 1e9)
    roofline = {"bound": "hbm", "achieved": round(achieved, 1), "peak": HBM_PEAK_GBS,
                "unit": "GB/s", "frac": round(achieved / HBM_PEAK_GBS, 4),
                "traffic": measured_traffic(name, opts.label()),
                "kernel": (f"level step: parent_kernel + child_kernel"
                           f"{' + parent_kernel pass 2' if wl.kind == 'sssp' else ''} + harvest_kernel "
                           f"<{wl.kind.upper()}, {opts.label()}>"),
                "launches_per_traversal": float(launches.mean()),
                "mean_launch_us": round(float(mean_call_ms.sum() / launches.sum() * 1e3), 2),
                "algorithmic_bytes_per_launch": round(float(bytes_call.sum() / launches.sum()))}

    # second roofline: the child body's dependent random probes (BFS: the
    # n-bit visited bitmap; SSSP: the n-word distance array), one per edge
    # run, against the rate the chip sustains for random 4-byte loads from a
    # table of that size (measured here, 8 loads in flight per lane)
    probed_bytes = wl.g.n // 8 if wl.kind == "bfs" else 4 * wl.g.n
    table = 1 << max(12, int(np.ceil(np.log2(max(probed_bytes, 1)))))
    ceiling = random_load_rate(torch, table)
    probes = np.array([r[2]["edges_serial"] + r[2]["edges_child"] for r in rs], dtype=np.float64)
    p_rate = float((probes.sum() / launches.sum()) / ((mean_call_ms.sum() * 1e-3) / launches.sum()))
    counters = measured_traffic(name, opts.label(), "l2_requests_per_s")
    roofline_probe = {"bound": "random 4-byte loads", "achieved": round(p_rate / 1e9, 2),
                      "peak": round(ceiling / 1e9, 2), "unit": "G loads/s",
                      "frac": round(p_rate / ceiling, 4),
                      "table_bytes": table, "probes_per_traversal": float(probes.mean()),
                      "child_l2_requests_per_s_counters": counters,
                      "hbm_frac_cap": round(float(bytes_call.sum() / probes.sum()) * ceiling / 1e9
                                            / HBM_PEAK_GBS, 4)}
    log(f"[bench] probes {p_rate / 1e9:.1f} G/s of {ceiling / 1e9:.1f} G/s measured ceiling")

    baselines = {}
    if with_baselines:
        for name, o in (("flat", dpo.Options.flat()),
                        ("naive", dpo.Options.naive(child_block=opts.child_block))):
            o.steps_per_replay = opts.steps_per_replay
            pc, _ = measure(dpo, torch, wl, dg, o, 1, 1)
            g_b = edges_step / (pc.sum() * 1e-3) / 1e9
            baselines[name] = {"gteps": round(g_b, 3), "ms_per_step": round(float(pc.sum()), 3),
                               "options": o.label()}
            log(f"[bench] {name}: {g_b:.3f} GTEPS")

    # the same options with the paper's literal serial children (each in its
    # parent's lane, Sec. III-B) and with the library's default replay length
    # (16 level steps per replay instead of the traversal's level count + 1)
    variants = {}
    if with_baselines:
        for vname, over in (("serial_wave_0", {"serial_wave": 0}),
                            ("default_steps_per_replay", {"steps_per_replay": 0})):
            o = dpo.Options(**{**opts.__dict__, **over})
            pc, _ = measure(dpo, torch, wl, dg, o, max(1, min(steps, 3)), 1)
            g_v = edges_step * pc.shape[0] / (pc.sum() * 1e-3) / 1e9
            variants[vname] = {"gteps": round(g_v, 3), "ms_per_step": round(float(pc.sum(axis=1).mean()), 3),
                               "options": o.label(), "steps_per_replay": o.steps_per_replay or 16}
            log(f"[bench] {vname}: {g_v:.3f} GTEPS")

    cpu = None
    if with_cpu:
        cpu = cpu_baseline(wl, args.cpu_seconds)
        log(f"[bench] oracle: {cpu['value']} GTEPS ({cpu['sample']})")

    line = {
        "metric": "GTEPS (BFS/SSSP, R-MAT s22) vs flat & naive-nested",
        "value": round(gteps, 3),
        "unit": "GTEPS",
        "n_gpus": 1,
        "steps": steps,
        "warmup": warmup,
        "ms_per_step": round(float(t_step_ms.mean()), 4),
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "int32",
        "data": ("synthetic (seeded Erdos-Renyi control)" if name == "er22" else
                 "synthetic (seeded R-MAT, stands in for the paper's Kronecker graph)"),
        "config": {"workload": wl.desc, "n": wl.g.n, "m": wl.g.m,
                   "sources": int(len(wl.sources)), "options": opts.label(),
                   "steps_per_replay": opts.steps_per_replay,
                   "mean_reached_edges": float(m_r.mean()),
                   "gteps_convention": "undirected edges in the reached component / time, "
                                       "summed over sources",
                   "directed_edges_per_s": round(2 * gteps * 1e9),
                   "ms_per_traversal_mean": round(float(per_call.mean()), 4),
                   "ms_per_traversal_median": round(float(np.median(per_call)), 4),
                   "verified": (f"edge certificates {certified}/{len(wl.sources)} pass "
                                f"(every source's result, untimed run with the timed options)"),
                   # edges the traversal actually relaxes per reached directed edge
                   # (1 for BFS; above 1 for the frontier Bellman-Ford of SSSP)
                   "work_efficiency": round(float(np.mean(
                       [(r[2]["edges_serial"] + r[2]["edges_child"]) / max(r[0], 1) for r in rs])), 3)},
        "roofline": roofline,
        "roofline_probe": roofline_probe,
        "baselines": baselines,
        "variants": variants,
        "speedup_vs_flat": round(gteps / baselines["flat"]["gteps"], 2) if baselines else None,
        "speedup_vs_naive": round(gteps / baselines["naive"]["gteps"], 2) if baselines else None,
        "cpu_baseline": cpu,
    }
    line["_graph"] = (wl, dg)
    return line


def main():
    args = parse()
    if args.summarize_profiles:
        return summarize_profiles(args, args.summarize_profiles)
    if args.summarize_counters:
        return summarize_counters(args, args.summarize_counters)
    if args.simulate_bands:
        print(json.dumps(simulate_bands()), flush=True)
        return
    if args.gpus != 1:
        print(f"bench.py runs on one GPU only (asked for --gpus {args.gpus}); "
              "(independent traversals shard by graph across GPUs)", file=sys.stderr)
        sys.exit(2)
    import torch
    from paper_2201_02789_amd import dpo
    assert torch.cuda.is_available(), "bench.py needs a GPU"
    if args.calibrate_copy:
        # a plain copy of known size: its FETCH_SIZE / WRITE_SIZE counters give
        # the scale between those counters and bytes
        n = COPY_BYTES // 4
        src = torch.ones(n, dtype=torch.int32, device="cuda")
        dst = torch.empty_like(src)
        for _ in range(COPY_REPS):
            dst.copy_(src)
        torch.cuda.synchronize()
        print(json.dumps({"copy_bytes_read": n * 4, "copy_bytes_written": n * 4, "copies": COPY_REPS}))
        return
    dpo.lib()  # fail loudly if the HIP library is missing
    if args.calibrate_primitives:
        res = calibrate_primitives(torch)
        cmd = "python3 bench.py " + " ".join(sys.argv[1:])
        md = ["# Memory primitives of the level kernels (MI355X)", "",
              f"Command (repository root): `{cmd}` (kernels in "
              "`paper_2201_02789_amd/csrc/dpo_calib.hip`; best of 3 after a warm-up, HIP events; "
              "2048 workgroups of 256 lanes)", "", "| primitive | rate |", "|---|---|"]
        md += [f"| {k} | {v} |" for k, v in res.items()]
        with open(os.path.join(ROOT, "profiles", "primitives.md"), "w") as f:
            f.write("\n".join(md) + "\n")
        print(json.dumps(res), flush=True)
        return

    if args.breakdown:
        print(json.dumps(bench_breakdown(args, dpo, torch)), flush=True)
        return
    if args.workload == "batch":
        print(json.dumps(bench_batch(args, dpo, torch, full_line=True)), flush=True)
        return
    if args.workload == "serve":
        print(json.dumps(bench_serve(args, dpo, torch, full_line=True)), flush=True)
        return
    if args.workload == "road":
        print(json.dumps(bench_road(args, dpo, torch)), flush=True)
        return
    line = workload_line(args, dpo, torch, args.workload, args.steps, args.warmup,
                         not args.no_cpu, not args.no_baselines)
    if line is None:
        return
    del line["_graph"]
    if not args.no_extras and args.workload == "bfs22":
        torch.cuda.empty_cache()
        # the SSSP half of the metric: s21, tuned options, flat and naive beside it
        sp = workload_line(args, dpo, torch, "sssp21", 3, 1, not args.no_cpu, True,
                           overrides=False)
        del sp["_graph"]
        line["sssp"] = {k: sp[k] for k in ("value", "unit", "ms_per_step", "dtype", "config",
                                             "roofline", "roofline_probe", "baselines", "variants",
                                             "speedup_vs_flat", "speedup_vs_naive",
                                             "cpu_baseline")}
        torch.cuda.empty_cache()
        line["batched"] = bench_batch(args, dpo, torch)
        line["serving"] = bench_serve(args, dpo, torch)
    print(json.dumps(line), flush=True)


# ---------------------------------------------------------------- batched
def bench_batch(args, dpo, torch, full_line=False):
    """512 BFS over 64 R-MAT graphs (scales 10..18, edgefactor 8..32, 8
    sources each) packed in one CSR arena; threshold and coarsening tuned per
    size bucket (scales 10-12, 13-15, 16-18); one batch call per step."""
    from paper_2201_02789_amd import autotune
    from paper_2201_02789_amd import graphgen as gg
    t0 = time.time()
    graphs, queries = gg.batch_workload()
    arena, vbase = gg.pack_arena(graphs)
    da = dpo.DeviceArena(arena, vbase)
    scales = [int(np.log2(g.n)) for g in graphs]
    bucket = [0 if sc <= 12 else (1 if sc <= 15 else 2) for sc in scales]
    log(f"[batch] {len(graphs)} graphs, {len(queries)} queries, arena n={arena.n} m={arena.m} "
        f"({time.time() - t0:.1f}s)")
    base = dpo.Options(threshold=32, coarsen=1, agg=dpo.DPO_AGG_MULTIBLOCK, agg_blocks=4,
                       steps_per_replay=16, child_block=128)
    tuned, traces, gtrace = autotune.tune("bfs", da, graphs, queries, bucket, 3, base, max_runs=8,
                                          log=log)
    qs = [(g, s, bucket[g]) for g, s in queries]
    tot, slot0 = dpo.dpo_batch_slots(da, qs)
    out = torch.empty(tot, dtype=torch.int32, device="cuda")
    # one workspace for the tuned and the untuned point (granularities differ)
    ws = torch.empty(max(dpo.dpo_batch_workspace_bytes(da, qs, tuned[0]),
                         dpo.dpo_batch_workspace_bytes(da, qs, base)), dtype=torch.uint8,
                     device="cuda")
    deg = [g.degrees() for g in graphs]
    st = dpo.dpo_bfs_batch(da, qs, tuned, out, ws, stats=True)
    host = out.cpu().numpy()
    edges = 0
    for i, (g, s, b) in enumerate(qs):
        edges += int(deg[g][host[slot0[i]:slot0[i] + graphs[g].n] >= 0].sum())
    # one replay covers the batch (the counted run gave its level count)
    for o in tuned:
        o.steps_per_replay = st["levels"] + 1
    steps, warm = max(1, args.steps), max(1, args.warmup)
    for _ in range(warm):
        dpo.dpo_bfs_batch(da, qs, tuned, out, ws)
    torch.cuda.synchronize()
    ev0, ev1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
    ev0.record()
    for _ in range(steps):
        dpo.dpo_bfs_batch(da, qs, tuned, out, ws)
    ev1.record()
    torch.cuda.synchronize()
    ms = ev0.elapsed_time(ev1) / steps
    res = {"traversals_per_s": round(len(qs) / (ms * 1e-3), 1), "ms_per_batch": round(ms, 3),
           "gteps": round(edges / 2 / (ms * 1e-3) / 1e9, 3), "queries": len(qs),
           "levels": st["levels"],
           "tuned": [o.label() for o in tuned],
           "tuning_runs": [len(t) for t in traces],
           "tuning_trace": {"threshold_coarsening_per_bucket": [
                                {lbl: round(v * 1e3, 3) for lbl, v in t} for t in traces],
                            "granularity_then_check_ms": {lbl: round(v * 1e3, 3) for lbl, v in gtrace}}}
    # a sample of the same queries, one dpo_bfs call each on its own graph
    one = dpo.Options(threshold=32, coarsen=1, steps_per_replay=16, child_block=128)
    sub = qs[::8]
    dgs = {g: dpo.DeviceGraph.from_host(graphs[g]) for g, _, _ in sub}
    bufs = {g: (torch.empty(graphs[g].n, dtype=torch.int32, device="cuda"),
                dpo.alloc_workspace(dgs[g], one)) for g in dgs}
    for g, s, b in sub:  # warm-up: instantiates each graph's replay
        dpo.dpo_bfs(dgs[g], int(s), one, *bufs[g])
    torch.cuda.synchronize()
    t1 = time.perf_counter()
    for g, s, b in sub:
        dpo.dpo_bfs(dgs[g], int(s), one, *bufs[g])
    torch.cuda.synchronize()
    per = (time.perf_counter() - t1) / len(sub)
    res["one_by_one_traversals_per_s"] = round(1.0 / per, 1)
    del dgs, bufs
    # untuned: every bucket at the base point (same replay length)
    base.steps_per_replay = st["levels"] + 1
    qs0 = [(g, s, 0) for g, s, _ in qs]
    dpo.dpo_bfs_batch(da, qs0, [base], out, ws)
    torch.cuda.synchronize()
    ev0.record()
    dpo.dpo_bfs_batch(da, qs0, [base], out, ws)
    ev1.record()
    torch.cuda.synchronize()
    res["untuned_ms_per_batch"] = round(ev0.elapsed_time(ev1), 3)
    res["untuned"] = base.label()
    res["tuned_speedup_vs_untuned"] = round(res["untuned_ms_per_batch"] / res["ms_per_batch"], 3)
    log(f"[batch] {res}")
    if not args.no_cpu:
        res["cpu_baseline"] = cpu_batch(graphs, queries)
    if full_line:
        return {"metric": "batched BFS traversals/s (512 over 64 R-MAT graphs, scales 10-18)",
                "value": res["traversals_per_s"], "unit": "traversals/s", "n_gpus": 1,
                "steps": steps, "warmup": warm, "ms_per_step": res["ms_per_batch"],
                "higher_is_better": True, "scaling": "weak", "vs_baseline": None, "dtype": "int32",
                "data": "synthetic", "config": {"workload": "batched BFS, 64 R-MAT graphs, 8 sources each"},
                "batched": res}
    return res


def host_threads():
    """Oracle pool size: the cores this process may use, at most 16 (one GPU's
    share of the host)."""
    return max(1, min(16, len(os.sched_getaffinity(0))))


def cpu_batch(graphs, queries, min_seconds=5.0):
    """Oracle BFS of the batch's queries on a pool of host threads, all 512
    in order, repeated until at least min_seconds."""
    import oracle
    from concurrent.futures import ThreadPoolExecutor
    nthreads = host_threads()
    done, rounds = 0, 0
    t0 = time.perf_counter()
    with ThreadPoolExecutor(nthreads) as ex:
        while True:
            list(ex.map(lambda q: oracle.bfs(graphs[q[0]], q[1]), queries))
            done += len(queries)
            rounds += 1
            dt = time.perf_counter() - t0
            if dt >= min_seconds:
                break
    return {"value": round(done / dt, 1), "unit": "traversals/s", "cores": nthreads,
            "kind": "oracle", "host": host_cpu(),
            "sample": f"all {len(queries)} queries x {rounds} round(s), queue BFS, "
                      f"{nthreads} threads, {dt:.2f} s"}


def cpu_serve(graphs, pools, lam, nq, serve_seconds):
    """The oracle as a server: a pool of host threads takes the queries of the
    GPU run's Poisson trace for offered rate lam (same seed, kinds, graphs and
    sources) at their arrival times; latency = completion - arrival.  Only the
    first nq arrivals are served (a bounded sample: the pool saturates far
    below the GPU's rates, so the backlog and the latencies grow with it)."""
    import threading
    import oracle
    from concurrent.futures import ThreadPoolExecutor
    rng = np.random.default_rng(7 + lam)
    total = max(50, min(int(lam * serve_seconds), 25000))
    arr = np.cumsum(rng.exponential(1.0 / lam, size=total))
    kinds = np.where(rng.random(total) < 0.7, "bfs", "sssp")
    gsel = rng.integers(0, len(graphs), size=total)
    ssel = rng.integers(0, 64, size=total)
    nthreads = host_threads()
    lat = np.full(nq, np.nan)
    lock = threading.Lock()

    def job(i, t_start):
        g, s = int(gsel[i]), int(pools[gsel[i]][ssel[i]])
        if kinds[i] == "bfs":
            oracle.bfs(graphs[g], s)
        else:
            oracle.dijkstra(graphs[g], s)
        with lock:
            lat[i] = time.perf_counter() - t_start - arr[i]

    t_start = time.perf_counter()
    with ThreadPoolExecutor(nthreads) as ex:
        for i in range(nq):
            wait = arr[i] - (time.perf_counter() - t_start)
            if wait > 0:
                time.sleep(wait)
            ex.submit(job, i, t_start)
    wall = time.perf_counter() - t_start
    return {"value": round(nq / wall, 1), "unit": "q/s", "cores": nthreads, "kind": "oracle",
            "host": host_cpu(), "offered_qps": lam,
            "p50_ms": round(float(np.percentile(lat, 50)) * 1e3, 3),
            "p99_ms": round(float(np.percentile(lat, 99)) * 1e3, 3),
            "sample": f"first {nq} arrivals of the offered-{lam} q/s trace (70/30 queue BFS / "
                      f"binary-heap Dijkstra), {nthreads} threads, {wall:.2f} s"}


# ---------------------------------------------------------------- serving
def bench_serve(args, dpo, torch, full_line=False):
    """Poisson stream of BFS/SSSP queries (70/30) against 8 resident R-MAT
    graphs (scales 14..20 and a second scale-20 graph, edgefactor 16, weights
    U[1,255]); two continuous-batching engines on two streams."""
    from paper_2201_02789_amd import graphgen as gg
    t0 = time.time()
    scales = [14, 15, 16, 17, 18, 19, 20, 20]
    graphs = [gg.add_weights(gg.rmat(sc, 16, 3000 + i, perm_seed=9000 + i), 5000 + i)
              for i, sc in enumerate(scales)]
    arena, vbase = gg.pack_arena(graphs)
    da = dpo.DeviceArena(arena, vbase)
    pools = [gg.sample_sources(g, 64, 6000 + i) for i, g in enumerate(graphs)]
    log(f"[serve] graphs ready, arena n={arena.n} m={arena.m} ({time.time() - t0:.1f}s)")
    def opts(kind):
        T = args.threshold if args.threshold is not None else SERVE_T[kind]
        return [dpo.Options(threshold=T, coarsen=1, agg=dpo.DPO_AGG_MULTIBLOCK, agg_blocks=4,
                            steps_per_replay=4, child_block=SERVE_CB[kind], dyn_share=SERVE_DYN[kind],
                            claim_hint=args.claim_hint or 0)]
    s_bfs, s_sssp = torch.cuda.Stream(), torch.cuda.Stream()
    max_slots = 1 << 24
    engines = {"bfs": dpo.Engine(da, "bfs", opts("bfs"), max_queries=256, max_slots=max_slots,
                                 stream=s_bfs),
               "sssp": dpo.Engine(da, "sssp", opts("sssp"), max_queries=256, max_slots=max_slots,
                                  stream=s_sssp)}
    sinks = [torch.empty(g.n, dtype=torch.int32, device="cuda") for g in graphs]
    rates = [int(x) for x in args.rates.split(",")]
    results = []
    for lam in rates:
        rng = np.random.default_rng(7 + lam)
        nq = max(50, min(int(lam * args.serve_seconds), 25000))
        arr = np.cumsum(rng.exponential(1.0 / lam, size=nq))
        kinds = np.where(rng.random(nq) < 0.7, "bfs", "sssp")
        gsel = rng.integers(0, len(graphs), size=nq)
        ssel = rng.integers(0, 64, size=nq)
        tick = {"bfs": {}, "sssp": {}}
        lat = np.full(nq, np.nan)
        nxt = 0
        done = 0
        t_start = time.perf_counter()
        while done < nq:
            now = time.perf_counter() - t_start
            while nxt < nq and arr[nxt] <= now:
                k = kinds[nxt]
                g = int(gsel[nxt])
                t = engines[k].submit(g, int(pools[g][ssel[nxt]]), sinks[g])
                tick[k][t] = nxt
                nxt += 1
            for k, e in engines.items():
                e.step()
                for t in e.poll():
                    i = tick[k].pop(t)
                    lat[i] = time.perf_counter() - t_start - arr[i]
                    done += 1
            if time.perf_counter() - t_start > 60:
                break
        wall = time.perf_counter() - t_start
        ok = ~np.isnan(lat)
        r = {"offered_qps": lam, "queries": int(ok.sum()),
             "achieved_qps": round(float(ok.sum()) / max(wall, arr[-1]), 1),
             "p50_ms": round(float(np.percentile(lat[ok], 50)) * 1e3, 3),
             "p99_ms": round(float(np.percentile(lat[ok], 99)) * 1e3, 3)}
        results.append(r)
        log(f"[serve] {r}")
    for e in engines.values():
        e.close()
    cpu = None
    if not args.no_cpu:
        cpu = cpu_serve(graphs, pools, rates[0], args.cpu_serve_queries, args.serve_seconds)
        log(f"[serve] oracle pool: {cpu}")
    if full_line:
        best = max(results, key=lambda r: r["achieved_qps"])
        return {"metric": "serving q/s and p99 latency (BFS/SSSP 70/30, 8 resident R-MAT graphs)",
                "value": best["achieved_qps"], "unit": "q/s", "n_gpus": 1, "steps": len(rates),
                "warmup": 0, "ms_per_step": None, "higher_is_better": True, "scaling": "weak",
                "vs_baseline": None, "dtype": "int32", "data": "synthetic",
                "config": {"workload": "Poisson BFS/SSSP 70/30, scales 14..20 + second 20"},
                "serving": results, "cpu_baseline": cpu}
    return {"rates": results, "graphs": "R-MAT scales 14..20 + second 20, ef 16",
            "mix": "70% BFS / 30% SSSP", "steps_per_replay": 4, "max_slots": max_slots,
            "serve_seconds": args.serve_seconds,
            "thresholds": {k: opts(k)[0].threshold for k in engines}, "cpu_baseline": cpu}


# ---------------------------------------------------------------- low nesting
def bench_road(args, dpo, torch):
    """Low-nesting control (the paper's road-graph experiment, Sec. VIII-D):
    a perturbed 514 x 514 grid (264,196 vertices, average degree ~3, maximum
    8) standing in for USA-road-d.NY.  Flat vs nested with the threshold above
    the largest degree (every child serialised, no launch) vs nested T=0."""
    from paper_2201_02789_amd import graphgen as gg
    g = gg.road_like(514, 514, 3)
    srcs = gg.sample_sources(g, 4, 1)
    dg = dpo.DeviceGraph.from_host(g)
    deg = g.degrees()
    out = torch.empty(g.n, dtype=torch.int32, device="cuda")
    res = {"graph": {"n": g.n, "m": g.m, "avg_degree": round(float(deg.mean()), 3),
                     "max_degree": int(deg.max())}}
    cfgs = {"flat": dpo.Options.flat(),
            "nested_T_above_max": dpo.Options(threshold=int(deg.max()) + 1, coarsen=1),
            # each serialised child in its parent's lane, as in the paper
            "nested_T_above_max_lane": dpo.Options(threshold=int(deg.max()) + 1, coarsen=1,
                                                   serial_wave=0),
            "nested_T0_4block": dpo.Options(threshold=0, coarsen=1),
            "naive": dpo.Options.naive()}
    for name, o in cfgs.items():
        o.steps_per_replay = 64
        ws = dpo.alloc_workspace(dg, o)
        dpo.dpo_bfs(dg, int(srcs[0]), o, out, ws)
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        for s in srcs:
            dpo.dpo_bfs(dg, int(s), o, out, ws)
        torch.cuda.synchronize()
        ms = (time.perf_counter() - t0) / len(srcs) * 1e3
        res[name] = {"ms_per_bfs": round(ms, 3), "options": o.label()}
        log(f"[road] {name}: {ms:.3f} ms")
    return {"workload": "road-like grid BFS (low nested parallelism)", **res}


# ---------------------------------------------------------------- breakdown
REALTIME_MHZ = 100.0  # the constant-rate clock the timed kernels stamp


def phase_split(rows, mhz=REALTIME_MHZ):
    """Execution-time breakdown of one timed traversal (Sec. VIII-B).

    rows: uint64 [levels, 4 kernels, workgroups, 8] as written by
    dpo_traverse_timed.  Per level and kernel, the kernel's span (first
    workgroup entry to last exit) is split among the phases in proportion to
    the cycles its waves spent in each; the gap from the parent kernel's end to
    the child kernel's start is launch time too (the aggregated grids start
    there); every other gap between kernels (including empty kernels, which
    write no rows) is reported as "gaps".  Returns (totals in us, per-level
    list of (level, {phase: us}), child-kernel imbalance = time-weighted
    busiest-workgroup span / mean workgroup span)."""
    phases = ("parent", "aggregation", "launch", "disaggregation", "child")
    tot = dict.fromkeys(phases + ("gaps",), 0.0)
    per_level, prev_end = [], None
    imb_num = imb_den = 0.0
    for L in range(rows.shape[0]):
        lv = dict.fromkeys(phases + ("gaps",), 0.0)
        kern = {}
        for k in range(rows.shape[1]):
            r = rows[L, k]
            r = r[r[:, 1] != 0]
            if r.size == 0:
                continue
            t0, t1 = int(r[:, 0].min()), int(r[:, 1].max())
            cyc = r[:, 2:7].astype(np.float64).sum(axis=0)
            span = (t1 - t0) / mhz
            share = cyc / cyc.sum() if cyc.sum() > 0 else np.zeros(5)
            for p, x in zip(phases, share):
                lv[p] += span * x
            kern[k] = (t0, t1)
            if k == 1:
                wg = (r[:, 1] - r[:, 0]).astype(np.float64) / mhz
                imb_num += span * wg.max() / max(wg.mean(), 1e-9)
                imb_den += span
        if not kern:
            continue
        order = sorted(kern.items(), key=lambda kv: kv[1][0])
        if prev_end is not None:
            lv["gaps"] += max(0, order[0][1][0] - prev_end) / mhz
        for (ka, (a0, a1)), (kb, (b0, b1)) in zip(order, order[1:]):
            gap = max(0, b0 - a1) / mhz
            lv["launch" if (ka, kb) == (0, 1) else "gaps"] += gap
        prev_end = order[-1][1][1]
        per_level.append((L, lv))
        for p in tot:
            tot[p] += lv[p]
    return tot, per_level, (imb_num / imb_den if imb_den else 1.0)


def child_skew(rows, mhz=REALTIME_MHZ):
    """Where the child kernel's imbalance comes from, time-weighted over the
    levels: spread of workgroup entries and exits (us) and the ratio of the
    slowest to the fastest XCD's mean workgroup span (workgroup % 8)."""
    acc = {"start_spread_us": 0.0, "end_spread_us": 0.0, "xcd_span_ratio": 0.0}
    wsum = 0.0
    for L in range(rows.shape[0]):
        r = rows[L, 1]
        idx = np.flatnonzero(r[:, 1] != 0)
        if idx.size < 8:
            continue
        r = r[idx]
        t0, t1 = r[:, 0].astype(np.float64), r[:, 1].astype(np.float64)
        span = (t1.max() - t0.min()) / mhz
        wg = (t1 - t0) / mhz
        per = [wg[idx % 8 == x].mean() for x in range(8) if np.any(idx % 8 == x)]
        acc["start_spread_us"] += span * (t0.max() - t0.min()) / mhz
        acc["end_spread_us"] += span * (t1.max() - t1.min()) / mhz
        acc["xcd_span_ratio"] += span * max(per) / max(min(per), 1e-9)
        wsum += span
    return {k: round(v / wsum, 3) if wsum else None for k, v in acc.items()}


def level_table(rows, mhz=REALTIME_MHZ):
    """Per level of one timed traversal: each kernel's span (first entry to last
    exit, us) and, for the child kernel, the mean and the largest workgroup span
    and the spread of workgroup exits (kernels: parent, child, SSSP's
    thresholded children, harvest)."""
    out = []
    for L in range(rows.shape[0]):
        row = {"level": L}
        for k, name in ((0, "parent"), (1, "child"), (2, "serial"), (3, "harvest")):
            r = rows[L, k]
            r = r[r[:, 1] != 0]
            if r.size == 0:
                continue
            t0, t1 = r[:, 0].astype(np.float64), r[:, 1].astype(np.float64)
            row[name + "_us"] = round((t1.max() - t0.min()) / mhz, 1)
            if k == 1:
                wg = (t1 - t0) / mhz
                row["child_wg_mean_us"] = round(float(wg.mean()), 1)
                row["child_wg_max_us"] = round(float(wg.max()), 1)
                row["child_exit_spread_us"] = round(float(t1.max() - t1.min()) / mhz, 1)
                row["child_workgroups"] = int(r.shape[0])
        if len(row) > 1:
            out.append(row)
    return out


def bench_breakdown(args, dpo, torch):
    """Sec. VIII-B: parent / aggregation / launch / disaggregation / child time
    per traversal at CF 1, 2, 4, 8 and a few thresholds, from the timed
    instantiations of the level kernels; writes profiles/<workload>_breakdown.md."""
    name = args.workload if args.workload in ("bfs22", "sssp21") else "bfs22"
    wl = Workload(name)
    dg = dpo.DeviceGraph.from_host(wl.g)
    tuned = TUNED[name]
    Ts = (0, 16, 64) if wl.kind == "bfs" else (0, 128, 512)
    rs, _ = reached_stats(dpo, torch, wl, dg, dpo.Options(**tuned))
    steps = max(r[2]["levels"] for r in rs) + 1
    timing = torch.zeros(dpo.TIMING_BYTES // 8, dtype=torch.int64, device="cuda")
    out = torch.empty(dg.n, dtype=torch.int32, device="cuda")
    stream = torch.cuda.current_stream()
    phases = ("parent", "aggregation", "launch", "disaggregation", "child", "gaps")
    results = []
    levels_of = None  # per-level table of the tuned options' first source
    for CF in (1, 2, 4, 8):
        for T in Ts:
            o = dpo.Options(**{**tuned, "threshold": T, "coarsen": CF, "steps_per_replay": steps})
            pc, _ = measure(dpo, torch, wl, dg, o, 2, 1)
            ws = dpo.alloc_workspace(dg, o)
            acc = dict.fromkeys(phases, 0.0)
            longest, imb, timed_ms, skews = None, [], [], []
            for s in wl.sources:
                e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
                e0.record(stream)
                dpo.dpo_traverse_timed(wl.kind, dg, int(s), o, out, ws, timing)
                e1.record(stream)
                torch.cuda.synchronize()
                timed_ms.append(e0.elapsed_time(e1))
                rows = timing.cpu().numpy().view(np.uint64).reshape(64, 4, 4096, 8)
                tot, per_level, ib = phase_split(rows)
                skews.append(child_skew(rows))
                grids = [int((rows[:, k, :, 1] != 0).sum(axis=1).max()) for k in range(4)]
                if levels_of is None and T == tuned["threshold"] and CF == tuned["coarsen"]:
                    levels_of = (int(s), level_table(rows))
                for p in phases:
                    acc[p] += tot[p] / len(wl.sources)
                imb.append(ib)
                big = max(per_level, key=lambda x: sum(x[1].values()))
                if longest is None or sum(big[1].values()) > sum(longest[1].values()):
                    longest = big
            r = {"threshold": T, "coarsen": CF, "options": o.label(),
                 "product_ms_per_traversal": round(float(pc.mean()), 4),
                 "timed_ms_per_traversal": round(float(np.mean(timed_ms)), 4),
                 "us_per_traversal": {p: round(v, 1) for p, v in acc.items()},
                 "child_imbalance": round(float(np.mean(imb)), 3),
                 "workgroups_with_rows": grids,
                 "child_skew": {k: round(float(np.mean([x[k] for x in skews if x[k] is not None])), 3)
                                for k in skews[0]},
                 "longest_level": {"level": longest[0],
                                   "us": {p: round(v, 1) for p, v in longest[1].items()}}}
            results.append(r)
            log(f"[breakdown] {o.label()}: product {r['product_ms_per_traversal']} ms, "
                f"timed {r['timed_ms_per_traversal']} ms, {r['us_per_traversal']}")
            del ws
    cmd = "python3 bench.py " + " ".join(sys.argv[1:])
    md = [f"# {name}: execution-time breakdown (parent / aggregation / launch / disaggregation / child)",
          "", f"Workload: {wl.desc}; child block {tuned.get('child_block', 256)}, 4-block "
          f"aggregation, {steps} level steps per replay, {len(wl.sources)} source(s).", "",
          f"Command (MI355X, repository root): `{cmd}`", "",
          "Method: the timed instantiations of the level kernels (dpo_traverse_timed: the same "
          "kernels as the product ones on the same grids (or, where a timed kernel needs more "
          "registers, the grid resident at its own occupancy: see the workgroup counts below), "
          "with a shader-clock stamp at each phase "
          "boundary after the wave's outstanding memory operations) give each workgroup's "
          "cycles per phase and its entry / exit on a 100 MHz clock.  Each kernel's span is "
          "split among the phases in proportion to the cycles; the gap from the parent "
          "kernel's end to the child kernel's start is launch time (the aggregated grids "
          "start there); other gaps between kernels (including child kernels of levels with "
          "no launch, which stamp nothing) are gaps.  Phases: parent = frontier reads, "
          "threshold decisions and the thresholded children run in the parent kernel(s); "
          "aggregation = scans, launch records and group counters; launch = publishing grids "
          "and reading the level's published grids, plus the parent-to-child gap; "
          "disaggregation = finding each wave's first record and loading record windows; "
          "child = the coarsening loop and the child body (also the harvest kernel, which "
          "turns a level's found vertices into the next frontier, with their levels for "
          "BFS).  The stamps wait for memory, so "
          "the timed traversal is slower than the product one (both columns shown); the "
          "phase split is of the timed run.", "",
          "## Mean per traversal (us)", "",
          "| T | CF | product ms | timed ms | parent | aggregation | launch | disaggregation | child | gaps | child imbalance |",
          "|---|---|---|---|---|---|---|---|---|---|---|"]
    for r in results:
        u = r["us_per_traversal"]
        md.append(f"| {r['threshold']} | {r['coarsen']} | {r['product_ms_per_traversal']:.3f} | "
                  f"{r['timed_ms_per_traversal']:.3f} | " +
                  " | ".join(f"{u[p]:.1f}" for p in phases) + f" | {r['child_imbalance']:.2f} |")
    md += ["", "child imbalance: time-weighted ratio of the busiest child workgroup's span to the "
           "mean workgroup span.", "", "## Child kernel skew (time-weighted over levels)", "",
           "| T | CF | entry spread us | exit spread us | slowest / fastest XCD mean span |",
           "|---|---|---|---|---|"]
    md += [f"| {r['threshold']} | {r['coarsen']} | {r['child_skew']['start_spread_us']} | "
           f"{r['child_skew']['end_spread_us']} | {r['child_skew']['xcd_span_ratio']} |" for r in results]
    md += ["", "Workgroups that stamped rows (largest level; parent, child, thresholded-children "
           "and harvest kernel): " + "; ".join(f"T{r['threshold']} CF{r['coarsen']}: {r['workgroups_with_rows']}"
                                               for r in results[:3]) + "."]
    if levels_of is not None:
        src, table = levels_of
        cols = ["level", "parent_us", "child_us"] + (["serial_us"] if wl.kind == "sssp" else []) + [
                "harvest_us", "child_wg_mean_us", "child_wg_max_us",
                "child_exit_spread_us", "child_workgroups"]
        md += ["", f"## Per level, tuned options ({tuned['threshold']}, CF {tuned['coarsen']}), "
                   f"source {src}", "", "| " + " | ".join(cols) + " |", "|" + "---|" * len(cols)]
        md += ["| " + " | ".join(str(r.get(c, "")) for c in cols) + " |" for r in table]
    md += ["", "## Longest level of any source (us)", "",
           "| T | CF | level | parent | aggregation | launch | disaggregation | child | gaps |",
           "|---|---|---|---|---|---|---|---|---|"]
    for r in results:
        u = r["longest_level"]["us"]
        md.append(f"| {r['threshold']} | {r['coarsen']} | {r['longest_level']['level']} | " +
                  " | ".join(f"{u[p]:.1f}" for p in phases) + " |")
    outp = os.path.join(ROOT, "profiles", f"{name}_breakdown.md")
    with open(outp, "w") as f:
        f.write("\n".join(md) + "\n")
    log(f"[breakdown] wrote {outp}")
    return {"workload": wl.desc, "breakdown": results}


def sweep(dpo, torch, wl, dg, cmd):
    """Sweep of T x CF x granularity (and the aggregation threshold), plus flat
    and naive, on the workload's graph and sources, at its tuned child block
    size (and SSSP's one-copy threshold).  Prints one JSON line per point and
    writes profiles/<workload>_sweep.md."""
    import itertools
    import platform
    tuned = TUNED[wl.name]
    fixed = {k: tuned[k] for k in ("child_block", "split_min", "dyn_share") if k in tuned}
    rs, _ = reached_stats(dpo, torch, wl, dg, dpo.Options(**{**tuned, "steps_per_replay": 0}))
    edges = float(sum(r[0] for r in rs) / 2)
    steps = max(r[2]["levels"] for r in rs) + 1
    grans = [(1, 4, "wave"), (2, 4, "block"), (3, 4, "4-block"), (3, 16, "16-block"), (4, 4, "grid")]
    grid = [("flat", "-", "-", dpo.Options.flat()),
            ("naive", 0, 1, dpo.Options.naive(child_block=fixed.get("child_block", 256)))]
    for T, CF, (agg, k, gname) in itertools.product([0, 8, 16, 32, 64, 128, 512, 2048],
                                                    [1, 2, 4, 8], grans):
        grid.append((gname, T, CF, dpo.Options(threshold=T, coarsen=CF, agg=agg, agg_blocks=k,
                                               **fixed)))
    for T, (agg, gname), at in itertools.product([8, 32], [(1, "wave"), (2, "block")], [8, 32]):
        grid.append((f"{gname} A{at}", T, 1, dpo.Options(threshold=T, coarsen=1, agg=agg,
                                                         agg_threshold=at, **fixed)))
    rows = []
    for gname, T, CF, o in grid:
        o.steps_per_replay = steps
        pc, _ = measure(dpo, torch, wl, dg, o, 2, 1)
        g = 2 * edges / (pc.sum() * 1e-3) / 1e9
        rows.append((g, gname, T, CF, o.label(), float(pc.mean())))
        print(json.dumps({"options": o.label(), "gteps": round(g, 3),
                          "ms_per_traversal": round(float(pc.mean()), 4)}), flush=True)
    nested = [r for r in rows if r[1] not in ("flat", "naive")]
    best = max(nested)
    md = [f"# {wl.name}: threshold x coarsening x granularity sweep", "",
          f"Workload: {wl.desc} (n = {wl.g.n}, m = {wl.g.m}).  Child block {fixed.get('child_block', 256)}"
          f", dyn_share {fixed.get('dyn_share', 0)}"
          f"{', one visited copy below ' + str(fixed['split_min']) + ' frontier entries' if 'split_min' in fixed else ''}; "
          f"{steps} level steps per replay; each point 1 warm-up + 2 timed passes over the "
          f"{len(wl.sources)} source(s), hipEvents around each call.  GTEPS = undirected edges "
          f"in the reached components / time.", "",
          f"Command (MI355X, repository root): `{cmd}`", "",
          f"Best nested point: **{best[4]}, {best[0]:.2f} GTEPS** ({best[5]:.3f} ms per traversal); "
          f"flat {rows[0][0]:.3f}, naive {rows[1][0]:.3f} GTEPS.", "",
          "## Best point per granularity", "", "| granularity | best options | GTEPS |", "|---|---|---|"]
    for gname in [g[2] for g in grans] + ["wave A8", "wave A32", "block A8", "block A32"]:
        cand = [r for r in nested if r[1] == gname]
        if cand:
            b = max(cand)
            md.append(f"| {gname} | {b[4]} | {b[0]:.2f} |")
    md += ["", "## Best point per coarsening factor", "", "| CF | best options | GTEPS |", "|---|---|---|"]
    for CF in (1, 2, 4, 8):
        b = max(r for r in nested if r[3] == CF)
        md.append(f"| {CF} | {b[4]} | {b[0]:.2f} |")
    md += ["", "## Best point per threshold", "", "| T | best options | GTEPS |", "|---|---|---|"]
    for T in (0, 8, 16, 32, 64, 128, 512, 2048):
        b = max(r for r in nested if r[2] == T)
        md.append(f"| {T} | {b[4]} | {b[0]:.2f} |")
    md += ["", "## Every point", "", "| options | GTEPS | ms / traversal |", "|---|---|---|"]
    md += [f"| {r[4]} | {r[0]:.3f} | {r[5]:.4f} |" for r in sorted(rows, reverse=True)]
    out = os.path.join(ROOT, "profiles", f"{wl.name}_sweep.md")
    with open(out, "w") as f:
        f.write("\n".join(md) + "\n")
    log(f"[sweep] wrote {out} (host {platform.node()})")


if __name__ == "__main__":
    main()
