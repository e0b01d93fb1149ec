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
    p.add_argument("--serve-seconds", type=float, default=0.5)
    p.add_argument("--rates", default="1000,2000,5000,10000,20000,50000")
    p.add_argument("--threshold", type=int, default=None)
    p.add_argument("--coarsen", type=int, default=None)
    p.add_argument("--split-min", type=int, default=None,
                   help="frontier size from which a level uses two visited copies")
    p.add_argument("--agg", default=None, help="none|wave|block|<k>-block")
    p.add_argument("--sweep", action="store_true",
                   help="threshold x coarsening x granularity sweep of the workload instead")
    p.add_argument("--no-cpu", action="store_true")
    p.add_argument("--no-baselines", action="store_true")
    p.add_argument("--cpu-seconds", type=float, default=10.0,
                   help="minimum oracle time of the cpu_baseline sample")
    p.add_argument("--calibrate-copy", action="store_true",
                   help="only run a plain 512 MiB device copy (counter calibration)")
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
TUNED = {"bfs22": dict(threshold=64, coarsen=1, agg=3, agg_blocks=4, child_block=128),
         "er22": dict(threshold=8, coarsen=1, agg=3, agg_blocks=4, child_block=128),
         "bfs25": dict(threshold=64, coarsen=1, agg=3, agg_blocks=4, child_block=128),
         "bfs12": dict(threshold=32, coarsen=8, agg=3, agg_blocks=4),
         "sssp21": dict(threshold=512, coarsen=1, agg=3, agg_blocks=4, split_min=262144,
                        child_block=128)}


SERVE_T = {"bfs": 64, "sssp": 256}  # thresholds of the serving engines


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


def certify(g, kind, src, out):
    """Edge certificates of one result (no oracle): BFS (i) level[s] = 0,
    (ii) every reached v != s has an in-neighbour one level lower, (iii) every
    edge from a reached u reaches v with level[v] <= level[u] + 1; SSSP the same
    with dist and w (>= 1).  Together they fix levels / distances exactly."""
    rp = np.asarray(g.row_ptr, dtype=np.int64)
    u = np.repeat(np.arange(g.n, dtype=np.int32), np.diff(rp))
    v = np.asarray(g.col_idx, dtype=np.int32)
    if kind == "bfs":
        x = out.astype(np.int64)
        unreached, step = -1, 1
    else:
        x = out.astype(np.int64) & 0xFFFFFFFF
        unreached, step = 0xFFFFFFFF, np.asarray(g.weights, dtype=np.int64)
    if x[src] != 0:
        return False
    xu, xv = x[u], x[v]
    ru = xu != unreached
    bound = xu + step
    if np.any(ru & ((xv == unreached) | (xv > bound))):
        return False
    tight = np.zeros(g.n, dtype=bool)
    tight[v[ru & (xv == bound)]] = True
    need = x != unreached
    need[src] = False
    return bool(np.all(tight[need]))


def reached_stats(dpo, torch, wl, dg, opts):
    """(m_r, n_r, stats) per source from one untimed run with counters, and
    whether the first source's result passes its edge certificates."""
    out = torch.empty(dg.n, dtype=torch.int32, device="cuda")
    ws = dpo.alloc_workspace(dg, opts)
    deg = np.diff(wl.g.row_ptr).astype(np.int64)
    res, ok = [], None
    for s in wl.sources:
        if wl.kind == "bfs":
            st = dpo.dpo_bfs(dg, int(s), opts, out, ws, stats=True)
            host = out.cpu().numpy()
            reached = host >= 0
        else:
            st = dpo.dpo_sssp(dg, int(s), opts, out, ws, stats=True)
            host = out.cpu().numpy()
            reached = dpo.as_uint32(out) != 0xFFFFFFFF
        if ok is None:
            ok = certify(wl.g, wl.kind, int(s), host)
        res.append((int(deg[reached].sum()), int(reached.sum()), st))
    return res, ok


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


def measured_traffic(workload, options_label):
    """HBM bytes per launch from the committed counter summary
    (profiles/<workload>_traffic.json: FETCH_SIZE and WRITE_SIZE per traversal,
    scaled by a plain copy of known size), or None when the kernels changed
    since the counters were taken or the options differ."""
    path = os.path.join(ROOT, "profiles", f"{workload}_traffic.json")
    if not os.path.exists(path):
        return None
    with open(path) as f:
        t = json.load(f)
    if t.get("kernel_sources_sha256") != kernel_sources_sha() or t.get("options") != options_label:
        return None
    return t["hbm_bytes_per_launch"]


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


def summarize_profiles(args, d):
    """Level-step kernel time from a kernel trace and HBM bytes from FETCH_SIZE
    / WRITE_SIZE counter runs, each counter scaled by what it reads for a plain
    copy of known size."""
    with open(os.path.join(d, "trace", "out.json")) as f:
        line = json.loads([ln for ln in f if ln.startswith("{")][-1])
    label, launches_per = line["config"]["options"], line["roofline"]["launches_per_traversal"]
    step = ("parent_kernel", "child_kernel")

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
    top = sorted(stats.items(), key=lambda kv: -kv[1][1])[:8]
    md = [f"# {args.workload}: kernel time and HBM traffic ({label})", "",
          "Commands (MI355X, from the repository root, after `export TMPDIR=/tmp`):", "",
          "```"] + [ln.rstrip() for ln in open(os.path.join(d, "commands.txt"))] + ["```", "",
          "## Kernel trace (`rocprofv3 --kernel-trace --stats`)", "",
          "| kernel | calls | total ms | mean us |", "|---|---|---|---|"]
    md += [f"| {n} | {c} | {t / 1e6:.3f} | {t / c / 1e3:.2f} |" for n, (c, t) in top]
    md += ["", f"Traversals traced: {traversals}; level-step launches per traversal "
               f"{launches_per:.4g} (levels + 1).",
           f"Level step (parent_kernel + child_kernel"
           f"{'; the parent kernel runs as two kernels, pass 1 before and pass 2 after the child kernel' if args.workload.startswith('sssp') else ''}"
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
    a = agg_of(args.agg) if overrides else None
    if a:
        tuned["agg"], tuned["agg_blocks"] = a
    opts = dpo.Options(**tuned)

    if args.sweep:
        sweep(dpo, torch, wl, dg)
        return None

    # untimed run with counters: edges reached and level count per source
    rs, certified = reached_stats(dpo, torch, wl, dg, opts)
    if not certified:
        log(f"[bench] ERROR: the result of source {int(wl.sources[0])} fails its edge certificates")
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
                           f"{' + parent_kernel pass 2' if wl.kind == 'sssp' else ''} "
                           f"<{wl.kind.upper()}, {opts.label()}>"),
                "launches_per_traversal": float(launches.mean()),
                "mean_launch_us": round(float(mean_call_ms.sum() / launches.sum() * 1e3), 2),
                "algorithmic_bytes_per_launch": round(float(bytes_call.sum() / launches.sum()))}

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
                   "verified": (f"edge certificates of source {int(wl.sources[0])}'s result "
                                f"({'pass' if certified else 'FAIL'}), untimed run"),
                   # edges the traversal actually relaxes per reached directed edge
                   # (1 for BFS; above 1 for the frontier Bellman-Ford of SSSP)
                   "work_efficiency": round(float(np.mean(
                       [(r[2]["edges_serial"] + r[2]["edges_child"]) / max(r[0], 1) for r in rs])), 3)},
        "roofline": roofline,
        "baselines": baselines,
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
        sp = workload_line(args, dpo, torch, "sssp21", 3, 1, False, True, overrides=False)
        del sp["_graph"]
        line["sssp"] = {k: sp[k] for k in ("value", "unit", "ms_per_step", "dtype", "config",
                                             "roofline", "baselines", "speedup_vs_flat",
                                             "speedup_vs_naive")}
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
    tuned, traces = autotune.tune("bfs", da, graphs, queries, bucket, 3, base, max_runs=8, log=log)
    qs = [(g, s, bucket[g]) for g, s in queries]
    tot, slot0 = dpo.dpo_batch_slots(da, qs)
    out = torch.empty(tot, dtype=torch.int32, device="cuda")
    ws = torch.empty(dpo.dpo_batch_workspace_bytes(da, qs, tuned[0]), dtype=torch.uint8,
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
           "tuning_runs": [len(t) for t in traces]}
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


def cpu_batch(graphs, queries, sample=64):
    """Oracle BFS of a sample of the batch's queries on a pool of host threads."""
    import oracle
    from concurrent.futures import ThreadPoolExecutor
    nthreads = os.cpu_count() or 1
    sub = queries[::max(1, len(queries) // sample)]
    t0 = time.perf_counter()
    with ThreadPoolExecutor(nthreads) as ex:
        list(ex.map(lambda q: oracle.bfs(graphs[q[0]], q[1]), sub))
    dt = time.perf_counter() - t0
    return {"value": round(len(sub) / dt, 1), "unit": "traversals/s", "cores": nthreads,
            "kind": "oracle", "sample": f"{len(sub)} of {len(queries)} queries, queue BFS, "
                                        f"{nthreads} threads, {dt:.2f} s"}


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
                            steps_per_replay=4, child_block=128)]
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
    if full_line:
        best = max(results, key=lambda r: r["achieved_qps"])
        return {"metric": "serving q/s and p99 latency (BFS/SSSP 70/30, 8 resident R-MAT graphs)",
                "value": best["achieved_qps"], "unit": "q/s", "n_gpus": 1, "steps": len(rates),
                "warmup": 0, "ms_per_step": None, "higher_is_better": True, "scaling": "weak",
                "vs_baseline": None, "dtype": "int32", "data": "synthetic",
                "config": {"workload": "Poisson BFS/SSSP 70/30, scales 14..20 + second 20"},
                "serving": results}
    return {"rates": results, "graphs": "R-MAT scales 14..20 + second 20, ef 16",
            "mix": "70% BFS / 30% SSSP", "steps_per_replay": 4, "max_slots": max_slots,
            "thresholds": {k: opts(k)[0].threshold for k in engines}}


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


def sweep(dpo, torch, wl, dg):
    """Sweep of T x CF x granularity (and the aggregation threshold), plus flat
    and naive, on the workload's graph and sources (JSON lines)."""
    import itertools
    rs, _ = reached_stats(dpo, torch, wl, dg, dpo.Options())
    edges = float(sum(r[0] for r in rs) / 2)
    steps = max(r[2]["levels"] for r in rs) + 1
    grid = [dpo.Options.flat(), dpo.Options.naive()]
    for T, CF, (agg, k) in itertools.product([0, 8, 16, 32, 64, 128, 512], [1, 2, 4, 8],
                                             [(1, 4), (2, 4), (3, 4), (3, 16), (4, 4)]):
        grid.append(dpo.Options(threshold=T, coarsen=CF, agg=agg, agg_blocks=k))
    for T, agg, at in itertools.product([8, 32], [1, 2], [8, 32]):  # aggregation threshold
        grid.append(dpo.Options(threshold=T, coarsen=1, agg=agg, agg_threshold=at))
    for o in grid:
        o.steps_per_replay = steps
        pc, _ = measure(dpo, torch, wl, dg, o, 2, 1)
        g = 2 * edges / (pc.sum() * 1e-3) / 1e9
        print(json.dumps({"options": o.label(), "gteps": round(g, 3),
                          "ms_per_traversal": round(float(pc.mean()), 4)}), flush=True)


if __name__ == "__main__":
    main()
