"""Host-side pieces of bench.py that need no GPU: the edge-certificate check
that the bench runs on every untimed result (torch ops, here on CPU tensors),
against the oracle and against planted mistakes."""
import numpy as np
import pytest
import torch

import bench
import oracle
from paper_2201_02789_amd import dpo
from paper_2201_02789_amd import graphgen as gg


class _Cert:
    """bench.Certifier over a graph held in CPU tensors."""

    def __init__(self, g):
        self.c = bench.Certifier(torch, dpo.DeviceGraph.from_host(g, device="cpu"))

    def __call__(self, g, kind, s, out):
        return self.c(kind, s, torch.from_numpy(np.ascontiguousarray(out).view(np.int32)))


@pytest.mark.parametrize("scale,seed", [(9, 1), (11, 4)])
def test_certify_accepts_oracle_results(scale, seed):
    g = gg.add_weights(gg.rmat(scale, 16, seed, perm_seed=seed + 10), seed + 20)
    certify = _Cert(g)
    for s in gg.sample_sources(g, 3, seed):
        s = int(s)
        assert certify(g, "bfs", s, oracle.bfs(g, s)[0])
        assert certify(g, "sssp", s, oracle.dijkstra(g, s).view(np.int32))


def test_certify_rejects_planted_mistakes():
    g = gg.add_weights(gg.rmat(10, 16, 2, perm_seed=3), 4)
    s = int(gg.sample_sources(g, 1, 7)[0])
    lv = oracle.bfs(g, s)[0]
    d = oracle.dijkstra(g, s)
    far = int(np.nonzero(lv == lv.max())[0][0])
    certify = _Cert(g)
    for bad in (lambda x: x.__setitem__(far, x[far] + 1),    # a level too high
                lambda x: x.__setitem__(far, x[far] - 1),    # a level too low
                lambda x: x.__setitem__(far, -1),            # a reached vertex dropped
                lambda x: x.__setitem__(s, 1)):              # the source moved
        x = lv.copy()
        bad(x)
        assert not certify(g, "bfs", s, x)
    for delta in (1, -1):
        x = d.copy()
        x[far] = np.uint32(int(x[far]) + delta)
        assert not certify(g, "sssp", s, x.view(np.int32))
    iso = gg.from_edges(5, [(0, 1), (1, 2)])
    lv5 = oracle.bfs(iso, 0)[0]
    certify = _Cert(iso)
    assert certify(iso, "bfs", 0, lv5)
    x = lv5.copy()
    x[4] = 2  # an unreachable vertex claimed reached
    assert not certify(iso, "bfs", 0, x)


def test_phase_split_on_known_rows():
    """Two levels of hand-made timing rows (100 ticks = 1 us): each kernel's
    span is split by its cycle shares, the parent-to-child gap is launch time,
    the gaps into the harvest and into the next level are gaps, workgroups that
    did not run (zero rows) are ignored."""
    rows = np.zeros((64, 4, 4096, 8), dtype=np.uint64)

    def put(L, k, wg, t0, t1, cyc):
        rows[L, k, wg, 0], rows[L, k, wg, 1] = t0, t1
        rows[L, k, wg, 2:7] = cyc

    # level 0: parent kernel 0..100 (two workgroups), child kernel 120..320,
    # harvest 330..340 (its cycles are child work)
    put(0, 0, 0, 0, 100, [30, 15, 5, 0, 0])
    put(0, 0, 7, 10, 90, [30, 15, 5, 0, 0])
    put(0, 1, 0, 120, 320, [0, 0, 0, 10, 90])
    put(0, 1, 3, 130, 220, [0, 0, 0, 10, 90])
    put(0, 3, 2, 330, 340, [0, 0, 0, 0, 10])
    # level 1 starts 10 ticks after level 0 ends: parent only (no launches)
    put(1, 0, 0, 350, 450, [100, 0, 0, 0, 0])
    tot, per_level, imb = bench.phase_split(rows)
    want = {"parent": 0.6 + 1.0, "aggregation": 0.3, "launch": 0.1 + 0.2,
            "disaggregation": 0.2, "child": 1.8 + 0.1, "gaps": 0.1 + 0.1}
    for k, v in want.items():
        assert abs(tot[k] - v) < 1e-9, (k, tot[k], v)
    assert [L for L, _ in per_level] == [0, 1]
    assert abs(sum(per_level[0][1].values()) - 3.4) < 1e-9  # 0 .. 340 ticks
    # child workgroup spans 200 and 90 ticks: busiest / mean = 200 / 145
    assert abs(imb - 200 / 145) < 1e-9


def test_level_table_names_the_four_kernels():
    """Per level: each kernel's span (first entry to last exit) under its own
    name, and the child kernel's workgroup statistics."""
    rows = np.zeros((64, 4, 4096, 8), dtype=np.uint64)
    rows[0, 0, 0, :2] = (0, 50)
    rows[0, 1, 0, :2], rows[0, 1, 1, :2] = (60, 160), (70, 110)
    rows[0, 2, 5, :2] = (170, 200)
    rows[0, 3, 9, :2] = (210, 220)
    rows[1, 0, 0, :2] = (300, 320)
    t = bench.level_table(rows)
    assert [r["level"] for r in t] == [0, 1]
    r = t[0]
    assert (r["parent_us"], r["child_us"], r["serial_us"], r["harvest_us"]) == (0.5, 1.0, 0.3, 0.1)
    assert (r["child_wg_mean_us"], r["child_wg_max_us"], r["child_workgroups"]) == (0.7, 1.0, 2)
    assert r["child_exit_spread_us"] == 0.5
    assert t[1] == {"level": 1, "parent_us": 0.2}


def test_child_skew_on_known_rows():
    """Sixteen child workgroups, those on XCD 3 (workgroups 3 and 11) twice as
    long as the others; entries spread over 10 ticks, exits as they fall."""
    rows = np.zeros((64, 4, 4096, 8), dtype=np.uint64)
    for w in range(16):
        t0 = 100 + (w % 11)  # entries 100 .. 110
        span = 200 if w % 8 == 3 else 100
        rows[0, 1, w, 0], rows[0, 1, w, 1] = t0, t0 + span
        rows[0, 1, w, 6] = 1
    sk = bench.child_skew(rows)
    assert abs(sk["start_spread_us"] - 0.10) < 1e-9
    assert abs(sk["xcd_span_ratio"] - 2.0) < 1e-9
    t1 = [100 + (w % 11) + (200 if w % 8 == 3 else 100) for w in range(16)]
    assert abs(sk["end_spread_us"] - (max(t1) - min(t1)) / 100) < 1e-9


def test_summarize_counters_on_synthetic_passes(tmp_path, monkeypatch):
    """The counter summary divides by the traversal count of each pass (one CSV
    row per counter per dispatch) and by the edges of the run's bench line."""
    import csv
    import json

    d = tmp_path / "sq"
    edges = 1000.0
    for i, passes in enumerate(bench.COUNTER_PASSES, start=1):
        names = passes.split()
        pd = d / f"bfs22_p{i}"
        pd.mkdir(parents=True)
        with open(pd / "c_counter_collection.csv", "w", newline="") as f:
            w = csv.DictWriter(f, fieldnames=["Dispatch_Id", "Kernel_Name", "Counter_Name",
                                              "Counter_Value"])
            w.writeheader()
            for t in range(2):  # two traversals: init, parent, child dispatches
                for k, kern in enumerate(("dpo::init_kernel(dpo::Args)",
                                          "void dpo::child_kernel<0, false>(dpo::Args, unsigned int)")):
                    for c in names:
                        val = {"SQ_WAVE_CYCLES": 1000.0, "SQ_WAIT_INST_ANY": 500.0,
                               "SQ_INSTS_VALU": 300.0, "TCP_TCC_READ_REQ_sum": 10.0,
                               "TCP_TCC_READ_REQ_LATENCY_sum": 4000.0}.get(c, 1.0)
                        w.writerow({"Dispatch_Id": 10 * t + k, "Kernel_Name": kern,
                                    "Counter_Name": c, "Counter_Value": val})
        (d / f"bfs22_p{i}.out").write_text(json.dumps(
            {"roofline_probe": {"probes_per_traversal": edges}}) + "\n")
    monkeypatch.setattr(bench, "ROOT", str(tmp_path))
    (tmp_path / "profiles").mkdir()

    class A:
        workload = "bfs22"

    bench.summarize_counters(A(), str(d))
    md = (tmp_path / "profiles" / "bfs22_counters.md").read_text()
    row = [ln for ln in md.splitlines() if ln.startswith("| child_kernel<0, false>") and "/" in ln][0]
    cells = [c.strip() for c in row.strip("|").split("|")]
    assert cells[2] == "0.500"                  # waiting share: 2 x 500 / 2 x 1000
    assert cells[4].startswith("0.30 /")        # VALU per edge: 2 x 300 / (2 traversals x 1000)
    assert cells[5] == "400"                    # L2 read latency: 8000 / 20
    assert "Traversals per run: 2;" in md
