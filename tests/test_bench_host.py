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
    the gap into the next level is a gap, workgroups that did not run (zero
    rows) are ignored."""
    rows = np.zeros((64, 3, 4096, 8), dtype=np.uint64)

    def put(L, k, wg, t0, t1, cyc):
        rows[L, k, wg, 0], rows[L, k, wg, 1] = t0, t1
        rows[L, k, wg, 2:7] = cyc

    # level 0: parent kernel 0..100 (two workgroups), child kernel 120..320
    put(0, 0, 0, 0, 100, [30, 15, 5, 0, 0])
    put(0, 0, 7, 10, 90, [30, 15, 5, 0, 0])
    put(0, 1, 0, 120, 320, [0, 0, 0, 10, 90])
    put(0, 1, 3, 130, 220, [0, 0, 0, 10, 90])
    # level 1 starts 30 ticks after level 0 ends: parent only (no launches)
    put(1, 0, 0, 350, 450, [100, 0, 0, 0, 0])
    tot, per_level, imb = bench.phase_split(rows)
    want = {"parent": 0.6 + 1.0, "aggregation": 0.3, "launch": 0.1 + 0.2,
            "disaggregation": 0.2, "child": 1.8, "gaps": 0.3}
    for k, v in want.items():
        assert abs(tot[k] - v) < 1e-9, (k, tot[k], v)
    assert [L for L, _ in per_level] == [0, 1]
    assert abs(sum(per_level[0][1].values()) - 3.2) < 1e-9  # 0 .. 320 ticks
    # child workgroup spans 200 and 90 ticks: busiest / mean = 200 / 145
    assert abs(imb - 200 / 145) < 1e-9


def test_child_skew_on_known_rows():
    """Sixteen child workgroups, those on XCD 3 (workgroups 3 and 11) twice as
    long as the others; entries spread over 10 ticks, exits as they fall."""
    rows = np.zeros((64, 3, 4096, 8), dtype=np.uint64)
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
