"""Pins of the CPU oracle against things other than itself.

Brute force (hop distances from boolean matrix powers, Floyd-Warshall),
closed forms of structured graphs, edge certificates, and planted mistakes
that the certificates must catch.  No GPU.
"""
import itertools

import numpy as np
import pytest

import oracle
from paper_2201_02789_amd import graphgen as gg
from tests import certificates as cert

U = 0xFFFFFFFF


def all_graphs(n):
    pairs = list(itertools.combinations(range(n), 2))
    for mask in range(1 << len(pairs)):
        yield [p for i, p in enumerate(pairs) if mask >> i & 1]


def hop_matrix(n, edges):
    """All-pairs hop distance: the smallest k with a walk of length k."""
    a = np.zeros((n, n), dtype=bool)
    for u, v in edges:
        a[u, v] = a[v, u] = True
    d = np.full((n, n), -1, dtype=np.int64)
    reach = np.eye(n, dtype=bool)
    d[reach] = 0
    for k in range(1, n):
        reach = (reach.astype(np.int64) @ a.astype(np.int64)) > 0
        d[(d == -1) & reach] = k
    return d


def floyd_warshall(n, edges, weights):
    inf = np.iinfo(np.int64).max // 4
    d = np.full((n, n), inf, dtype=np.int64)
    np.fill_diagonal(d, 0)
    for (u, v), w in zip(edges, weights):
        d[u, v] = min(d[u, v], w)
        d[v, u] = min(d[v, u], w)
    for k in range(n):
        d = np.minimum(d, d[:, k:k + 1] + d[k:k + 1, :])
    out = np.where(d >= inf, U, d).astype(np.uint64)
    return out


@pytest.mark.parametrize("n", [1, 2, 3, 4, 5])
def test_bfs_all_graphs_brute_force(n):
    for edges in all_graphs(n):
        g = gg.from_edges(n, edges)
        hop = hop_matrix(n, edges)
        for s in range(n):
            lv, depth = oracle.bfs(g, s)
            assert np.array_equal(lv, hop[s]), (edges, s)
            assert depth == hop[s].max() + 1


def test_bfs_all_graphs_n6():
    """Every one of the 2^15 labelled simple graphs on 6 vertices, every
    source: hop distances from boolean matrix powers, computed for all graphs
    at once (stacked 6 x 6 adjacency matrices)."""
    n = 6
    pairs = list(itertools.combinations(range(n), 2))
    masks = np.arange(1 << len(pairs))
    adj = np.zeros((masks.size, n, n), dtype=np.int64)
    for i, (u, v) in enumerate(pairs):
        bit = (masks >> i) & 1
        adj[:, u, v] = bit
        adj[:, v, u] = bit
    hop = np.full((masks.size, n, n), -1, dtype=np.int64)
    reach = np.broadcast_to(np.eye(n, dtype=np.int64), adj.shape).copy()
    hop[reach > 0] = 0
    for k in range(1, n):
        reach = ((reach @ adj) > 0).astype(np.int64)
        hop[(hop == -1) & (reach > 0)] = k
    for mask in masks:
        edges = [p for i, p in enumerate(pairs) if mask >> i & 1]
        g = gg.from_edges(n, edges)
        for s in range(n):
            assert np.array_equal(oracle.bfs(g, s)[0], hop[mask, s]), (edges, s)


@pytest.mark.parametrize("seed", range(12))
def test_bfs_and_dijkstra_random_vs_floyd_warshall(seed):
    rng = np.random.default_rng(seed)
    n = int(rng.integers(2, 65))
    p = float(rng.uniform(0.02, 0.3))
    edges = [(u, v) for u in range(n) for v in range(u + 1, n) if rng.random() < p]
    w = rng.integers(1, 256, size=len(edges))
    g = gg.from_edges(n, edges, w)
    fw = floyd_warshall(n, edges, w)
    hop = hop_matrix(n, edges)
    for s in range(0, n, max(1, n // 8)):
        assert np.array_equal(oracle.dijkstra(g, s), fw[s])
        assert np.array_equal(oracle.bfs(g, s)[0], hop[s])


def test_dijkstra_exhaustive_small_weights():
    n = 4
    for edges in all_graphs(n):
        for ws in itertools.product((1, 2, 3), repeat=len(edges)):
            g = gg.from_edges(n, edges, list(ws))
            fw = floyd_warshall(n, edges, ws)
            for s in range(n):
                assert np.array_equal(oracle.dijkstra(g, s), fw[s])


@pytest.mark.parametrize("seed", range(16))
def test_dijkstra_zero_and_near_2_32_weights_vs_floyd_warshall(seed):
    """Weights 0 and just below 2^32 (sums past 32 bits) against
    Floyd-Warshall in int64: exact when every distance fits below
    0xFFFFFFFF, an error otherwise."""
    rng = np.random.default_rng(1000 + seed)
    n = int(rng.integers(3, 41))
    edges = [(u, v) for u in range(n) for v in range(u + 1, n) if rng.random() < 0.15]
    kind = rng.integers(0, 3, size=len(edges))
    w = np.where(kind == 0, 0, np.where(kind == 1, rng.integers(1, 1 << 20, size=len(edges)),
                                        (1 << 32) - rng.integers(1, 1 << 20, size=len(edges))))
    g = gg.from_edges(n, edges, w)
    fw = floyd_warshall(n, edges, w)
    for s in range(n):
        finite = fw[s][fw[s] != U]
        if finite.size and finite.max() >= U:
            with pytest.raises(ValueError):
                oracle.dijkstra(g, s)
        else:
            assert np.array_equal(oracle.dijkstra(g, s), fw[s])


def test_unit_weights_dijkstra_equals_bfs():
    g = gg.rmat(10, 8, 3, perm_seed=5)
    g1 = gg.Graph(g.row_ptr, g.col_idx, np.ones(g.m, dtype=np.uint32))
    for s in gg.sample_sources(g, 4, 9):
        lv, _ = oracle.bfs(g, s)
        d = oracle.dijkstra(g1, s)
        assert np.array_equal(np.where(lv < 0, U, lv.astype(np.int64)).astype(np.uint64), d.astype(np.uint64))


# ------------------------------------------------------------------ closed forms
@pytest.mark.parametrize("n", [1, 2, 7, 100])
def test_path(n):
    lv, depth = oracle.bfs(gg.path_graph(n), 0)
    assert np.array_equal(lv, np.arange(n)) and depth == n


@pytest.mark.parametrize("n", [3, 4, 9, 50])
def test_cycle(n):
    i = np.arange(n)
    assert np.array_equal(oracle.bfs(gg.cycle_graph(n), 0)[0], np.minimum(i, n - i))


def test_star_complete_tree_grid():
    lv = oracle.bfs(gg.star_graph(300), 0)[0]
    assert lv[0] == 0 and np.all(lv[1:] == 1)
    lv = oracle.bfs(gg.star_graph(300), 5)[0]
    assert lv[5] == 0 and lv[0] == 1 and np.all(np.delete(lv, [0, 5]) == 2)
    lv = oracle.bfs(gg.complete_graph(30), 3)[0]
    assert lv[3] == 0 and np.all(np.delete(lv, 3) == 1)
    n = 1000
    lv = oracle.bfs(gg.binary_tree(n), 0)[0]
    assert np.array_equal(lv, np.floor(np.log2(np.arange(n) + 1)).astype(np.int32))
    r, c = 13, 17
    lv = oracle.bfs(gg.grid_graph(r, c), 0)[0]
    assert np.array_equal(lv, (np.arange(r * c) // c) + (np.arange(r * c) % c))


def test_isolated_and_two_components():
    g = gg.from_edges(5, [(1, 2), (3, 4)])
    lv = oracle.bfs(g, 0)[0]
    assert lv.tolist() == [0, -1, -1, -1, -1]
    lv = oracle.bfs(g, 1)[0]
    assert lv.tolist() == [-1, 0, 1, -1, -1]
    gw = gg.from_edges(5, [(1, 2), (3, 4)], [7, 9])
    d = oracle.dijkstra(gw, 3)
    assert d.tolist() == [U, U, U, 0, 9]


def test_weighted_path_prefix_sums():
    rng = np.random.default_rng(4)
    n = 200
    w = rng.integers(1, 256, size=n - 1)
    g = gg.from_edges(n, [(i, i + 1) for i in range(n - 1)], w)
    assert np.array_equal(oracle.dijkstra(g, 0), np.concatenate([[0], np.cumsum(w)]))
    assert np.array_equal(oracle.dijkstra(g, n - 1)[::-1], np.concatenate([[0], np.cumsum(w[::-1])]))


def test_relabel_invariance():
    g = gg.rmat(9, 8, 11)
    perm = gg.permutation(g.n, 77)
    h = gg.relabel(g, perm)
    s = int(gg.sample_sources(g, 1, 2)[0])
    a = oracle.bfs(g, s)[0]
    b = oracle.bfs(h, int(perm[s]))[0]
    assert np.array_equal(b[perm], a)


# ------------------------------------------------------------------ certificates
@pytest.mark.parametrize("scale", [10, 12, 14])
def test_certificates_hold_on_oracle_output(scale):
    g = gg.add_weights(gg.rmat(scale, 16, scale, perm_seed=24), 31)
    for s in gg.sample_sources(g, 3, 1):
        lv, _ = oracle.bfs(g, s)
        cert.check_bfs(g, s, lv)
        cert.check_sssp(g, s, oracle.dijkstra(g, s))


def test_certificates_catch_planted_mistakes():
    g = gg.add_weights(gg.rmat(11, 16, 2, perm_seed=3), 5)
    s = int(gg.sample_sources(g, 1, 1)[0])
    lv, _ = oracle.bfs(g, s)
    d = oracle.dijkstra(g, s)
    reached = np.flatnonzero(lv > 0)
    for bad in (lambda a: a + (np.arange(a.size) == reached[0]),        # one level too high
                lambda a: a - (np.arange(a.size) == reached[-1]),       # one level too low
                lambda a: np.where(np.arange(a.size) == reached[3], -1, a),  # dropped vertex
                lambda a: np.where(a > 0, a + 1, a)):                   # wrong offset
        with pytest.raises(AssertionError):
            cert.check_bfs(g, s, bad(lv.copy()).astype(np.int32))
    for bad in (lambda a: a + (np.arange(a.size) == reached[1]).astype(np.uint32),
                lambda a: a - (np.arange(a.size) == reached[2]).astype(np.uint32),
                lambda a: np.where(np.arange(a.size) == reached[4], U, a).astype(np.uint32)):
        with pytest.raises(AssertionError):
            cert.check_sssp(g, s, bad(d.copy()))


# ------------------------------------------------------------------ schedule counts
def test_schedule_paper_threshold_example():
    """Sec. III-D: child blocks of 1024 threads, one parent with 2 units of
    nested work -> one block; the count compared with the threshold is 2,
    not gDim * bDim = 1024."""
    import json, os
    fx = json.load(open(os.path.join(os.path.dirname(__file__), "golden", "threshold_example.json")))
    g = gg.star_graph(fx["nested_work"] + 1)
    lv = np.full(g.n, -1, dtype=np.int32)
    lv[0] = 0  # the hub alone is the frontier
    for T, expect_serial in ((fx["nested_work"] + 1, True), (fx["nested_work"], False)):
        c = oracle.schedule_counts(g, lv, T, fx["child_block"], 1)
        assert c["serial_parents"] == int(expect_serial)
        assert c["records"] == int(not expect_serial)
        if not expect_serial:
            assert c["child_blocks"] == fx["grid_dim"]
    assert fx["grid_dim"] * fx["child_block"] == fx["naive_thread_count"]


def test_schedule_star_closed_form():
    n = 5000
    g = gg.star_graph(n)
    lv, _ = oracle.bfs(g, 0)
    for T, CB, CF in ((0, 256, 1), (2, 256, 4), (8, 64, 8), (n, 128, 2)):
        c = oracle.schedule_counts(g, lv, T, CB, CF)
        hub_launch = (n - 1) >= max(T, 1)
        leaf_launch = 1 >= max(T, 1)
        assert c["records"] == int(hub_launch) + (n - 1) * int(leaf_launch)
        hub_cb = -(-(-(-(n - 1) // CB)) // CF)
        assert c["child_blocks"] == hub_cb * int(hub_launch) + (n - 1) * int(leaf_launch)
        assert c["edges_serial"] + c["edges_child"] == 2 * (n - 1)
        f = oracle.schedule_counts(g, lv, T, CB, CF, flat=True)
        assert f["serial_parents"] == n and f["records"] == 0


@pytest.mark.parametrize("T,CB,CF,grp", [(0, 4, 1, 1), (3, 4, 2, 8), (5, 2, 3, 64), (0, 8, 8, 16),
                                        (100, 4, 1, 4)])
def test_simulated_schedule_covers_each_edge_once(T, CB, CF, grp):
    g = gg.rmat(8, 8, 6, perm_seed=2)
    s = int(gg.sample_sources(g, 1, 3)[0])
    lv, depth = oracle.bfs(g, s)
    rp = g.row_ptr
    tot = {"serial": 0, "child": 0, "records": 0, "blocks": 0}
    for L in range(depth):
        frontier = np.flatnonzero(lv == L)
        serial, child, grids = oracle.simulate_nested(rp, frontier, T, CB, CF, grp)
        got = sorted(serial + child)
        want = sorted((int(u), e) for u in frontier for e in range(rp[u], rp[u + 1]))
        assert got == want
        assert len(grids) <= -(-frontier.size // grp)  # at most one grid per group
        tot["serial"] += len(serial)
        tot["child"] += len(child)
        tot["records"] += sum(r for r, _ in grids)
        tot["blocks"] += sum(b for _, b in grids)
    c = oracle.schedule_counts(g, lv, T, CB, CF)
    assert c["edges_serial"] == tot["serial"] and c["edges_child"] == tot["child"]
    assert c["records"] == tot["records"] and c["child_blocks"] == tot["blocks"]
