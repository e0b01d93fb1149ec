"""Seeded input generators: determinism and CSR well-formedness (no GPU)."""
import numpy as np
import pytest

from paper_2201_02789_amd import graphgen as gg


def well_formed(g):
    rp, col = g.row_ptr, g.col_idx
    assert rp[0] == 0 and rp[-1] == col.size and np.all(np.diff(rp) >= 0)
    src = np.repeat(np.arange(g.n), np.diff(rp))
    assert np.all((col >= 0) & (col < g.n))
    assert not np.any(src == col), "self loop"
    key = src.astype(np.int64) * g.n + col
    assert np.all(np.diff(key) > 0), "rows not sorted or duplicate entries"
    rkey = col.astype(np.int64) * g.n + src
    assert np.array_equal(np.sort(rkey), key), "not symmetric"


@pytest.mark.parametrize("scale,ef,perm", [(8, 8, 0), (12, 16, 0), (12, 16, 24), (14, 32, 7)])
def test_rmat_deterministic_and_well_formed(scale, ef, perm):
    a = gg.rmat(scale, ef, 1, perm_seed=perm)
    b = gg.rmat(scale, ef, 1, perm_seed=perm)
    assert np.array_equal(a.row_ptr, b.row_ptr) and np.array_equal(a.col_idx, b.col_idx)
    well_formed(a)
    assert a.n == 1 << scale
    assert a.m <= 2 * ef * a.n
    c = gg.rmat(scale, ef, 2, perm_seed=perm)
    assert not np.array_equal(a.col_idx[: min(a.m, c.m)], c.col_idx[: min(a.m, c.m)])


def test_rmat_unpermuted_hub_is_vertex0_and_skewed():
    g = gg.rmat(12, 16, 1)
    d = g.degrees()
    assert int(np.argmax(d)) == 0
    assert d.max() > 20 * d[d > 0].mean()


def test_permutation_is_a_relabelling():
    a = gg.rmat(10, 16, 1)
    b = gg.rmat(10, 16, 1, perm_seed=24)
    perm = gg.permutation(a.n, 24)
    assert np.array_equal(np.sort(perm), np.arange(a.n))
    assert a.m == b.m
    assert np.array_equal(np.sort(a.degrees()), np.sort(b.degrees()))
    assert np.array_equal(b.degrees()[perm], a.degrees())


def test_er_same_counts():
    g = gg.rmat(12, 16, 5, perm_seed=3)
    e = gg.erdos_renyi(g.n, g.m // 2, 23)
    well_formed(e)
    assert e.n == g.n and e.m == g.m
    d = e.degrees()
    assert d.max() < 5 * d.mean()  # Poisson-like, no hubs


def test_weights_symmetric_in_range():
    g = gg.add_weights(gg.rmat(11, 16, 3, perm_seed=4), 31)
    w = g.weights
    assert w.min() >= 1 and w.max() <= 255
    src = np.repeat(np.arange(g.n), g.degrees())
    fwd = dict(zip(zip(src.tolist(), g.col_idx.tolist()), w.tolist()))
    for (u, v), x in list(fwd.items())[:5000]:
        assert fwd[(v, u)] == x


def test_sources_rule():
    g = gg.rmat(12, 16, 1, perm_seed=24)
    s = gg.sample_sources(g, 16, 1)
    assert len(set(s.tolist())) == 16
    assert np.all(g.degrees()[s] >= 1)
    assert np.array_equal(s, gg.sample_sources(g, 16, 1))
    d = g.degrees()
    v = gg.max_degree_vertex(g)
    assert d[v] == d.max() and np.all(d[:v] < d[v])


def test_small_structures():
    well_formed(gg.grid_graph(5, 7))
    well_formed(gg.road_like(30, 30, 3))
    assert gg.road_like(30, 30, 3).degrees().max() <= 8
    well_formed(gg.binary_tree(100))
    assert gg.star_graph(10).degrees().tolist() == [9] + [1] * 9
