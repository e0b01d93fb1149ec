"""Host-side pieces of bench.py that need no GPU: the edge-certificate check
that the bench runs on an untimed result, against the oracle and against
planted mistakes."""
import numpy as np
import pytest

import bench
import oracle
from paper_2201_02789_amd import graphgen as gg


@pytest.mark.parametrize("scale,seed", [(9, 1), (11, 4)])
def test_certify_accepts_oracle_results(scale, seed):
    g = gg.add_weights(gg.rmat(scale, 16, seed, perm_seed=seed + 10), seed + 20)
    for s in gg.sample_sources(g, 3, seed):
        s = int(s)
        assert bench.certify(g, "bfs", s, oracle.bfs(g, s)[0])
        assert bench.certify(g, "sssp", s, oracle.dijkstra(g, s).view(np.int32))


def test_certify_rejects_planted_mistakes():
    g = gg.add_weights(gg.rmat(10, 16, 2, perm_seed=3), 4)
    s = int(gg.sample_sources(g, 1, 7)[0])
    lv = oracle.bfs(g, s)[0]
    d = oracle.dijkstra(g, s)
    far = int(np.nonzero(lv == lv.max())[0][0])
    for bad in (lambda x: x.__setitem__(far, x[far] + 1),    # a level too high
                lambda x: x.__setitem__(far, x[far] - 1),    # a level too low
                lambda x: x.__setitem__(far, -1),            # a reached vertex dropped
                lambda x: x.__setitem__(s, 1)):              # the source moved
        x = lv.copy()
        bad(x)
        assert not bench.certify(g, "bfs", s, x)
    for delta in (1, -1):
        x = d.copy()
        x[far] = np.uint32(int(x[far]) + delta)
        assert not bench.certify(g, "sssp", s, x.view(np.int32))
    iso = gg.from_edges(5, [(0, 1), (1, 2)])
    lv5 = oracle.bfs(iso, 0)[0]
    assert bench.certify(iso, "bfs", 0, lv5)
    x = lv5.copy()
    x[4] = 2  # an unreachable vertex claimed reached
    assert not bench.certify(iso, "bfs", 0, x)
