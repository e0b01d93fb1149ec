"""Edge certificates for BFS levels and SSSP distances (numpy, O(n + m)).

They pin a result without re-running any traversal, so they check the CPU
oracle and the GPU output alike, at every size.

BFS, source s, level[v] = -1 for unreached:
  (i)   level[s] == 0 and every reached level is >= 0, only s has level 0;
  (ii)  every reached v != s has a reached in-neighbour u, level[u] = level[v]-1;
  (iii) for every edge u->v with u reached: v reached, level[v] <= level[u]+1.
(ii) makes level[v] the length of a real path (>= hop distance); (iii) by
induction along a shortest path gives <= and closes reachability.

SSSP with weights >= 1, dist = 0xFFFFFFFF for unreached:
  (i)   dist[s] == 0;
  (ii)  for every edge u->v with u reached: v reached, dist[v] <= dist[u]+w;
  (iii) every reached v != s has a reached u with dist[v] == dist[u]+w(u,v).
"""
import numpy as np

UNREACHED = 0xFFFFFFFF


def _edges(g):
    src = np.repeat(np.arange(g.n, dtype=np.int64), np.diff(g.row_ptr).astype(np.int64))
    return src, g.col_idx.astype(np.int64)


def check_bfs(g, src, level):
    level = np.asarray(level).astype(np.int64)
    n = g.n
    assert level.shape == (n,)
    assert level[src] == 0, "level[source] != 0"
    assert np.all(level >= -1)
    zeros = np.flatnonzero(level == 0)
    assert zeros.size == 1 and zeros[0] == src, "vertex other than the source at level 0"
    u, v = _edges(g)
    ru = level[u] >= 0
    # (iii)
    lv, lu = level[v[ru]], level[u[ru]]
    assert np.all(lv >= 0), "edge from a reached vertex to an unreached one"
    assert np.all(lv <= lu + 1), "edge skips a level"
    # (ii): a reached predecessor one level up exists for each reached v != s
    tight = ru & (level[v] == level[u] + 1)
    has_parent = np.zeros(n, dtype=bool)
    has_parent[v[tight]] = True
    need = (level > 0)
    assert np.all(has_parent[need]), "reached vertex without a parent one level up"
    return True


def check_sssp(g, src, dist):
    dist = np.asarray(dist).astype(np.uint64)
    n = g.n
    assert dist.shape == (n,)
    assert dist[src] == 0, "dist[source] != 0"
    u, v = _edges(g)
    w = g.weights.astype(np.uint64)
    assert np.all(w >= 1)
    reached = dist != UNREACHED
    ru = reached[u]
    du, dv, we = dist[u[ru]], dist[v[ru]], w[ru]
    assert np.all(dv != UNREACHED), "edge from a reached vertex to an unreached one"
    assert np.all(dv <= du + we), "relaxable edge left"
    tight = np.zeros(u.shape, dtype=bool)
    tight[ru] = dv == du + we
    has_pred = np.zeros(n, dtype=bool)
    has_pred[v[tight]] = True
    need = reached.copy()
    need[src] = False
    assert np.all(has_pred[need]), "reached vertex without a tight predecessor"
    return True
