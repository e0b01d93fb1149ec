"""Seeded synthetic inputs: R-MAT / Erdos-Renyi CSR graphs, edge weights, sources.

This module only builds inputs.  It holds none of the traversal arithmetic and
is shared by the GPU path, the CPU oracle and the tests.  The bulk generators
are C (``graphgen.c``, OpenMP) loaded with ctypes; the small structured graphs
used by the tests are plain numpy.

The paper's graph benchmarks run on a Kronecker graph (Table I,
kron_g500-simple-logn16); R-MAT with the Graph500 parameters a/b/c/d =
0.57/0.19/0.19/0.05 is the same family and stands in for it at any scale.
"""
from __future__ import annotations

import ctypes
import os
from dataclasses import dataclass
from typing import Optional

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(_HERE, "libgraphgen.so")
SRC_PATH = os.path.join(_HERE, "graphgen.c")

RMAT_ABCD = (0.57, 0.19, 0.19, 0.05)
PHI = 0x9E3779B97F4A7C15
MASK64 = (1 << 64) - 1

_lib = None


def build(verbose: bool = False) -> str:
    """Compile graphgen.c into libgraphgen.so (gcc, -O3, OpenMP)."""
    import subprocess
    cmd = ["gcc", "-O3", "-fopenmp", "-fPIC", "-shared", "-o", LIB_PATH + ".tmp", SRC_PATH]
    if verbose:
        print(" ".join(cmd))
    subprocess.check_call(cmd)
    os.replace(LIB_PATH + ".tmp", LIB_PATH)
    return LIB_PATH


def _load():
    global _lib
    if _lib is not None:
        return _lib
    if not os.path.exists(LIB_PATH):
        build()
    lib = ctypes.CDLL(LIB_PATH)
    i32p = ctypes.POINTER(ctypes.c_int32)
    u32p = ctypes.POINTER(ctypes.c_uint32)
    lib.gg_rmat.restype = ctypes.c_int64
    lib.gg_rmat.argtypes = [ctypes.c_int32, ctypes.c_int32, ctypes.c_double, ctypes.c_double,
                            ctypes.c_double, ctypes.c_uint64, ctypes.c_uint64, i32p, i32p,
                            ctypes.c_int64]
    lib.gg_er.restype = ctypes.c_int64
    lib.gg_er.argtypes = [ctypes.c_int32, ctypes.c_int64, ctypes.c_uint64, i32p, i32p, ctypes.c_int64]
    lib.gg_weights.restype = None
    lib.gg_weights.argtypes = [ctypes.c_int32, i32p, i32p, ctypes.c_uint64, u32p]
    lib.gg_permutation.restype = None
    lib.gg_permutation.argtypes = [ctypes.c_int32, ctypes.c_uint64, i32p]
    lib.gg_splitmix64.restype = ctypes.c_uint64
    lib.gg_splitmix64.argtypes = [ctypes.c_uint64]
    lib.gg_num_threads.restype = ctypes.c_int32
    _lib = lib
    return lib


def _p(a: np.ndarray, t):
    return a.ctypes.data_as(ctypes.POINTER(t))


@dataclass
class Graph:
    """Int32 CSR graph; ``weights`` is None for unweighted graphs."""
    row_ptr: np.ndarray
    col_idx: np.ndarray
    weights: Optional[np.ndarray] = None
    name: str = ""

    @property
    def n(self) -> int:
        return int(self.row_ptr.shape[0] - 1)

    @property
    def m(self) -> int:
        return int(self.col_idx.shape[0])

    def degrees(self) -> np.ndarray:
        return np.diff(self.row_ptr)


def splitmix64(x: int) -> int:
    return int(_load().gg_splitmix64(ctypes.c_uint64(x & MASK64)))


def rmat(scale: int, edgefactor: int, seed: int, perm_seed: int = 0,
         abcd=RMAT_ABCD, name: str = "") -> Graph:
    """R-MAT graph, 2^scale vertices, symmetric, deduplicated, no self loops.

    ``perm_seed`` = 0 keeps generated ids (vertex 0 is then the hub); any other
    value relabels the vertices by a seeded Fisher-Yates permutation.
    """
    lib = _load()
    n = 1 << scale
    cap = 2 * edgefactor * n
    rp = np.empty(n + 1, dtype=np.int32)
    col = np.empty(cap, dtype=np.int32)
    a, b, c, _ = abcd
    m = lib.gg_rmat(scale, edgefactor, a, b, c, seed & MASK64, perm_seed & MASK64,
                    _p(rp, ctypes.c_int32), _p(col, ctypes.c_int32), cap)
    if m < 0:
        raise RuntimeError(f"gg_rmat failed ({m})")
    return Graph(rp, col[:m].copy(), None, name or f"rmat-s{scale}-ef{edgefactor}-seed{seed}")


def erdos_renyi(n: int, num_undirected: int, seed: int, name: str = "") -> Graph:
    """G(n, M) with exactly M distinct undirected edges (no self loops)."""
    lib = _load()
    cap = 2 * num_undirected
    rp = np.empty(n + 1, dtype=np.int32)
    col = np.empty(max(cap, 1), dtype=np.int32)
    m = lib.gg_er(n, num_undirected, seed & MASK64, _p(rp, ctypes.c_int32),
                  _p(col, ctypes.c_int32), cap)
    if m < 0:
        raise RuntimeError(f"gg_er failed ({m})")
    return Graph(rp, col[:m].copy(), None, name or f"er-n{n}-M{num_undirected}-seed{seed}")


def add_weights(g: Graph, wseed: int) -> Graph:
    """Attach uint32 weights in [1, 255], one per undirected edge."""
    lib = _load()
    w = np.empty(max(g.m, 1), dtype=np.uint32)
    lib.gg_weights(g.n, _p(g.row_ptr, ctypes.c_int32), _p(g.col_idx, ctypes.c_int32),
                   wseed & MASK64, _p(w, ctypes.c_uint32))
    return Graph(g.row_ptr, g.col_idx, w[: g.m].copy(), g.name + f"-w{wseed}")


def permutation(n: int, seed: int) -> np.ndarray:
    perm = np.empty(n, dtype=np.int32)
    _load().gg_permutation(n, seed & MASK64, _p(perm, ctypes.c_int32))
    return perm


def sample_sources(g: Graph, count: int, seed: int) -> np.ndarray:
    """``count`` distinct sources, uniform over vertices with degree >= 1.

    Candidate i is splitmix64(seed * PHI + i) mod n; it is kept if its degree
    is at least one and it was not drawn before (Graph500 source rule).
    """
    deg = g.degrees()
    eligible = int(np.count_nonzero(deg))
    if eligible < count:
        raise ValueError("not enough vertices with degree >= 1")
    out, seen, i = [], set(), 0
    while len(out) < count:
        v = splitmix64((seed * PHI + i) & MASK64) % g.n
        i += 1
        if deg[v] >= 1 and v not in seen:
            seen.add(v)
            out.append(v)
    return np.array(out, dtype=np.int32)


def max_degree_vertex(g: Graph) -> int:
    """Vertex of maximum degree; ties go to the smallest id."""
    return int(np.argmax(g.degrees()))


# ---------------------------------------------------------------- small graphs
def from_edges(n: int, edges, weights=None, symmetric: bool = True, name: str = "") -> Graph:
    """CSR from an edge list.  Rows sorted; duplicates kept only once.

    With ``symmetric`` every (u, v, w) is also stored as (v, u, w).
    """
    e = np.asarray(edges, dtype=np.int64).reshape(-1, 2)
    w = None if weights is None else np.asarray(weights, dtype=np.uint64).reshape(-1)
    if symmetric:
        e = np.concatenate([e, e[:, ::-1]], axis=0)
        if w is not None:
            w = np.concatenate([w, w])
    if e.shape[0]:
        key = e[:, 0] * n + e[:, 1]
        key, idx = np.unique(key, return_index=True)
        e = e[idx]
        if w is not None:
            w = w[idx]
    rp = np.zeros(n + 1, dtype=np.int64)
    if e.shape[0]:
        np.add.at(rp, e[:, 0] + 1, 1)
    rp = np.cumsum(rp).astype(np.int32)
    col = e[:, 1].astype(np.int32) if e.shape[0] else np.zeros(0, dtype=np.int32)
    wt = None if w is None else w.astype(np.uint32)
    return Graph(rp, col, wt, name)


def path_graph(n: int) -> Graph:
    return from_edges(n, [(i, i + 1) for i in range(n - 1)], name=f"path{n}")


def cycle_graph(n: int) -> Graph:
    return from_edges(n, [(i, (i + 1) % n) for i in range(n)], name=f"cycle{n}")


def star_graph(n: int) -> Graph:
    """Vertex 0 joined to 1..n-1."""
    return from_edges(n, [(0, i) for i in range(1, n)], name=f"star{n}")


def complete_graph(n: int) -> Graph:
    return from_edges(n, [(i, j) for i in range(n) for j in range(i + 1, n)], name=f"K{n}")


def binary_tree(n: int) -> Graph:
    """Heap-ordered complete binary tree: parent of i is (i - 1) // 2."""
    return from_edges(n, [((i - 1) // 2, i) for i in range(1, n)], name=f"bintree{n}")


def grid_graph(r: int, c: int) -> Graph:
    """r x c 4-neighbour grid, vertex (i, j) -> i * c + j."""
    ed = []
    for i in range(r):
        for j in range(c):
            if j + 1 < c:
                ed.append((i * c + j, i * c + j + 1))
            if i + 1 < r:
                ed.append((i * c + j, (i + 1) * c + j))
    return from_edges(r * c, ed, name=f"grid{r}x{c}")


def road_like(r: int, c: int, seed: int, drop: float = 0.25) -> Graph:
    """Low-nesting control: an r x c grid with a seeded share of edges removed
    and a few diagonals added, so that degrees stay in [0, 8] (the paper's road
    graph has average degree 3 and maximum degree 8)."""
    rng = np.random.default_rng(seed)
    ed = []
    for i in range(r):
        for j in range(c):
            v = i * c + j
            if j + 1 < c and rng.random() >= drop:
                ed.append((v, v + 1))
            if i + 1 < r and rng.random() >= drop:
                ed.append((v, v + c))
            if i + 1 < r and j + 1 < c and rng.random() < 0.1:
                ed.append((v, v + c + 1))
    return from_edges(r * c, ed, name=f"road{r}x{c}-seed{seed}")


def relabel(g: Graph, perm: np.ndarray) -> Graph:
    """Graph with vertex v renamed perm[v] (rows re-sorted)."""
    n = g.n
    src = np.repeat(np.arange(n, dtype=np.int64), np.diff(g.row_ptr))
    e = np.stack([perm[src], perm[g.col_idx]], axis=1)
    return from_edges(n, e, g.weights, symmetric=False, name=g.name + "-relabel")


def pack_arena(graphs):
    """Packs graphs into one CSR arena: graph g's vertex v becomes arena vertex
    vbase[g] + v.  Returns (arena Graph, vbase int32[len(graphs) + 1])."""
    vbase = np.zeros(len(graphs) + 1, dtype=np.int64)
    ebase = np.zeros(len(graphs) + 1, dtype=np.int64)
    for i, g in enumerate(graphs):
        vbase[i + 1] = vbase[i] + g.n
        ebase[i + 1] = ebase[i] + g.m
    if vbase[-1] >= 2**31 or ebase[-1] >= 2**31:
        raise ValueError("arena exceeds int32 indexing")
    rp = np.empty(vbase[-1] + 1, dtype=np.int32)
    col = np.empty(ebase[-1], dtype=np.int32)
    weighted = all(g.weights is not None for g in graphs)
    w = np.empty(ebase[-1], dtype=np.uint32) if weighted else None
    for i, g in enumerate(graphs):
        rp[vbase[i]:vbase[i + 1]] = g.row_ptr[:-1] + ebase[i]
        col[ebase[i]:ebase[i + 1]] = g.col_idx + vbase[i]
        if weighted:
            w[ebase[i]:ebase[i + 1]] = g.weights
    rp[-1] = ebase[-1]
    return Graph(rp, col, w, "arena"), vbase.astype(np.int32)


def batch_workload(seed: int = 40, ngraphs: int = 64, sources_per_graph: int = 8,
                   scales=(10, 18), edgefactors=(8, 32)):
    """The batched workload: ngraphs R-MAT graphs with scale ~ U{scales} and
    edgefactor ~ U{edgefactors} drawn from `seed`, graph g generated with seed
    1000 + g (permuted), sources_per_graph sources each from seed 2000 + g.
    Returns (graphs, [(graph, source)])."""
    rng = np.random.default_rng(seed)
    sc = rng.integers(scales[0], scales[1] + 1, size=ngraphs)
    ef = rng.integers(edgefactors[0], edgefactors[1] + 1, size=ngraphs)
    graphs, queries = [], []
    for g in range(ngraphs):
        gr = rmat(int(sc[g]), int(ef[g]), 1000 + g, perm_seed=7000 + g,
                  name=f"rmat-s{sc[g]}-ef{ef[g]}-seed{1000 + g}")
        graphs.append(gr)
        for s in sample_sources(gr, sources_per_graph, 2000 + g):
            queries.append((g, int(s)))
    return graphs, queries
