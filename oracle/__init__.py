"""CPU oracle for nested-parallel BFS / SSSP.

TEST INFRASTRUCTURE ONLY.  Only the tests, ``__graft_entry__.smoke()`` and
the CPU-baseline leg of ``bench.py`` may import this package.  The GPU
library never links, loads or calls it, and it imports nothing from the GPU
path (the seeded input generators are the only shared module, and they hold
none of the traversal arithmetic).

Contents
  bfs(g, src)            plain FIFO BFS (C, ``oracle.c``)
  dijkstra(g, src)       binary-heap Dijkstra, uint64 accumulation (C)
  schedule_counts(...)   what thresholding and coarsening do to each level's
                         parents: serial / launched parents, child blocks
                         (numpy, Sec. III-B, III-D and IV-B)
  simulate_nested(...)   pure-Python walk of the thresholded, coarsened,
                         aggregated schedule of one level (Sec. III-V), for
                         small inputs only
"""
from __future__ import annotations

import ctypes
import os
import subprocess

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(_HERE, "liboracle.so")
SRC_PATH = os.path.join(_HERE, "oracle.c")
UNREACHED_LEVEL = -1
UNREACHED_DIST = 0xFFFFFFFF

_lib = None


def build(verbose: bool = False) -> str:
    """Compile oracle.c into liboracle.so with gcc -O3 (single thread)."""
    cmd = ["gcc", "-O3", "-fPIC", "-shared", "-o", LIB_PATH + ".tmp", SRC_PATH]
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
    lib.oracle_bfs.restype = ctypes.c_int32
    lib.oracle_bfs.argtypes = [ctypes.c_int32, i32p, i32p, ctypes.c_int32, i32p]
    lib.oracle_dijkstra.restype = ctypes.c_int64
    lib.oracle_dijkstra.argtypes = [ctypes.c_int32, i32p, i32p, u32p, ctypes.c_int32, u32p]
    _lib = lib
    return lib


def _p(a, t):
    return a.ctypes.data_as(ctypes.POINTER(t))


def bfs(g, src: int):
    """Returns (level int32[n], depth).  depth = number of non-empty levels."""
    rp = np.ascontiguousarray(g.row_ptr, dtype=np.int32)
    col = np.ascontiguousarray(g.col_idx, dtype=np.int32)
    if col.size == 0:
        col = np.zeros(1, dtype=np.int32)
    level = np.empty(g.n, dtype=np.int32)
    depth = _load().oracle_bfs(g.n, _p(rp, ctypes.c_int32), _p(col, ctypes.c_int32), int(src),
                               _p(level, ctypes.c_int32))
    if depth < 0:
        raise ValueError(f"oracle_bfs failed ({depth})")
    return level, int(depth)


def dijkstra(g, src: int) -> np.ndarray:
    """Returns dist uint32[n]; 0xFFFFFFFF marks unreachable vertices."""
    rp = np.ascontiguousarray(g.row_ptr, dtype=np.int32)
    col = np.ascontiguousarray(g.col_idx, dtype=np.int32)
    w = np.ascontiguousarray(g.weights, dtype=np.uint32)
    if col.size == 0:
        col = np.zeros(1, dtype=np.int32)
        w = np.zeros(1, dtype=np.uint32)
    dist = np.empty(g.n, dtype=np.uint32)
    rc = _load().oracle_dijkstra(g.n, _p(rp, ctypes.c_int32), _p(col, ctypes.c_int32),
                                 _p(w, ctypes.c_uint32), int(src), _p(dist, ctypes.c_uint32))
    if rc < 0:
        raise ValueError(f"oracle_dijkstra failed ({rc})")
    return dist


def _ceil_div(a, b):
    return (a + b - 1) // b


def schedule_counts(g, level: np.ndarray, threshold: int, child_block: int, coarsen: int,
                    flat: bool = False) -> dict:
    """Counts of a level-synchronous nested BFS under thresholding and coarsening.

    Every reached vertex u is a parent thread exactly once (in the level after
    its own).  Its number of child threads is its degree (Sec. III-D: the
    desired thread count, not gDim * bDim).  Sec. III-B: the child is launched
    only when that count is at least the threshold, otherwise the parent runs
    it serially; a parent with no child threads launches nothing (Sec. V-A:
    only threads with a non-zero grid dimension take part).  Sec. IV-B: the
    launched grid has gDim = ceil(deg / bDim) blocks and is coarsened to
    ceil(gDim / CF) blocks.  ``flat`` is the version without nesting: every
    parent with work walks its neighbours itself.
    """
    deg = np.diff(g.row_ptr).astype(np.int64)[level >= 0]
    has = deg > 0
    if flat:
        serial = has
        launch = np.zeros_like(has)
    else:
        launch = deg >= max(threshold, 1)
        serial = has & ~launch
    gdim = _ceil_div(deg, child_block)
    cgdim = _ceil_div(gdim, coarsen)
    return {
        "frontier_total": int(deg.size),
        "serial_parents": int(serial.sum()),
        "records": int(launch.sum()),
        "child_blocks": int(cgdim[launch].sum()),
        "edges_serial": int(deg[serial].sum()),
        "edges_child": int(deg[launch].sum()),
    }


def simulate_nested(row_ptr, frontier, threshold: int, child_block: int, coarsen: int,
                    group_parents: int):
    """One level of the transformed nested schedule, walked in pure Python.

    Returns (serial, child, grids): ``serial`` lists (parent, edge) pairs run
    inside the parent thread, ``child`` lists (parent, edge) pairs run by
    aggregated, coarsened child blocks, ``grids`` lists (records, blocks) of
    each aggregated grid launched (a group with at least one launching
    parent).  Steps, in the order Sec. VI applies them:

      thresholding (Sec. III-B): deg < T -> serial loop over the child
        threads in the parent; otherwise a launch of gDim = ceil(deg/bDim)
        blocks of bDim threads;
      coarsening (Sec. IV-B): the launch becomes ceil(gDim/CF) blocks, each
        running CF original blocks in a loop;
      aggregation (Sec. II-B, V-A): parents are grouped ``group_parents`` at a
        time; within a group each launching parent stores its arguments and
        the exclusive scan of the coarsened grid sizes; one aggregated grid of
        the summed size is launched; each of its blocks finds its parent by a
        binary search of the scanned sizes and runs the coarsening loop.
    Small inputs only (tests).
    """
    rp = [int(x) for x in row_ptr]
    serial, child, grids = [], [], []
    for g0 in range(0, len(frontier), group_parents):
        group = [int(u) for u in frontier[g0:g0 + group_parents]]
        records, scanned, total = [], [], 0
        for u in group:
            deg = rp[u + 1] - rp[u]
            if deg == 0:
                continue
            if deg < threshold:
                for b in range(_ceil_div(deg, child_block)):
                    for t in range(child_block):
                        i = b * child_block + t
                        if i < deg:
                            serial.append((u, rp[u] + i))
                continue
            gdim = _ceil_div(deg, child_block)
            cgdim = _ceil_div(gdim, coarsen)
            records.append((u, rp[u], deg, gdim))
            scanned.append(total)
            total += cgdim
        if records:
            grids.append((len(records), total))
        for blk in range(total):
            lo, hi = 0, len(scanned)          # upper bound of blk in scanned
            while lo < hi:
                mid = (lo + hi) // 2
                if scanned[mid] <= blk:
                    lo = mid + 1
                else:
                    hi = mid
            p = lo - 1
            u, start, deg, gdim = records[p]
            j = blk - scanned[p]
            for c in range(coarsen):
                ob = j * coarsen + c
                if ob >= gdim:
                    break
                for t in range(child_block):
                    i = ob * child_block + t
                    if i < deg:
                        child.append((u, start + i))
    return serial, child, grids
