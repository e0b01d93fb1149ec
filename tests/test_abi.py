"""The C ABI without a GPU: every declared symbol is exported, sizes are
consistent, and argument errors come back before anything touches a device."""
import ctypes
import os
import re

import numpy as np
import pytest

from paper_2201_02789_amd import dpo
from paper_2201_02789_amd import graphgen as gg

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
HEADER = os.path.join(ROOT, "include", "dpo.h")


def declared_functions():
    text = open(HEADER).read()
    text = re.sub(r"/\*.*?\*/", "", text, flags=re.S)
    names = re.findall(r"^\s*(?:[A-Za-z_][\w\s\*]*?)\b(dpo_\w+)\s*\(", text, flags=re.M)
    return sorted(set(names))


def test_library_exports_every_declared_function():
    lib = ctypes.CDLL(dpo.LIB_PATH)
    names = declared_functions()
    assert "dpo_bfs" in names and "dpo_sssp_batch" in names
    for n in names:
        assert hasattr(lib, n), n


def test_strerror_and_defaults():
    assert dpo.dpo_strerror(dpo.DPO_ERR_WORKSPACE) == "workspace too small"
    assert dpo.dpo_strerror(12345) == "unknown status"
    o = dpo.dpo_default_options()
    assert (o.threshold, o.coarsen, o.agg, o.agg_blocks, o.child_block) == (128, 8, 3, 4, 256)


class _G:
    def __init__(self, n, m):
        self.n, self.m = n, m


def test_workspace_bytes_grows_and_rejects_bad_options():
    a = dpo.dpo_workspace_bytes(_G(1000, 10), dpo.Options())
    b = dpo.dpo_workspace_bytes(_G(100000, 10), dpo.Options())
    assert 0 < a < b
    assert dpo.dpo_workspace_bytes(_G(1000, 10), dpo.Options(coarsen=3)) == 0
    assert dpo.dpo_workspace_bytes(_G(1000, 10), dpo.Options(child_block=100)) == 0
    assert dpo.dpo_workspace_bytes(_G(1000, 10), dpo.Options(dyn_share=101)) == 0
    assert dpo.dpo_workspace_bytes(_G(1000, 10), dpo.Options(dyn_share=-1)) == 0
    assert dpo.dpo_workspace_bytes(_G(1000, 10), dpo.Options(claim_hint=3)) == 0
    assert dpo.dpo_workspace_bytes(_G(1000, 10), dpo.Options(claim_hint=-1)) == 0
    for h in (dpo.DPO_HINT_AUTO, dpo.DPO_HINT_ON, dpo.DPO_HINT_OFF):
        assert dpo.dpo_workspace_bytes(_G(1000, 10), dpo.Options(claim_hint=h)) > 0
    assert dpo.dpo_workspace_bytes(_G(0, 0), dpo.Options()) == 0
    # naive keeps one descriptor slot per parent: the largest workspace
    assert dpo.dpo_workspace_bytes(_G(10**5, 1), dpo.Options.naive()) > b


def _call_bfs(n, m, src, opts, ws_bytes, levels=1, ws=1):
    csr = dpo._Csr(n, m, 8, 8 if m else None, None)
    return dpo.lib().dpo_bfs(ctypes.byref(csr) if n >= 0 else None, src, ctypes.byref(opts.c()),
                             ctypes.c_void_p(levels), ctypes.c_void_p(ws), ws_bytes, None, None)


def test_argument_errors_before_any_device_work():
    o = dpo.Options()
    big = 1 << 40
    assert _call_bfs(100, 10, 100, o, big) == dpo.DPO_ERR_SOURCE
    assert _call_bfs(100, 10, -1, o, big) == dpo.DPO_ERR_SOURCE
    assert _call_bfs(100, 10, 0, o, 16) == dpo.DPO_ERR_WORKSPACE
    assert _call_bfs(100, 10, 0, dpo.Options(coarsen=5), big) == dpo.DPO_ERR_ARG
    assert _call_bfs(100, 10, 0, o, big, levels=0) == dpo.DPO_ERR_ARG
    assert _call_bfs(0, 0, 0, o, big) == dpo.DPO_ERR_ARG
    assert dpo.lib().dpo_bfs(None, 0, ctypes.byref(o.c()), ctypes.c_void_p(1), ctypes.c_void_p(1),
                             big, None, None) == dpo.DPO_ERR_ARG
    # SSSP needs weights
    csr = dpo._Csr(100, 10, 8, 8, None)
    assert dpo.lib().dpo_sssp(ctypes.byref(csr), 0, ctypes.byref(o.c()), ctypes.c_void_p(1),
                              ctypes.c_void_p(1), big, None, None) == dpo.DPO_ERR_ARG


def _host_arena(graphs):
    ar, vb = gg.pack_arena(graphs)
    c = dpo._Arena(len(graphs), vb.ctypes.data_as(ctypes.POINTER(ctypes.c_int32)),
                   dpo._Csr(ar.n, ar.m, 8, 8, None))
    return c, vb


def test_batch_slot_layout():
    graphs = [gg.path_graph(5), gg.star_graph(40), gg.complete_graph(33)]
    c, vb = _host_arena(graphs)
    qs = [(1, 0), (0, 4), (2, 2), (1, 7)]
    qa = dpo._queries(qs)
    slot0 = np.zeros(len(qs) + 1, dtype=np.int64)
    tot = dpo.lib().dpo_batch_slots(ctypes.byref(c), qa, len(qs),
                                    slot0.ctypes.data_as(ctypes.POINTER(ctypes.c_int64)))
    sizes = [64, 32, 64, 64]  # n rounded up to 32 per query, in query order
    assert tot == sum(sizes)
    assert slot0.tolist() == [0, 64, 96, 160, 224]
    bad = dpo._queries([(3, 0)])
    assert dpo.lib().dpo_batch_slots(ctypes.byref(c), bad, 1, None) == -1


def test_batch_argument_errors():
    graphs = [gg.path_graph(5), gg.star_graph(40)]
    c, vb = _host_arena(graphs)
    o = dpo.Options()
    ob = (dpo._Options * 1)(o.c())
    big = 1 << 40
    f = dpo.lib().dpo_bfs_batch
    qa = dpo._queries([(0, 5)])  # source outside graph 0
    assert f(ctypes.byref(c), qa, 1, ob, 1, ctypes.c_void_p(1), ctypes.c_void_p(1), big, None,
             None) == dpo.DPO_ERR_SOURCE
    qa = dpo._queries([(1, 3, 2)])  # bucket 2 of 1
    assert f(ctypes.byref(c), qa, 1, ob, 1, ctypes.c_void_p(1), ctypes.c_void_p(1), big, None,
             None) == dpo.DPO_ERR_ARG
    qa = dpo._queries([(1, 3)])
    assert f(ctypes.byref(c), qa, 1, ob, 1, ctypes.c_void_p(1), ctypes.c_void_p(1), 64, None,
             None) == dpo.DPO_ERR_WORKSPACE
    vb_bad = np.array([0, 5, 44], dtype=np.int32)  # does not end at n = 45
    c.graph_vbase = vb_bad.ctypes.data_as(ctypes.POINTER(ctypes.c_int32))
    assert f(ctypes.byref(c), qa, 1, ob, 1, ctypes.c_void_p(1), ctypes.c_void_p(1), big, None,
             None) == dpo.DPO_ERR_ARG


def test_noalloc_rejects_before_any_device_work():
    """The no-allocation entry point checks its arguments and the static
    workspace bound on the host: a graph whose workspace exceeds the static
    array is refused with DPO_ERR_WORKSPACE, as are bad sources and options."""
    f = dpo.lib().dpo_bfs_noalloc
    o = dpo.Options()

    def call(n, m, src, opts=o, levels=1):
        csr = dpo._Csr(n, m, 8, 8 if m else None, None)
        return f(ctypes.byref(csr), src, ctypes.byref(opts.c()), ctypes.c_void_p(levels), None)

    assert call(1_000_000, 10, 0) == dpo.DPO_ERR_WORKSPACE
    assert call(800_000, 10, 0, dpo.Options.naive()) == dpo.DPO_ERR_WORKSPACE
    assert call(1000, 10, 1000) == dpo.DPO_ERR_SOURCE
    assert call(1000, 10, 0, dpo.Options(child_block=100)) == dpo.DPO_ERR_ARG
    assert call(1000, 10, 0, levels=0) == dpo.DPO_ERR_ARG
    # the bound is the ordinary workspace size
    assert dpo.dpo_workspace_bytes(_G(900_000, 1), o) <= dpo.NOALLOC_SCRATCH_BYTES
    assert dpo.dpo_workspace_bytes(_G(1_000_000, 1), o) > dpo.NOALLOC_SCRATCH_BYTES
