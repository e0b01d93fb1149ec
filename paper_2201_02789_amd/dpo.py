"""ctypes binding of libdpo.so (C ABI declared in include/dpo.h).

Argument marshalling only: every step of a traversal runs in the HIP kernels
of libdpo.so.  PyTorch provides device memory and the stream.  There is no
CPU fallback: if the library is missing, every call raises.
"""
from __future__ import annotations

import ctypes
import os
from dataclasses import dataclass, fields

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(_HERE, "libdpo.so")

DPO_OK = 0
DPO_ERR_ARG = -1
DPO_ERR_SOURCE = -2
DPO_ERR_WORKSPACE = -3
DPO_ERR_CAPACITY = -4
DPO_ERR_TIMEOUT = -5
DPO_ERR_HIP = -6
DPO_ERR_UNSUPPORTED = -7

DPO_MODE_NESTED = 0
DPO_MODE_FLAT = 1
DPO_AGG_NONE = 0
DPO_AGG_WAVE = 1
DPO_AGG_BLOCK = 2
DPO_AGG_MULTIBLOCK = 3
DPO_AGG_GRID = 4
DPO_HINT_AUTO = 0
DPO_HINT_ON = 1
DPO_HINT_OFF = 2

UNREACHED_LEVEL = -1
UNREACHED_DIST = 0xFFFFFFFF


class DpoError(RuntimeError):
    def __init__(self, status: int, what: str = ""):
        self.status = status
        super().__init__(f"{what}: {dpo_strerror(status)} ({status})")


class _Options(ctypes.Structure):
    _fields_ = [("mode", ctypes.c_int32), ("threshold", ctypes.c_int32),
                ("coarsen", ctypes.c_int32), ("agg", ctypes.c_int32),
                ("agg_blocks", ctypes.c_int32), ("child_block", ctypes.c_int32),
                ("steps_per_replay", ctypes.c_int32), ("agg_threshold", ctypes.c_int32),
                ("split_min", ctypes.c_int32), ("serial_wave", ctypes.c_int32),
                ("dyn_share", ctypes.c_int32), ("claim_hint", ctypes.c_int32)]


class _Csr(ctypes.Structure):
    _fields_ = [("n", ctypes.c_int32), ("m", ctypes.c_int32), ("row_ptr", ctypes.c_void_p),
                ("col_idx", ctypes.c_void_p), ("weights", ctypes.c_void_p)]


class _Arena(ctypes.Structure):
    _fields_ = [("ngraphs", ctypes.c_int32), ("graph_vbase", ctypes.POINTER(ctypes.c_int32)),
                ("csr", _Csr)]


class _Query(ctypes.Structure):
    _fields_ = [("graph", ctypes.c_int32), ("source", ctypes.c_int32), ("bucket", ctypes.c_int32)]


class _Stats(ctypes.Structure):
    _fields_ = [("levels", ctypes.c_int32), ("reserved", ctypes.c_int32),
                ("frontier_total", ctypes.c_int64), ("serial_parents", ctypes.c_int64),
                ("records", ctypes.c_int64), ("child_blocks", ctypes.c_int64),
                ("edges_serial", ctypes.c_int64), ("edges_child", ctypes.c_int64),
                ("descriptors", ctypes.c_int64)]


@dataclass
class Options:
    """Mirror of dpo_options.  Defaults = dpo_default_options()."""
    mode: int = DPO_MODE_NESTED
    threshold: int = 128
    coarsen: int = 8
    agg: int = DPO_AGG_MULTIBLOCK
    agg_blocks: int = 4
    child_block: int = 256
    steps_per_replay: int = 0
    agg_threshold: int = 0
    split_min: int = 65536
    serial_wave: int = 1
    dyn_share: int = 0
    claim_hint: int = 0  # DPO_HINT_AUTO

    def c(self) -> _Options:
        return _Options(*(int(getattr(self, f.name)) for f in fields(self)))

    @staticmethod
    def flat(**kw) -> "Options":
        return Options(mode=DPO_MODE_FLAT, **kw)

    @staticmethod
    def naive(**kw) -> "Options":
        """One child grid per launching parent, no thresholding or coarsening
        (the paper's plain dynamic-parallelism version)."""
        kw.setdefault("threshold", 0)
        kw.setdefault("coarsen", 1)
        return Options(agg=DPO_AGG_NONE, **kw)

    def label(self) -> str:
        if self.mode == DPO_MODE_FLAT:
            return "flat"
        g = {0: "none", 1: "wave", 2: "block", 3: f"{self.agg_blocks}-block", 4: "grid"}[self.agg]
        at = f"-A{self.agg_threshold}" if self.agg_threshold else ""
        sm = f"-S{self.split_min}" if self.split_min != 65536 else ""
        sl = "-lane" if not self.serial_wave else ""
        sl += f"-D{self.dyn_share}" if self.dyn_share else ""
        sl += {DPO_HINT_ON: "-H1", DPO_HINT_OFF: "-H0"}.get(self.claim_hint, "")
        cb = f"-CB{self.child_block}" if self.child_block != 256 else ""
        return f"T{self.threshold}-CF{self.coarsen}-{g}{cb}{at}{sm}{sl}"


_lib = None


def lib():
    """The loaded libdpo.so.  Raises if it has not been built."""
    global _lib
    if _lib is not None:
        return _lib
    if not os.path.exists(LIB_PATH):
        raise RuntimeError(f"{LIB_PATH} is missing: build it with __graft_entry__.build() "
                           "(there is no CPU fallback)")
    L = ctypes.CDLL(LIB_PATH)
    L.dpo_default_options.restype = None
    L.dpo_default_options.argtypes = [ctypes.POINTER(_Options)]
    L.dpo_workspace_bytes.restype = ctypes.c_size_t
    L.dpo_workspace_bytes.argtypes = [ctypes.POINTER(_Csr), ctypes.POINTER(_Options)]
    for name in ("dpo_bfs", "dpo_sssp"):
        f = getattr(L, name)
        f.restype = ctypes.c_int32
        f.argtypes = [ctypes.POINTER(_Csr), ctypes.c_int32, ctypes.POINTER(_Options),
                      ctypes.c_void_p, ctypes.c_void_p, ctypes.c_size_t, ctypes.c_void_p,
                      ctypes.POINTER(_Stats)]
    L.dpo_bfs_noalloc.restype = ctypes.c_int32
    L.dpo_bfs_noalloc.argtypes = [ctypes.POINTER(_Csr), ctypes.c_int32, ctypes.POINTER(_Options),
                                  ctypes.c_void_p, ctypes.c_void_p]
    L.dpo_traverse_timed.restype = ctypes.c_int32
    L.dpo_traverse_timed.argtypes = [ctypes.c_int32, ctypes.POINTER(_Csr), ctypes.c_int32,
                                     ctypes.POINTER(_Options), ctypes.c_void_p, ctypes.c_void_p,
                                     ctypes.c_size_t, ctypes.c_void_p, ctypes.c_void_p,
                                     ctypes.c_size_t]
    L.dpo_batch_slots.restype = ctypes.c_int64
    L.dpo_batch_slots.argtypes = [ctypes.POINTER(_Arena), ctypes.POINTER(_Query), ctypes.c_int32,
                                  ctypes.POINTER(ctypes.c_int64)]
    L.dpo_batch_workspace_bytes.restype = ctypes.c_size_t
    L.dpo_batch_workspace_bytes.argtypes = [ctypes.POINTER(_Arena), ctypes.POINTER(_Query),
                                            ctypes.c_int32, ctypes.POINTER(_Options)]
    for name in ("dpo_bfs_batch", "dpo_sssp_batch"):
        f = getattr(L, name)
        f.restype = ctypes.c_int32
        f.argtypes = [ctypes.POINTER(_Arena), ctypes.POINTER(_Query), ctypes.c_int32,
                      ctypes.POINTER(_Options), ctypes.c_int32, ctypes.c_void_p, ctypes.c_void_p,
                      ctypes.c_size_t, ctypes.c_void_p, ctypes.POINTER(_Stats)]
    L.dpo_engine_workspace_bytes.restype = ctypes.c_size_t
    L.dpo_engine_workspace_bytes.argtypes = [ctypes.POINTER(_Options), ctypes.c_int32,
                                             ctypes.c_int64]
    L.dpo_engine_create.restype = ctypes.c_int32
    L.dpo_engine_create.argtypes = [ctypes.POINTER(_Arena), ctypes.c_int32, ctypes.POINTER(_Options),
                                    ctypes.c_int32, ctypes.POINTER(ctypes.c_int32), ctypes.c_int32,
                                    ctypes.c_int64, ctypes.c_void_p, ctypes.c_size_t,
                                    ctypes.c_void_p, ctypes.c_void_p, ctypes.POINTER(ctypes.c_void_p)]
    L.dpo_engine_submit.restype = ctypes.c_int32
    L.dpo_engine_submit.argtypes = [ctypes.c_void_p, ctypes.c_int32, ctypes.c_int32,
                                    ctypes.c_void_p, ctypes.POINTER(ctypes.c_uint64)]
    L.dpo_engine_step.restype = ctypes.c_int32
    L.dpo_engine_step.argtypes = [ctypes.c_void_p, ctypes.POINTER(ctypes.c_int32),
                                  ctypes.POINTER(ctypes.c_int32)]
    L.dpo_engine_poll.restype = ctypes.c_int32
    L.dpo_engine_poll.argtypes = [ctypes.c_void_p, ctypes.POINTER(ctypes.c_uint64), ctypes.c_int32]
    L.dpo_engine_destroy.restype = None
    L.dpo_engine_destroy.argtypes = [ctypes.c_void_p]
    L.dpo_strerror.restype = ctypes.c_char_p
    L.dpo_strerror.argtypes = [ctypes.c_int32]
    _lib = L
    return L


def dpo_strerror(status: int) -> str:
    return lib().dpo_strerror(int(status)).decode()


def dpo_default_options() -> Options:
    o = _Options()
    lib().dpo_default_options(ctypes.byref(o))
    return Options(*(getattr(o, f) for f, _ in _Options._fields_))


class DeviceGraph:
    """Int32 CSR resident in device memory (torch tensors on ``device``)."""

    def __init__(self, row_ptr, col_idx, weights=None):
        self.row_ptr = row_ptr
        self.col_idx = col_idx
        self.weights = weights
        self.n = int(row_ptr.numel() - 1)
        self.m = int(col_idx.numel())

    @classmethod
    def from_host(cls, g, device="cuda"):
        import torch
        rp = torch.from_numpy(np.ascontiguousarray(g.row_ptr, dtype=np.int32)).to(device)
        col = torch.from_numpy(np.ascontiguousarray(g.col_idx, dtype=np.int32)).to(device)
        w = None
        if g.weights is not None:
            w = torch.from_numpy(np.ascontiguousarray(g.weights, dtype=np.uint32).view(np.int32))
            w = w.to(device)
        return cls(rp, col, w)

    def csr(self) -> _Csr:
        return _Csr(self.n, self.m, self.row_ptr.data_ptr(),
                    self.col_idx.data_ptr() if self.m else None,
                    self.weights.data_ptr() if self.weights is not None and self.m else None)


def dpo_workspace_bytes(graph: DeviceGraph, opts: Options) -> int:
    csr = _Csr(graph.n, graph.m, None, None, None)
    return int(lib().dpo_workspace_bytes(ctypes.byref(csr), ctypes.byref(opts.c())))


def _stream_ptr(stream):
    import torch
    if stream is None:
        stream = torch.cuda.current_stream()
    return ctypes.c_void_p(stream.cuda_stream)


def _traverse(fn, what, graph, source, opts, out, ws, stream, stats):
    st = _Stats() if stats else None
    rc = fn(ctypes.byref(graph.csr()), int(source), ctypes.byref(opts.c()),
            ctypes.c_void_p(out.data_ptr()), ctypes.c_void_p(ws.data_ptr()),
            ctypes.c_size_t(ws.numel() * ws.element_size()), _stream_ptr(stream),
            ctypes.byref(st) if st is not None else None)
    if rc != DPO_OK:
        raise DpoError(rc, what)
    if st is None:
        return None
    return {f: int(getattr(st, f)) for f, _ in _Stats._fields_ if f != "reserved"}


def dpo_bfs(graph: DeviceGraph, source: int, opts: Options, levels, ws, stream=None,
            stats: bool = False):
    """levels: int32 device tensor [n] (written).  ws: device byte tensor of at
    least dpo_workspace_bytes(graph, opts).  Returns counters if ``stats``."""
    return _traverse(lib().dpo_bfs, "dpo_bfs", graph, source, opts, levels, ws, stream, stats)


def dpo_sssp(graph: DeviceGraph, source: int, opts: Options, dist, ws, stream=None,
             stats: bool = False):
    """dist: int32/uint32 device tensor [n] (written as uint32)."""
    return _traverse(lib().dpo_sssp, "dpo_sssp", graph, source, opts, dist, ws, stream, stats)


NOALLOC_SCRATCH_BYTES = 64 << 20  # DPO_NOALLOC_SCRATCH_BYTES


def dpo_bfs_noalloc(graph: DeviceGraph, source: int, opts: Options, levels, stream=None):
    """dpo_bfs with the library's static device workspace (no allocation; for
    graphs whose workspace fits NOALLOC_SCRATCH_BYTES)."""
    rc = lib().dpo_bfs_noalloc(ctypes.byref(graph.csr()), int(source), ctypes.byref(opts.c()),
                               ctypes.c_void_p(levels.data_ptr()), _stream_ptr(stream))
    if rc != DPO_OK:
        raise DpoError(rc, "dpo_bfs_noalloc")


TIMING_BYTES = 64 * 4 * 4096 * 8 * 8  # DPO_TIMING_BYTES
TIMING_PHASES = ("parent", "aggregation", "launch", "disaggregation", "child")


def dpo_traverse_timed(kind: str, graph: DeviceGraph, source: int, opts: Options, out, ws,
                       timing, stream=None):
    """dpo_bfs / dpo_sssp with the timed kernels; timing: device tensor of at
    least TIMING_BYTES bytes, filled with the per-workgroup phase rows."""
    rc = lib().dpo_traverse_timed(0 if kind == "bfs" else 1, ctypes.byref(graph.csr()), int(source),
                                  ctypes.byref(opts.c()), ctypes.c_void_p(out.data_ptr()),
                                  ctypes.c_void_p(ws.data_ptr()),
                                  ctypes.c_size_t(ws.numel() * ws.element_size()),
                                  _stream_ptr(stream), ctypes.c_void_p(timing.data_ptr()),
                                  ctypes.c_size_t(timing.numel() * timing.element_size()))
    if rc != DPO_OK:
        raise DpoError(rc, "dpo_traverse_timed")


def alloc_workspace(graph: DeviceGraph, opts: Options, device="cuda"):
    import torch
    return torch.empty(dpo_workspace_bytes(graph, opts), dtype=torch.uint8, device=device)


def bfs(graph: DeviceGraph, source: int, opts: Options | None = None, stats: bool = False):
    """Convenience: allocates the output and workspace, returns (levels, stats)."""
    import torch
    opts = opts or Options()
    levels = torch.empty(graph.n, dtype=torch.int32, device=graph.row_ptr.device)
    ws = alloc_workspace(graph, opts, graph.row_ptr.device)
    st = dpo_bfs(graph, source, opts, levels, ws, stats=stats)
    return levels, st


def sssp(graph: DeviceGraph, source: int, opts: Options | None = None, stats: bool = False):
    """Convenience: allocates the output and workspace, returns (dist, stats);
    dist is an int32 tensor holding the uint32 bit patterns."""
    import torch
    opts = opts or Options()
    dist = torch.empty(graph.n, dtype=torch.int32, device=graph.row_ptr.device)
    ws = alloc_workspace(graph, opts, graph.row_ptr.device)
    st = dpo_sssp(graph, source, opts, dist, ws, stats=stats)
    return dist, st


class DeviceArena:
    """Graphs packed in one CSR arena on the device (see graphgen.pack_arena)."""

    def __init__(self, arena_graph, vbase, device="cuda"):
        self.graph = DeviceGraph.from_host(arena_graph, device)
        self.vbase = np.ascontiguousarray(vbase, dtype=np.int32)
        self.ngraphs = int(self.vbase.size - 1)

    def c(self) -> _Arena:
        return _Arena(self.ngraphs, self.vbase.ctypes.data_as(ctypes.POINTER(ctypes.c_int32)),
                      self.graph.csr())


def _queries(queries):
    """[(graph, source[, bucket])] -> ctypes array of dpo_query."""
    arr = (_Query * len(queries))()
    for i, q in enumerate(queries):
        arr[i] = _Query(int(q[0]), int(q[1]), int(q[2]) if len(q) > 2 else 0)
    return arr


def dpo_batch_slots(arena: DeviceArena, queries):
    """(total slots, slot0 int64[nq + 1]) of the batch output layout."""
    qa = _queries(queries)
    slot0 = np.zeros(len(queries) + 1, dtype=np.int64)
    tot = lib().dpo_batch_slots(ctypes.byref(arena.c()), qa, len(queries),
                                slot0.ctypes.data_as(ctypes.POINTER(ctypes.c_int64)))
    if tot < 0:
        raise DpoError(DPO_ERR_ARG, "dpo_batch_slots")
    return int(tot), slot0


def dpo_batch_workspace_bytes(arena: DeviceArena, queries, opts: Options) -> int:
    qa = _queries(queries)
    return int(lib().dpo_batch_workspace_bytes(ctypes.byref(arena.c()), qa, len(queries),
                                               ctypes.byref(opts.c())))


def _batch(fn, what, arena, queries, bucket_opts, out, ws, stream, stats):
    qa = _queries(queries)
    ob = (_Options * len(bucket_opts))(*[o.c() for o in bucket_opts])
    st = _Stats() if stats else None
    rc = fn(ctypes.byref(arena.c()), qa, len(queries), ob, len(bucket_opts),
            ctypes.c_void_p(out.data_ptr()), ctypes.c_void_p(ws.data_ptr()),
            ctypes.c_size_t(ws.numel() * ws.element_size()), _stream_ptr(stream),
            ctypes.byref(st) if st is not None else None)
    if rc != DPO_OK:
        raise DpoError(rc, what)
    if st is None:
        return None
    return {f: int(getattr(st, f)) for f, _ in _Stats._fields_ if f != "reserved"}


def dpo_bfs_batch(arena: DeviceArena, queries, bucket_opts, levels, ws, stream=None,
                  stats: bool = False):
    """queries: [(graph, source[, bucket])]; bucket_opts: [Options] (threshold and
    coarsen per bucket, the rest from bucket_opts[0]); levels: int32 device
    tensor of dpo_batch_slots(...)[0] entries."""
    return _batch(lib().dpo_bfs_batch, "dpo_bfs_batch", arena, queries, bucket_opts, levels, ws,
                  stream, stats)


def dpo_sssp_batch(arena: DeviceArena, queries, bucket_opts, dist, ws, stream=None,
                   stats: bool = False):
    return _batch(lib().dpo_sssp_batch, "dpo_sssp_batch", arena, queries, bucket_opts, dist, ws,
                  stream, stats)


class Engine:
    """Continuous-batching engine (dpo_engine_*): kind "bfs" or "sssp".

    Holds references to the arena, its workspace and output scratch so they
    outlive the engine.
    """

    def __init__(self, arena: DeviceArena, kind: str, bucket_opts, graph_bucket=None,
                 max_queries: int = 256, max_slots: int = 1 << 22, stream=None, workspace=None):
        """workspace: optional device uint8 tensor of at least
        dpo_engine_workspace_bytes; allocated here when None."""
        import torch
        self.arena = arena
        self.kind = kind
        self.bucket_opts = list(bucket_opts)
        ob = (_Options * len(self.bucket_opts))(*[o.c() for o in self.bucket_opts])
        self._ob = ob
        nbytes = lib().dpo_engine_workspace_bytes(ctypes.byref(ob[0]), max_queries, max_slots)
        if nbytes == 0:
            raise DpoError(DPO_ERR_ARG, "dpo_engine_workspace_bytes")
        dev = arena.graph.row_ptr.device
        if workspace is None:
            self.ws = torch.empty(nbytes, dtype=torch.uint8, device=dev)
        else:
            if workspace.numel() * workspace.element_size() < nbytes:
                raise DpoError(DPO_ERR_WORKSPACE, "Engine workspace")
            self.ws = workspace
            nbytes = workspace.numel() * workspace.element_size()
        self.scratch = torch.empty(((max_slots + 31) // 32) * 32, dtype=torch.int32, device=dev)
        self.stream = stream if stream is not None else torch.cuda.current_stream()
        self._gb = None
        gbp = None
        if graph_bucket is not None:
            self._gb = np.ascontiguousarray(graph_bucket, dtype=np.int32)
            gbp = self._gb.ctypes.data_as(ctypes.POINTER(ctypes.c_int32))
        self._arena_c = arena.c()
        h = ctypes.c_void_p()
        rc = lib().dpo_engine_create(ctypes.byref(self._arena_c), 0 if kind == "bfs" else 1, ob,
                                     len(self.bucket_opts), gbp, max_queries, max_slots,
                                     ctypes.c_void_p(self.ws.data_ptr()), nbytes,
                                     ctypes.c_void_p(self.scratch.data_ptr()),
                                     ctypes.c_void_p(self.stream.cuda_stream), ctypes.byref(h))
        if rc != DPO_OK:
            raise DpoError(rc, "dpo_engine_create")
        self.h = h
        self._outs = {}

    def submit(self, graph: int, source: int, out) -> int:
        t = ctypes.c_uint64()
        rc = lib().dpo_engine_submit(self.h, int(graph), int(source), ctypes.c_void_p(out.data_ptr()),
                                     ctypes.byref(t))
        if rc != DPO_OK:
            raise DpoError(rc, "dpo_engine_submit")
        self._outs[t.value] = out  # keep the output alive until it is reported
        return int(t.value)

    def step(self):
        run, pend = ctypes.c_int32(), ctypes.c_int32()
        rc = lib().dpo_engine_step(self.h, ctypes.byref(run), ctypes.byref(pend))
        if rc != DPO_OK:
            raise DpoError(rc, "dpo_engine_step")
        return run.value, pend.value

    def poll(self, cap: int = 4096):
        buf = (ctypes.c_uint64 * cap)()
        k = lib().dpo_engine_poll(self.h, buf, cap)
        done = [int(buf[i]) for i in range(k)]
        for t in done:
            self._outs.pop(t, None)
        return done

    def close(self):
        if getattr(self, "h", None):
            lib().dpo_engine_destroy(self.h)
            self.h = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass


def as_uint32(t) -> np.ndarray:
    """Host copy of a device int32 tensor reinterpreted as uint32."""
    return t.cpu().numpy().view(np.uint32)
