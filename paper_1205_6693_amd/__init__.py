"""Python binding of libtruss.so (truss decomposition on MI355X).

Argument marshalling only: every step of support counting and peeling runs in
the library's HIP kernels.  PyTorch supplies device memory and the stream.

Entry points mirror the C ABI in include/truss.h:
    truss_support(graph)              -> (sup int32[m] cuda tensor, triangles)
    truss_decompose(graph, ...)       -> (truss int32[m] cuda tensor, stats dict)
    truss_decompose_noalloc(graph, out, ...) -> (out, stats dict), scratch in a fixed
                                         device array (callers that cannot allocate)
    truss_batch(vtx_off, edge_off, src, dst, ...) -> (truss int32[M], stats dict)
    truss_workspace_size(graph)       -> bytes
    truss_decompose_traced(graph, ...) -> (truss, stats, trace dict)
    truss_upper_bound(graph)          -> psi int32[m] (Procedure 6)
    truss_topdown(graph, t)           -> (top-t classes int32[m], kmin, kmax, stats)
    truss_core_numbers(graph)         -> (core int32[n] cuda tensor, c_max)
    truss_cohesion(graph)             -> Table 6's statistics (dict)
    truss_bottomup(n, src, dst, cap)  -> (truss, lower bound, stats) for a graph in
                                         host memory (numpy int32 arrays)
    truss_cohen(graph)                -> (truss int32[m], stats) by Algorithm 1
    BatchPlan / truss_batch_autotune  -> a replayable batch and its shape
    mlp_forward / mlp_backward / mlp_train / sched_train -> the scheduler network
Graphs are built with Graph.from_edges(n, src, dst) or
Graph.from_csr(n, row_ptr, col) from int32/int64 CUDA tensors.  Tensors are
checked (device, dtype, contiguity, length) before each call, which runs with
their device current and, unless a stream is given, on its current stream.
"""
from __future__ import annotations

import contextlib
import ctypes
import os

_HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(_HERE, "libtruss.so")

TRUSS_VERSION = 10000
OK = 0
E_INVAL, E_TOOBIG, E_ROWPTR, E_RANGE, E_SELFLOOP, E_UNSORTED, E_DUP, E_ASYM, E_NOMEM, E_WORKSPACE, \
    E_DEVICE, E_INTERNAL = range(-1, -13, -1)
FMT_EDGES, FMT_CSR = 0, 1
SUP_AUTO, SUP_HASH, SUP_BSEARCH, SUP_MERGE = 0, 1, 2, 3
PEEL_AUTO, PEEL_SPARSE, PEEL_DENSE = 0, 1, 2
PROBE_AUTO, PROBE_HASH, PROBE_BSEARCH = 0, 1, 2
SHAPE_AUTO, SHAPE_NARROW, SHAPE_WIDE = 0, 1, 2
SCHED_PLAIN, SCHED_HEURISTIC, SCHED_LEARNED = 0, 1, 2
SCHED_PEEL_F, SCHED_PEEL_A, SCHED_SUP_BINS, SCHED_SUP_F, SCHED_SUP_A = 8, 4, 4, 6, 3


class TrussError(RuntimeError):
    def __init__(self, code: int, msg: str):
        super().__init__("truss error %d: %s" % (code, msg))
        self.code = code


class _Graph(ctypes.Structure):
    _fields_ = [("n", ctypes.c_int32), ("fmt", ctypes.c_int32), ("m", ctypes.c_int64),
                ("src", ctypes.c_void_p), ("dst", ctypes.c_void_p),
                ("row_ptr", ctypes.c_void_p), ("col", ctypes.c_void_p)]


class Options(ctypes.Structure):
    _fields_ = [("version", ctypes.c_int32), ("support_strategy", ctypes.c_int32),
                ("peel_mode", ctypes.c_int32), ("scheduler", ctypes.c_int32),
                ("model", ctypes.c_void_p), ("max_subrounds", ctypes.c_int64),
                ("grid_blocks", ctypes.c_int32), ("peel_probe", ctypes.c_int32),
                ("batch_block", ctypes.c_int32), ("batch_ilp", ctypes.c_int32),
                ("model_floats", ctypes.c_int32), ("peel_shape", ctypes.c_int32),
                ("reserved", ctypes.c_int32 * 2)]


class Stats(ctypes.Structure):
    _fields_ = [("n", ctypes.c_int64), ("m", ctypes.c_int64), ("triangles", ctypes.c_int64),
                ("kmax", ctypes.c_int32), ("levels", ctypes.c_int32),
                ("subrounds", ctypes.c_int64), ("peel_work", ctypes.c_int64),
                ("ms_build", ctypes.c_double), ("ms_support", ctypes.c_double),
                ("ms_peel", ctypes.c_double), ("ms_total", ctypes.c_double),
                ("sched_fallback", ctypes.c_int32), ("launches", ctypes.c_int32),
                ("frontier_hist", ctypes.c_int64 * 6), ("heavy_rounds", ctypes.c_int64),
                ("ms_phase", ctypes.c_double * 6), ("ms_peel_kernel", ctypes.c_double),
                ("support_work", ctypes.c_int64)]

    def to_dict(self):
        d = {k: getattr(self, k) for k, _ in self._fields_}
        d["frontier_hist"] = list(self.frontier_hist)
        d["ms_phase"] = list(self.ms_phase)
        return d


class Trace(ctypes.Structure):
    _fields_ = [("level_cap", ctypes.c_int32), ("levels", ctypes.c_int32),
                ("level_feat", ctypes.c_void_p), ("level_ms", ctypes.c_void_p),
                ("level_action", ctypes.c_void_p),
                ("sup_action", ctypes.c_int32 * SCHED_SUP_BINS),
                ("sup_feat", (ctypes.c_float * SCHED_SUP_F) * SCHED_SUP_BINS),
                ("sup_ms", ctypes.c_float * SCHED_SUP_BINS)]


class CohesionStats(ctypes.Structure):
    _fields_ = [("v_t", ctypes.c_int64), ("e_t", ctypes.c_int64), ("kmax", ctypes.c_int32),
                ("pad0", ctypes.c_int32), ("cc_t", ctypes.c_double),
                ("v_c", ctypes.c_int64), ("e_c", ctypes.c_int64), ("cmax", ctypes.c_int32),
                ("pad1", ctypes.c_int32), ("cc_c", ctypes.c_double)]

    def to_dict(self):
        return {"V_T": self.v_t, "E_T": self.e_t, "kmax": self.kmax, "CC_T": self.cc_t,
                "V_C": self.v_c, "E_C": self.e_c, "cmax": self.cmax, "CC_C": self.cc_c}


class BottomUpStats(ctypes.Structure):
    _fields_ = [(k, ctypes.c_int64) for k in (
        "passes", "subgraphs", "phi2_edges", "gnew_edges", "max_subgraph", "candidates", "proc9_calls",
        "proc9_scans", "max_candidate", "device_calls", "bytes_h2d", "bytes_d2h")] + [
        ("kstart", ctypes.c_int32), ("kmax", ctypes.c_int32), ("ms_lower", ctypes.c_double),
        ("ms_bottomup", ctypes.c_double), ("ms_total", ctypes.c_double)]

    def to_dict(self):
        return {k: getattr(self, k) for k, _ in self._fields_}


_lib = None


def load_library():
    """Load libtruss.so; raises if it has not been built (no CPU fallback)."""
    global _lib
    if _lib is not None:
        return _lib
    if not os.path.exists(LIB_PATH):
        raise ImportError("libtruss.so not built: run paper_1205_6693_amd/build.py "
                          "(or __graft_entry__.build())")
    # torch ships its own HIP runtime; load it first so that libtruss binds to
    # the same runtime (one process, one HIP runtime, shared streams and memory)
    import torch  # noqa: F401
    lib = ctypes.CDLL(LIB_PATH)
    vp, i32, i64 = ctypes.c_void_p, ctypes.c_int32, ctypes.c_int64
    gp = ctypes.POINTER(_Graph)
    op = ctypes.POINTER(Options)
    sp = ctypes.POINTER(Stats)
    lib.truss_default_options.argtypes = [op]
    lib.truss_default_options.restype = None
    lib.truss_workspace_size.argtypes = [gp, op, ctypes.POINTER(ctypes.c_size_t)]
    lib.truss_support.argtypes = [gp, vp, ctypes.POINTER(i64), vp, ctypes.c_size_t, vp]
    lib.truss_decompose.argtypes = [gp, vp, op, sp, vp, ctypes.c_size_t, vp]
    lib.truss_decompose_noalloc.argtypes = [gp, vp, op, sp, vp]
    lib.truss_batch_workspace_size.argtypes = [i32, vp, vp, op, ctypes.POINTER(ctypes.c_size_t)]
    lib.truss_batch.argtypes = [i32, vp, vp, vp, vp, vp, op, sp, vp, ctypes.c_size_t, vp]
    lib.truss_batch_plan_create.argtypes = [i32, vp, vp, vp, vp, vp, op, vp, ctypes.c_size_t, vp,
                                            ctypes.POINTER(ctypes.c_void_p)]
    lib.truss_batch_plan_run.argtypes = [vp, sp, vp]
    lib.truss_batch_plan_destroy.argtypes = [vp]
    lib.truss_batch_plan_destroy.restype = None
    lib.truss_batch_autotune.argtypes = [i32, vp, vp, vp, vp, vp, op, vp, ctypes.c_size_t, vp,
                                         ctypes.POINTER(i32), ctypes.POINTER(i32), ctypes.POINTER(ctypes.c_float)]
    tp = ctypes.POINTER(Trace)
    f32, u64, fp = ctypes.c_float, ctypes.c_uint64, ctypes.POINTER(ctypes.c_float)
    szp = ctypes.POINTER(ctypes.c_size_t)
    lib.truss_decompose_traced.argtypes = [gp, vp, op, sp, tp, vp, ctypes.c_size_t, vp]
    lib.truss_upper_bound.argtypes = [gp, vp, vp, ctypes.c_size_t, vp]
    lib.truss_topdown_workspace_size.argtypes = [gp, op, szp]
    lib.truss_topdown.argtypes = [gp, i32, vp, ctypes.POINTER(i32), ctypes.POINTER(i32), op, sp, vp,
                                  ctypes.c_size_t, vp]
    lib.truss_core_workspace_size.argtypes = [gp, szp]
    lib.truss_core_numbers.argtypes = [gp, vp, ctypes.POINTER(i32), vp, ctypes.c_size_t, vp]
    lib.truss_cohesion_workspace_size.argtypes = [gp, szp]
    lib.truss_cohesion.argtypes = [gp, op, ctypes.POINTER(CohesionStats), vp, ctypes.c_size_t, vp]
    lib.truss_cohen_workspace_size.argtypes = [gp, szp]
    lib.truss_cohen.argtypes = [gp, vp, sp, vp, ctypes.c_size_t, vp]
    lib.truss_bottomup_workspace_size.argtypes = [i64, szp]
    lib.truss_bottomup.argtypes = [i32, i64, vp, vp, vp, i64, vp, vp, op, ctypes.POINTER(BottomUpStats), vp,
                                   ctypes.c_size_t, vp]
    lib.truss_mlp_param_count.argtypes = [i32, i32, i32]
    lib.truss_mlp_workspace_size.argtypes = [i32, i32, i32, i32, szp]
    lib.truss_mlp_forward.argtypes = [vp, i32, i32, i32, vp, i32, vp, vp, ctypes.c_size_t, vp]
    lib.truss_mlp_backward.argtypes = [vp, i32, i32, i32, vp, i32, vp, vp, vp, ctypes.c_size_t, vp]
    lib.truss_mlp_train.argtypes = [vp, vp, vp, i32, i32, i32, vp, vp, vp, i32, i32, i32, f32, fp, vp,
                                    ctypes.c_size_t, vp]
    lib.truss_sched_part_floats.argtypes = [i32, i32]
    lib.truss_sched_model_floats.argtypes = [i32]
    lib.truss_sched_train_workspace_size.argtypes = [i32, i32, i32, szp]
    lib.truss_sched_train.argtypes = [i32, vp, vp, i32, i32, i32, f32, u64, vp, fp, vp, ctypes.c_size_t, vp]
    for f in ("truss_workspace_size", "truss_support", "truss_decompose",
              "truss_batch_workspace_size", "truss_batch", "truss_version", "truss_decompose_traced",
              "truss_batch_plan_create", "truss_batch_plan_run", "truss_batch_autotune",
              "truss_upper_bound", "truss_topdown_workspace_size", "truss_topdown",
              "truss_core_workspace_size", "truss_core_numbers", "truss_cohesion_workspace_size",
              "truss_cohesion", "truss_bottomup_workspace_size", "truss_bottomup", "truss_cohen_workspace_size",
              "truss_cohen",
              "truss_mlp_param_count", "truss_mlp_workspace_size", "truss_mlp_forward",
              "truss_mlp_backward", "truss_mlp_train", "truss_sched_part_floats",
              "truss_sched_model_floats", "truss_sched_train_workspace_size", "truss_sched_train"):
        getattr(lib, f).restype = ctypes.c_int
    lib.truss_strerror.argtypes = [ctypes.c_int]
    lib.truss_strerror.restype = ctypes.c_char_p
    lib.truss_last_error.restype = ctypes.c_char_p
    lib.truss_version.argtypes = []
    _lib = lib
    return lib


def _check(rc: int):
    if rc != OK:
        lib = load_library()
        raise TrussError(rc, (lib.truss_last_error() or lib.truss_strerror(rc)).decode())


def _torch():
    import torch
    return torch


def _ptr(t):
    return ctypes.c_void_p(t.data_ptr()) if t is not None and t.numel() else ctypes.c_void_p(0)


def _dev(t, name, dtype, numel=0, device=None):
    """Checks that t is a contiguous CUDA tensor of dtype holding at least
    numel elements (on `device` when given): the library dereferences it on
    the GPU and cannot check any of this itself."""
    torch = _torch()
    if not isinstance(t, torch.Tensor):
        raise TypeError("%s must be a torch tensor" % name)
    if t.device.type != "cuda":
        raise ValueError("%s must be in device memory (got %s)" % (name, t.device))
    if device is not None and t.device != torch.device(device):
        raise ValueError("%s is on %s, the rest on %s" % (name, t.device, device))
    if t.dtype != dtype:
        raise ValueError("%s must be %s (got %s)" % (name, dtype, t.dtype))
    if not t.is_contiguous():
        raise ValueError("%s must be contiguous" % name)
    if t.numel() < numel:
        raise ValueError("%s holds %d elements, %d needed" % (name, t.numel(), numel))
    return t


def _ws_bytes(ws, device=None):
    """Size in bytes of a workspace tensor (any dtype; the library checks
    that it is large enough)."""
    torch = _torch()
    if not isinstance(ws, torch.Tensor) or ws.device.type != "cuda" or not ws.is_contiguous():
        raise ValueError("the workspace must be a contiguous tensor in device memory")
    if device is not None and ws.device != torch.device(device):
        raise ValueError("the workspace is on %s, the rest on %s" % (ws.device, device))
    return ws.numel() * ws.element_size()


@contextlib.contextmanager
def _on(device, stream=None):
    """Makes the tensors' device current for a library call (the library
    launches on the calling thread's current device) and yields the stream
    handle: `stream`, else that device's current stream."""
    torch = _torch()
    dev = torch.device(device)
    if dev.index is None:
        dev = torch.device("cuda", torch.cuda.current_device())
    with torch.cuda.device(dev):
        s = stream if stream is not None else torch.cuda.current_stream(dev)
        if s.device != dev:
            raise ValueError("the stream is on %s, the tensors on %s" % (s.device, dev))
        yield ctypes.c_void_p(s.cuda_stream)


class Graph:
    """A simple undirected graph resident in device memory."""

    def __init__(self, n, m, fmt, src=None, dst=None, row_ptr=None, col=None):
        self.n, self.m, self.fmt = int(n), int(m), fmt
        self.src, self.dst, self.row_ptr, self.col = src, dst, row_ptr, col

    @classmethod
    def from_edges(cls, n, src, dst):
        torch = _torch()
        src = src.to(torch.int32).contiguous()
        dst = dst.to(torch.int32).contiguous()
        if src.shape != dst.shape or src.dim() != 1:
            raise ValueError("src and dst must be 1-D and of equal length")
        _dev(src, "src", torch.int32)
        _dev(dst, "dst", torch.int32, device=src.device)
        return cls(n, src.numel(), FMT_EDGES, src=src, dst=dst)

    @classmethod
    def from_csr(cls, n, row_ptr, col):
        torch = _torch()
        row_ptr = row_ptr.to(torch.int64).contiguous()
        col = col.to(torch.int32).contiguous()
        if col.numel() % 2:
            raise ValueError("a symmetric CSR has an even number of entries")
        if row_ptr.dim() != 1 or row_ptr.numel() != int(n) + 1 or col.dim() != 1:
            raise ValueError("row_ptr must hold n + 1 offsets and col be 1-D")
        _dev(row_ptr, "row_ptr", torch.int64)
        _dev(col, "col", torch.int32, device=row_ptr.device)
        return cls(n, col.numel() // 2, FMT_CSR, row_ptr=row_ptr, col=col)

    def _c(self):
        g = _Graph()
        g.n, g.fmt, g.m = self.n, self.fmt, self.m
        if self.fmt == FMT_EDGES:
            g.src, g.dst = _ptr(self.src).value, _ptr(self.dst).value
        else:
            g.row_ptr, g.col = _ptr(self.row_ptr).value, _ptr(self.col).value
        return g

    @property
    def device(self):
        t = self.src if self.fmt == FMT_EDGES else self.row_ptr
        return t.device


def make_options(support_strategy=SUP_AUTO, peel_mode=PEEL_AUTO, scheduler=SCHED_HEURISTIC,
                 model=None, max_subrounds=0, grid_blocks=0, peel_probe=PROBE_AUTO, batch_block=0,
                 batch_ilp=0, peel_shape=SHAPE_AUTO):
    o = Options()
    load_library().truss_default_options(ctypes.byref(o))
    o.support_strategy, o.peel_mode, o.scheduler = support_strategy, peel_mode, scheduler
    o.peel_probe, o.peel_shape = peel_probe, peel_shape
    o.batch_block, o.batch_ilp = batch_block, batch_ilp
    if model is not None:
        _dev(model, "model", _torch().float32, 4)
        o._model = model  # the options hold its address: keep it alive with them
        # the library reads no float past this count (a truncated model falls back)
        o.model_floats = min(model.numel(), 0x7fffffff)
    o.model = _ptr(model).value if model is not None else None
    o.max_subrounds, o.grid_blocks = max_subrounds, grid_blocks
    return o


def truss_workspace_size(graph: Graph, opts: Options | None = None) -> int:
    lib = load_library()
    b = ctypes.c_size_t(0)
    g = graph._c()
    _check(lib.truss_workspace_size(ctypes.byref(g), ctypes.byref(opts) if opts else None, ctypes.byref(b)))
    return b.value


def workspace(graph: Graph, opts: Options | None = None):
    torch = _torch()
    return torch.empty(truss_workspace_size(graph, opts), dtype=torch.uint8, device=graph.device)


def truss_support(graph: Graph, out=None, ws=None, stream=None):
    """sup(e) of every edge (Definition 1) and the triangle count."""
    torch = _torch()
    lib = load_library()
    if out is None:
        out = torch.empty(graph.m, dtype=torch.int32, device=graph.device)
    _dev(out, "out", torch.int32, graph.m, graph.device)
    if ws is None:
        ws = workspace(graph)
    tri = ctypes.c_int64(0)
    g = graph._c()
    with _on(graph.device, stream) as s_:
        _check(lib.truss_support(ctypes.byref(g), _ptr(out), ctypes.byref(tri), _ptr(ws), _ws_bytes(ws, graph.device),
                                 s_))
    return out, tri.value


def truss_decompose(graph: Graph, opts: Options | None = None, out=None, ws=None, stream=None):
    """Truss number of every edge (Definition 2) and run statistics."""
    torch = _torch()
    lib = load_library()
    if out is None:
        out = torch.empty(graph.m, dtype=torch.int32, device=graph.device)
    _dev(out, "out", torch.int32, graph.m, graph.device)
    if ws is None:
        ws = workspace(graph, opts)
    st = Stats()
    g = graph._c()
    with _on(graph.device, stream) as s_:
        _check(lib.truss_decompose(ctypes.byref(g), _ptr(out), ctypes.byref(opts) if opts else None,
                                   ctypes.byref(st), _ptr(ws), _ws_bytes(ws, graph.device), s_))
    return out, st.to_dict()


NOALLOC_SCRATCH_BYTES = 256 << 20


def truss_decompose_noalloc(graph: Graph, out, opts: Options | None = None, stream=None):
    """truss_decompose with its scratch in the library's fixed device array
    (no workspace, no allocation inside the call; graphs needing more than
    NOALLOC_SCRATCH_BYTES of scratch are refused).  out: caller's int32[m]
    CUDA tensor.  Calls that overlap on one GPU race."""
    torch = _torch()
    lib = load_library()
    _dev(out, "out", torch.int32, graph.m, graph.device)
    st = Stats()
    g = graph._c()
    with _on(graph.device, stream) as s_:
        _check(lib.truss_decompose_noalloc(ctypes.byref(g), _ptr(out), ctypes.byref(opts) if opts else None,
                                           ctypes.byref(st), s_))
    return out, st.to_dict()


def truss_batch_workspace_size(vtx_off, edge_off, opts: Options | None = None) -> int:
    import numpy as np
    lib = load_library()
    vo = np.ascontiguousarray(vtx_off, dtype=np.int64)
    eo = np.ascontiguousarray(edge_off, dtype=np.int64)
    b = ctypes.c_size_t(0)
    _check(lib.truss_batch_workspace_size(len(vo) - 1, vo.ctypes.data, eo.ctypes.data,
                                          ctypes.byref(opts) if opts else None, ctypes.byref(b)))
    return b.value


def _batch_args(vtx_off, edge_off, src, dst, out):
    import numpy as np
    torch = _torch()
    vo = np.ascontiguousarray(vtx_off, dtype=np.int64)
    eo = np.ascontiguousarray(edge_off, dtype=np.int64)
    src = src.to(torch.int32).contiguous()
    dst = dst.to(torch.int32).contiguous()
    if vo.ndim != 1 or vo.size < 1 or eo.shape != vo.shape:
        raise ValueError("vtx_off and edge_off must hold one offset per graph plus one")
    total = int(eo[-1])
    if src.dim() != 1 or src.shape != dst.shape or src.numel() < total:
        raise ValueError("src and dst must be 1-D, of equal length and hold edge_off[-1] edges")
    _dev(src, "src", torch.int32)
    _dev(dst, "dst", torch.int32, device=src.device)
    if out is None:
        out = torch.empty(src.numel(), dtype=torch.int32, device=src.device)
    _dev(out, "out", torch.int32, total, src.device)
    return vo, eo, src, dst, out


def truss_batch(vtx_off, edge_off, src, dst, opts: Options | None = None, out=None, ws=None, stream=None):
    """Truss numbers of many independent graphs packed together (graph-local ids)."""
    torch = _torch()
    lib = load_library()
    vo, eo, src, dst, out = _batch_args(vtx_off, edge_off, src, dst, out)
    if ws is None:
        ws = torch.empty(max(1, truss_batch_workspace_size(vo, eo, opts)), dtype=torch.uint8,
                         device=src.device)
    st = Stats()
    with _on(src.device, stream) as s_:
        _check(lib.truss_batch(len(vo) - 1, vo.ctypes.data, eo.ctypes.data, _ptr(src), _ptr(dst), _ptr(out),
                               ctypes.byref(opts) if opts else None, ctypes.byref(st), _ptr(ws),
                               _ws_bytes(ws, src.device), s_))
    return out, st.to_dict()


class BatchPlan:
    """A reusable batch (truss_batch_plan_*): offsets uploaded once, device work
    captured in a HIP graph and replayed by run()."""

    def __init__(self, vtx_off, edge_off, src, dst, opts: Options | None = None, out=None, ws=None,
                 stream=None):
        torch = _torch()
        lib = load_library()
        self.vo, self.eo, self.src, self.dst, self.out = _batch_args(vtx_off, edge_off, src, dst, out)
        self.opts = opts
        self.ws = ws if ws is not None else torch.empty(
            max(1, truss_batch_workspace_size(self.vo, self.eo, opts)), dtype=torch.uint8, device=self.src.device)
        h = ctypes.c_void_p(0)
        with _on(self.src.device, stream) as s_:
            _check(lib.truss_batch_plan_create(len(self.vo) - 1, self.vo.ctypes.data, self.eo.ctypes.data,
                                               _ptr(self.src), _ptr(self.dst), _ptr(self.out),
                                               ctypes.byref(opts) if opts else None, _ptr(self.ws),
                                               _ws_bytes(self.ws, self.src.device),
                                               s_, ctypes.byref(h)))
        self._h = h

    def run(self, stream=None):
        st = Stats()
        with _on(self.src.device, stream) as s_:
            _check(load_library().truss_batch_plan_run(self._h, ctypes.byref(st), s_))
        return self.out, st.to_dict()

    def close(self):
        if self._h and self._h.value:
            load_library().truss_batch_plan_destroy(self._h)
            self._h = ctypes.c_void_p(0)

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass


def truss_batch_autotune(vtx_off, edge_off, src, dst, opts: Options | None = None, out=None, ws=None,
                         stream=None):
    """Fastest (threads per workgroup, walk entries in flight per thread) for the batch,
    and its sample time in ms."""
    torch = _torch()
    lib = load_library()
    vo, eo, src, dst, out = _batch_args(vtx_off, edge_off, src, dst, out)
    if ws is None:
        ws = torch.empty(max(1, truss_batch_workspace_size(vo, eo, opts)), dtype=torch.uint8, device=src.device)
    tb, tl, ms = ctypes.c_int32(0), ctypes.c_int32(0), ctypes.c_float(0)
    with _on(src.device, stream) as s_:
        _check(lib.truss_batch_autotune(len(vo) - 1, vo.ctypes.data, eo.ctypes.data, _ptr(src), _ptr(dst), _ptr(out),
                                        ctypes.byref(opts) if opts else None, _ptr(ws), _ws_bytes(ws, src.device),
                                        s_,
                                        ctypes.byref(tb), ctypes.byref(tl), ctypes.byref(ms)))
    return tb.value, tl.value, ms.value


def truss_decompose_traced(graph: Graph, opts: Options | None = None, level_cap: int = 4096, out=None,
                           ws=None, stream=None):
    """truss_decompose plus the scheduler's record: per level the raw features,
    the time from the decision to the level's end and the action taken; per
    support bin the features, time and action."""
    torch = _torch()
    lib = load_library()
    if out is None:
        out = torch.empty(graph.m, dtype=torch.int32, device=graph.device)
    _dev(out, "out", torch.int32, graph.m, graph.device)
    if ws is None:
        ws = workspace(graph, opts)
    feat = torch.zeros((max(level_cap, 1), SCHED_PEEL_F), dtype=torch.float32, device=graph.device)
    lms = torch.zeros(max(level_cap, 1), dtype=torch.float32, device=graph.device)
    lact = torch.full((max(level_cap, 1),), -1, dtype=torch.int32, device=graph.device)
    tr = Trace()
    tr.level_cap = level_cap
    tr.level_feat, tr.level_ms, tr.level_action = _ptr(feat).value, _ptr(lms).value, _ptr(lact).value
    st = Stats()
    g = graph._c()
    with _on(graph.device, stream) as s_:
        _check(lib.truss_decompose_traced(ctypes.byref(g), _ptr(out), ctypes.byref(opts) if opts else None,
                                          ctypes.byref(st), ctypes.byref(tr), _ptr(ws), _ws_bytes(ws, graph.device),
                                          s_))
    L = tr.levels
    trace = {"levels": L,
             "level_feat": feat[:L].cpu().numpy(),
             "level_ms": lms[:L].cpu().numpy(),
             "level_action": lact[:L].cpu().numpy(),
             "sup_action": [int(x) for x in tr.sup_action],
             "sup_feat": [[float(v) for v in row] for row in tr.sup_feat],
             "sup_ms": [float(x) for x in tr.sup_ms]}
    return out, st.to_dict(), trace


def _f32(t):
    torch = _torch()
    return t.to(torch.float32).contiguous()


def mlp_param_count(F: int, H: int, O: int) -> int:
    rc = load_library().truss_mlp_param_count(F, H, O)
    if rc < 0:
        _check(rc)
    return rc


def _mlp_ws(F, H, O, B, device):
    torch = _torch()
    b = ctypes.c_size_t(0)
    _check(load_library().truss_mlp_workspace_size(F, H, O, B, ctypes.byref(b)))
    return torch.empty(b.value, dtype=torch.uint8, device=device)


def mlp_forward(params, X, H: int, O: int, stream=None):
    """Network outputs (B x O) for inputs X (B x F), all CUDA float32."""
    torch = _torch()
    X = _f32(X)
    params = _f32(params)
    B, F = X.shape
    _dev(X, "X", torch.float32)
    _dev(params, "params", torch.float32, mlp_param_count(F, H, O), X.device)
    Y = torch.empty((B, O), dtype=torch.float32, device=X.device)
    ws = _mlp_ws(F, H, O, B, X.device)
    with _on(X.device, stream) as s_:
        _check(load_library().truss_mlp_forward(_ptr(params), F, H, O, _ptr(X), B, _ptr(Y), _ptr(ws), _ws_bytes(ws),
                                                s_))
    return Y


def mlp_backward(params, X, dY, H: int, stream=None):
    """d(sum dY * network(X)) / d params."""
    torch = _torch()
    X, dY, params = _f32(X), _f32(dY), _f32(params)
    B, F = X.shape
    O = dY.shape[1]
    if dY.shape != (B, O):
        raise ValueError("dY must be B x O")
    _dev(X, "X", torch.float32)
    _dev(dY, "dY", torch.float32, device=X.device)
    _dev(params, "params", torch.float32, mlp_param_count(F, H, O), X.device)
    grad = torch.empty(params.numel(), dtype=torch.float32, device=X.device)
    ws = _mlp_ws(F, H, O, B, X.device)
    with _on(X.device, stream) as s_:
        _check(load_library().truss_mlp_backward(_ptr(params), F, H, O, _ptr(X), B, _ptr(dY), _ptr(grad), _ptr(ws),
                                                 _ws_bytes(ws), s_))
    return grad


def mlp_train(params, adam_m, adam_v, X, T, Wt, H: int, steps: int, step0: int = 0, lr: float = 1e-2,
              stream=None):
    """Adam steps on the weighted squared error, in place on params/adam_m/adam_v
    (contiguous CUDA float32 tensors); returns the final loss."""
    torch = _torch()
    X, T, Wt = _f32(X), _f32(T), _f32(Wt)
    B, F = X.shape
    O = T.shape[1]
    if T.shape != (B, O) or Wt.shape != (B, O):
        raise ValueError("T and Wt must be B x O")
    _dev(X, "X", torch.float32)
    _dev(T, "T", torch.float32, device=X.device)
    _dev(Wt, "Wt", torch.float32, device=X.device)
    P = mlp_param_count(F, H, O)
    for t, name in ((params, "params"), (adam_m, "adam_m"), (adam_v, "adam_v")):
        _dev(t, name, torch.float32, P, X.device)  # updated in place
    ws = _mlp_ws(F, H, O, B, X.device)
    loss = ctypes.c_float(0.0)
    with _on(X.device, stream) as s_:
        _check(load_library().truss_mlp_train(_ptr(params), _ptr(adam_m), _ptr(adam_v), F, H, O, _ptr(X), _ptr(T),
                                              _ptr(Wt), B, steps, step0, lr, ctypes.byref(loss), _ptr(ws),
                                              _ws_bytes(ws), s_))
    return loss.value


def sched_part_floats(kind: int, H: int) -> int:
    rc = load_library().truss_sched_part_floats(kind, H)
    if rc < 0:
        _check(rc)
    return rc


def sched_train(kind: int, X, T_ms, H: int = 32, steps: int = 3000, lr: float = 1e-2, seed: int = 1,
                out=None, stream=None):
    """Fit a scheduler model part (kind 0 peeling, 1 support) on traced
    decisions: X (B x F) raw features, T_ms (B x A) action times (<= 0 = not
    measured).  Returns (part float32 tensor, final loss)."""
    torch = _torch()
    lib = load_library()
    X, T_ms = _f32(X), _f32(T_ms)
    B = X.shape[0]
    n = sched_part_floats(kind, H)
    if X.dim() != 2 or T_ms.dim() != 2 or T_ms.shape[0] != B:
        raise ValueError("X and T_ms must be 2-D with one row per decision")
    _dev(X, "X", torch.float32)
    _dev(T_ms, "T_ms", torch.float32, device=X.device)
    if out is None:
        out = torch.empty(n, dtype=torch.float32, device=X.device)
    _dev(out, "out", torch.float32, n, X.device)
    b = ctypes.c_size_t(0)
    _check(lib.truss_sched_train_workspace_size(kind, H, B, ctypes.byref(b)))
    ws = torch.empty(b.value, dtype=torch.uint8, device=X.device)
    loss = ctypes.c_float(0.0)
    with _on(X.device, stream) as s_:
        _check(lib.truss_sched_train(kind, _ptr(X), _ptr(T_ms), B, H, steps, lr, seed, _ptr(out),
                                     ctypes.byref(loss), _ptr(ws), _ws_bytes(ws), s_))
    return out, loss.value


def truss_upper_bound(graph: Graph, out=None, ws=None, stream=None):
    """psi(e) = min{sup(e), x_u, x_v} + 2 of every edge (Procedure 6)."""
    torch = _torch()
    lib = load_library()
    if out is None:
        out = torch.empty(graph.m, dtype=torch.int32, device=graph.device)
    _dev(out, "out", torch.int32, graph.m, graph.device)
    if ws is None:
        ws = workspace(graph)
    g = graph._c()
    with _on(graph.device, stream) as s_:
        _check(lib.truss_upper_bound(ctypes.byref(g), _ptr(out), _ptr(ws), _ws_bytes(ws, graph.device),
                                     s_))
    return out


def truss_topdown(graph: Graph, t: int, opts: Options | None = None, out=None, ws=None, stream=None):
    """The top-t k-classes: (phi where phi > kmax - t else 0, kmin, kmax, stats)."""
    torch = _torch()
    lib = load_library()
    if out is None:
        out = torch.empty(graph.m, dtype=torch.int32, device=graph.device)
    _dev(out, "out", torch.int32, graph.m, graph.device)
    g = graph._c()
    if ws is None:
        b = ctypes.c_size_t(0)
        _check(lib.truss_topdown_workspace_size(ctypes.byref(g), ctypes.byref(opts) if opts else None,
                                                ctypes.byref(b)))
        ws = torch.empty(max(1, b.value), dtype=torch.uint8, device=graph.device)
    kmin, kmax = ctypes.c_int32(0), ctypes.c_int32(0)
    st = Stats()
    with _on(graph.device, stream) as s_:
        _check(lib.truss_topdown(ctypes.byref(g), t, _ptr(out), ctypes.byref(kmin), ctypes.byref(kmax),
                                 ctypes.byref(opts) if opts else None, ctypes.byref(st), _ptr(ws),
                                 _ws_bytes(ws, graph.device), s_))
    return out, kmin.value, kmax.value, st.to_dict()


def truss_core_numbers(graph: Graph, out=None, ws=None, stream=None):
    """(core numbers of every vertex as int32[n], c_max): the c-core is the
    largest subgraph with minimum degree >= c (the k-core of Section 7)."""
    torch = _torch()
    lib = load_library()
    if out is None:
        out = torch.empty(max(graph.n, 1), dtype=torch.int32, device=graph.device)
    _dev(out, "out", torch.int32, graph.n, graph.device)
    g = graph._c()
    if ws is None:
        b = ctypes.c_size_t(0)
        _check(lib.truss_core_workspace_size(ctypes.byref(g), ctypes.byref(b)))
        ws = torch.empty(max(1, b.value), dtype=torch.uint8, device=graph.device)
    cmax = ctypes.c_int32(0)
    with _on(graph.device, stream) as s_:
        _check(lib.truss_core_numbers(ctypes.byref(g), _ptr(out), ctypes.byref(cmax), _ptr(ws),
                                      _ws_bytes(ws, graph.device), s_))
    return out[:graph.n], cmax.value


def truss_cohesion(graph: Graph, opts: Options | None = None, ws=None, stream=None):
    """Table 6's columns for the k_max-truss and the c_max-core: dict with
    V_T, E_T, kmax, CC_T, V_C, E_C, cmax, CC_C."""
    torch = _torch()
    lib = load_library()
    g = graph._c()
    if ws is None:
        b = ctypes.c_size_t(0)
        _check(lib.truss_cohesion_workspace_size(ctypes.byref(g), ctypes.byref(b)))
        ws = torch.empty(max(1, b.value), dtype=torch.uint8, device=graph.device)
    st = CohesionStats()
    with _on(graph.device, stream) as s_:
        _check(lib.truss_cohesion(ctypes.byref(g), ctypes.byref(opts) if opts else None, ctypes.byref(st), _ptr(ws),
                                  _ws_bytes(ws, graph.device), s_))
    return st.to_dict()


def truss_bottomup(n: int, src, dst, cap: int, first_part=None, opts: Options | None = None, ws=None,
                   stream=None):
    """Bottom-up truss decomposition of a graph held in host memory (Section 5:
    LowerBounding, then Algorithm 4 with Procedures 5 and 9), the device
    holding one neighbourhood subgraph of at most `cap` edges at a time.
    src, dst: host int32 arrays.  Returns (phi, lower bound, stats) as numpy
    arrays and a dict."""
    import numpy as np
    torch = _torch()
    lib = load_library()
    src = np.ascontiguousarray(src, dtype=np.int32)
    dst = np.ascontiguousarray(dst, dtype=np.int32)
    if src.ndim != 1 or src.shape != dst.shape:
        raise ValueError("src and dst must be 1-D and of equal length")
    m = src.size
    fp = None if first_part is None else np.ascontiguousarray(first_part, dtype=np.int32)
    if fp is not None and fp.shape != (max(int(n), 0),):
        raise ValueError("first_part must hold one part id per vertex")
    if ws is None:
        b = ctypes.c_size_t(0)
        _check(lib.truss_bottomup_workspace_size(int(cap), ctypes.byref(b)))
        ws = torch.empty(max(1, b.value), dtype=torch.uint8, device="cuda")
    out = np.zeros(max(m, 1), dtype=np.int32)
    low = np.zeros(max(m, 1), dtype=np.int32)
    st = BottomUpStats()
    with _on(ws.device, stream) as s_:
        _check(lib.truss_bottomup(int(n), m, src.ctypes.data, dst.ctypes.data,
                                  None if fp is None else fp.ctypes.data, int(cap), out.ctypes.data, low.ctypes.data,
                                  ctypes.byref(opts) if opts else None, ctypes.byref(st), _ptr(ws), _ws_bytes(ws),
                                  s_))
    return out[:m], low[:m], st.to_dict()


def truss_cohen(graph: Graph, out=None, ws=None, stream=None):
    """Algorithm 1 (Section 3.1) on the device: (truss numbers, stats).  The
    comparator of Algorithm 2's improvement; the same truss numbers as
    truss_decompose."""
    torch = _torch()
    lib = load_library()
    if out is None:
        out = torch.empty(graph.m, dtype=torch.int32, device=graph.device)
    _dev(out, "out", torch.int32, graph.m, graph.device)
    g = graph._c()
    if ws is None:
        b = ctypes.c_size_t(0)
        _check(lib.truss_cohen_workspace_size(ctypes.byref(g), ctypes.byref(b)))
        ws = torch.empty(max(1, b.value), dtype=torch.uint8, device=graph.device)
    st = Stats()
    with _on(graph.device, stream) as s_:
        _check(lib.truss_cohen(ctypes.byref(g), _ptr(out), ctypes.byref(st), _ptr(ws), _ws_bytes(ws, graph.device),
                               s_))
    return out, st.to_dict()
