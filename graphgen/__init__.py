"""Seeded synthetic graph inputs (ctypes wrapper over graphgen.c).

This module produces inputs only and holds none of the truss arithmetic; both
the GPU tests and the oracle tests draw their graphs from it.

Every graph is returned canonical: int32 arrays ``src < dst`` sorted by
``(src, dst)``, simple (no self-loops, no duplicates).  ``to_csr`` turns it into
the symmetric CSR (int64 row_ptr, int32 col, rows ascending).

Workload recipes (the synthetic stand-ins for the paper's real power-law
datasets; sizes and shapes follow the configurations the path is measured on):
  er_small   Erdos-Renyi G(n=2000, p=0.01), ~20k edges
  rmat20     R-MAT scale 20, edge factor 16, (a,b,c,d)=(.57,.19,.19,.05)
  chung_lu4m Chung-Lu n=4M, exponent 2.1, mean degree 30, cap 200k, plus 64
             planted cliques of size U{50..500}
  batch4096  4096 graphs, n~U{64..8192}, mean degree ~U[4,64], half ER half R-MAT
  rmat24     R-MAT scale 24, edge factor 16, same (a,b,c,d)
"""
from __future__ import annotations

import ctypes
import os
import subprocess

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
_SRC = os.path.join(_HERE, "graphgen.c")
_LIB = os.path.join(_HERE, "_graphgen.so")
_lib = None

RMAT_ABC = (0.57, 0.19, 0.19)


def build(force: bool = False) -> str:
    if force or not os.path.exists(_LIB) or os.path.getmtime(_LIB) < os.path.getmtime(_SRC):
        tmp = _LIB + ".tmp%d" % os.getpid()
        subprocess.check_call(["gcc", "-O3", "-fopenmp", "-fPIC", "-shared", "-std=gnu11",
                               "-Wall", "-o", tmp, _SRC, "-lm"])
        os.replace(tmp, _LIB)
    return _LIB


def _load():
    global _lib
    if _lib is None:
        build()
        lib = ctypes.CDLL(_LIB)
        vp = ctypes.c_void_p
        i32p = np.ctypeslib.ndpointer(dtype=np.int32, flags="C_CONTIGUOUS")
        i64p = np.ctypeslib.ndpointer(dtype=np.int64, flags="C_CONTIGUOUS")
        lib.gg_er.argtypes = [ctypes.c_int32, ctypes.c_double, ctypes.c_uint64]
        lib.gg_er.restype = vp
        lib.gg_rmat.argtypes = [ctypes.c_int32, ctypes.c_int64, ctypes.c_int32, ctypes.c_double,
                                ctypes.c_double, ctypes.c_double, ctypes.c_uint64, ctypes.c_int]
        lib.gg_rmat.restype = vp
        lib.gg_chung_lu.argtypes = [ctypes.c_int32, ctypes.c_double, ctypes.c_double,
                                    ctypes.c_double, ctypes.c_int32, ctypes.c_int32,
                                    ctypes.c_int32, ctypes.c_uint64]
        lib.gg_chung_lu.restype = vp
        lib.gg_chung_lu_clique_sizes.argtypes = [ctypes.c_int32, ctypes.c_int32, ctypes.c_int32,
                                                 ctypes.c_uint64, i32p]
        lib.gg_free.argtypes = [vp]
        lib.gg_m.argtypes = [vp]
        lib.gg_m.restype = ctypes.c_int64
        lib.gg_n.argtypes = [vp]
        lib.gg_n.restype = ctypes.c_int32
        lib.gg_copy.argtypes = [vp, i32p, i32p]
        lib.gg_to_csr.argtypes = [ctypes.c_int32, ctypes.c_int64, i32p, i32p, i64p, i32p]
        lib.gg_shuffle.argtypes = [ctypes.c_int64, i32p, i32p, ctypes.c_uint64]
        _lib = lib
    return _lib


def _take(handle):
    lib = _load()
    if not handle:
        raise MemoryError("graph generator failed (bad parameters or out of memory)")
    try:
        n, m = lib.gg_n(handle), lib.gg_m(handle)
        src = np.empty(max(m, 1), dtype=np.int32)
        dst = np.empty(max(m, 1), dtype=np.int32)
        if m:
            lib.gg_copy(handle, src, dst)
        return n, src[:m], dst[:m]
    finally:
        lib.gg_free(handle)


def er(n: int, p: float, seed: int):
    """Erdos-Renyi G(n, p) -> (n, src, dst)."""
    return _take(_load().gg_er(n, p, seed))


def rmat(scale: int, edge_factor: float, seed: int, n: int | None = None, samples: int | None = None,
         abc=RMAT_ABC, permute: bool = True):
    """R-MAT with 2^scale ids (or the first n of them) -> (n, src, dst)."""
    if n is None:
        n = 1 << scale
    if samples is None:
        samples = int(round(edge_factor * (1 << scale)))
    a, b, c = abc
    return _take(_load().gg_rmat(scale, samples, n, a, b, c, seed, 1 if permute else 0))


def chung_lu(n: int, gamma: float, mean_deg: float, max_deg: float, n_cliques: int,
             clique_min: int, clique_max: int, seed: int):
    """Chung-Lu power-law graph plus planted cliques -> (n, src, dst)."""
    return _take(_load().gg_chung_lu(n, gamma, mean_deg, max_deg, n_cliques, clique_min,
                                     clique_max, seed))


def chung_lu_clique_sizes(n_cliques: int, clique_min: int, clique_max: int, seed: int):
    out = np.zeros(max(n_cliques, 1), dtype=np.int32)
    _load().gg_chung_lu_clique_sizes(n_cliques, clique_min, clique_max, seed, out)
    return out[:n_cliques]


def to_csr(n: int, src, dst):
    """Symmetric CSR (row_ptr int64[n+1], col int32[2m]) of a canonical edge list."""
    src = np.ascontiguousarray(src, dtype=np.int32)
    dst = np.ascontiguousarray(dst, dtype=np.int32)
    m = src.size
    row_ptr = np.zeros(n + 1, dtype=np.int64)
    col = np.empty(max(2 * m, 1), dtype=np.int32)
    s = src if m else np.zeros(1, dtype=np.int32)
    d = dst if m else np.zeros(1, dtype=np.int32)
    _load().gg_to_csr(n, m, s, d, row_ptr, col)
    return row_ptr, col[: 2 * m]


def shuffle(src, dst, seed: int):
    """Copy of the edge list with seeded random order and orientation."""
    s = np.array(src, dtype=np.int32, copy=True)
    d = np.array(dst, dtype=np.int32, copy=True)
    if s.size:
        _load().gg_shuffle(s.size, s, d, seed)
    return s, d


def relabel(n: int, src, dst, seed: int):
    """Copy of the edge list with vertex ids permuted by a seeded permutation."""
    rng = np.random.Generator(np.random.Philox(seed))
    pi = rng.permutation(n).astype(np.int32)
    return pi[np.asarray(src)], pi[np.asarray(dst)]


# ---------------------------------------------------------------------------
# Workload recipes
# ---------------------------------------------------------------------------

def er_small(seed: int = 1):
    return er(2000, 0.01, seed)


def rmat20(seed: int = 1):
    return rmat(20, 16, seed)


def rmat24(seed: int = 1):
    return rmat(24, 16, seed)


def chung_lu4m(seed: int = 1):
    return chung_lu(4 << 20, 2.1, 30.0, 200000.0, 64, 50, 500, seed)


def batch_specs(num_graphs: int, seed: int, n_lo: int = 64, n_hi: int = 8192,
                d_lo: float = 4.0, d_hi: float = 64.0):
    """Per-graph (kind, n, mean degree, seed) of the uneven small-graph batch."""
    rng = np.random.Generator(np.random.Philox(seed))
    ns = rng.integers(n_lo, n_hi + 1, size=num_graphs)
    ds = rng.uniform(d_lo, d_hi, size=num_graphs)
    return [("er" if g % 2 == 0 else "rmat", int(ns[g]), float(ds[g]), seed * 1000003 + g)
            for g in range(num_graphs)]


def batch(num_graphs: int = 4096, seed: int = 1, **kw):
    """Uneven batch: list of (n, src, dst).  Even g: ER with p=min(1, d/(n-1));
    odd g: R-MAT with scale ceil(log2 n), round(n*d/2) samples, ids >= n rejected."""
    return [batch_graph(spec) for spec in batch_specs(num_graphs, seed, **kw)]


def batch_graph(spec):
    """One graph of the batch from its (kind, n, mean degree, seed) spec."""
    kind, n, d, s = spec
    if kind == "er":
        return er(n, min(1.0, d / (n - 1)), s)
    scale = max(1, int(np.ceil(np.log2(n))))
    return rmat(scale, 0, s, n=n, samples=int(round(n * d / 2)))


def pack(graphs):
    """Pack a list of (n, src, dst) into (vtx_off int64[G+1], edge_off int64[G+1],
    src int32[M], dst int32[M]) with graph-local vertex ids."""
    G = len(graphs)
    vtx_off = np.zeros(G + 1, dtype=np.int64)
    edge_off = np.zeros(G + 1, dtype=np.int64)
    for g, (n, s, d) in enumerate(graphs):
        vtx_off[g + 1] = vtx_off[g] + n
        edge_off[g + 1] = edge_off[g] + s.size
    src = np.concatenate([s for _, s, _ in graphs]) if G else np.zeros(0, np.int32)
    dst = np.concatenate([d for _, _, d in graphs]) if G else np.zeros(0, np.int32)
    return vtx_off, edge_off, src.astype(np.int32), dst.astype(np.int32)
