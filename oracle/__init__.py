"""Serial CPU oracle for truss decomposition (ctypes wrapper over truss_oracle.c).

TEST INFRASTRUCTURE ONLY: the test-suite, the smoke check and the CPU-baseline
leg of the benchmark use it; the GPU library never imports, links or calls it.

Functions follow Wang & Cheng, "Truss Decomposition in Massive Networks":
  validate_edges / validate_csr  -- Section 2 (simple undirected graphs)
  support_def                    -- Definition 1 via the support merge of Algorithm 1
  support_fwd                    -- Definition 1 via the triangle counting that
                                    Algorithm 2 starts from (Section 3.2)
  truss                          -- Definition 2 / truss number via Algorithm 2
  upper_bound                    -- psi(e) of Procedure 6 (Lemma 2: phi <= psi)
  top_classes                    -- the top-t k-classes of Algorithm 7 from phi
  core_numbers                   -- core number of every vertex (Section 7)
  cohesion                       -- Table 6's statistics of the k_max-truss and c_max-core
  lower_bounding                 -- Algorithm 3: per-edge lower bounds and Phi_2 over
                                    neighbourhood-subgraph partitions (Lemma 1)
  bottom_up                      -- Algorithm 4 with Procedures 5 and 9 on those bounds
  csr_to_edges                   -- canonical upper-CSR edge order
"""
from __future__ import annotations

import ctypes
import os
import subprocess

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
_SRC = os.path.join(_HERE, "truss_oracle.c")
_LIB = os.path.join(_HERE, "_truss_oracle.so")

# error-code magnitudes (negative on return)
INVAL, TOOBIG, ROWPTR, RANGE, SELFLOOP, UNSORTED, DUP, ASYM, NOMEM, CAP, STALL = range(1, 12)

_lib = None


def build(force: bool = False) -> str:
    """Compile truss_oracle.c with gcc -O3 into _truss_oracle.so."""
    if force or not os.path.exists(_LIB) or os.path.getmtime(_LIB) < os.path.getmtime(_SRC):
        tmp = _LIB + ".tmp%d" % os.getpid()
        subprocess.check_call(["gcc", "-O3", "-march=x86-64-v2", "-fPIC", "-shared",
                               "-std=c11", "-Wall", "-o", tmp, _SRC])
        os.replace(tmp, _LIB)
    return _LIB


def _load():
    global _lib
    if _lib is None:
        build()
        lib = ctypes.CDLL(_LIB)
        i32p = np.ctypeslib.ndpointer(dtype=np.int32, flags="C_CONTIGUOUS")
        i64p = np.ctypeslib.ndpointer(dtype=np.int64, flags="C_CONTIGUOUS")
        c_i64p = ctypes.POINTER(ctypes.c_int64)
        c_i32p = ctypes.POINTER(ctypes.c_int32)
        lib.oracle_validate_edges.argtypes = [ctypes.c_int32, ctypes.c_int64, i32p, i32p]
        lib.oracle_validate_csr.argtypes = [ctypes.c_int32, ctypes.c_int64, i64p, i32p]
        lib.oracle_csr_to_edges.argtypes = [ctypes.c_int32, ctypes.c_int64, i64p, i32p, i32p, i32p]
        for f in (lib.oracle_support_def, lib.oracle_support_fwd):
            f.argtypes = [ctypes.c_int32, ctypes.c_int64, i32p, i32p, i32p, c_i64p]
        lib.oracle_truss.argtypes = [ctypes.c_int32, ctypes.c_int64, i32p, i32p, i32p, c_i32p]
        lib.oracle_upper_bound.argtypes = [ctypes.c_int32, ctypes.c_int64, i32p, i32p, i32p, i32p]
        lib.oracle_core_numbers.argtypes = [ctypes.c_int32, ctypes.c_int64, i32p, i32p, i32p, c_i32p]
        lib.oracle_cohesion.argtypes = [ctypes.c_int32, ctypes.c_int64, i32p, i32p, i32p, i32p,
                                        np.ctypeslib.ndpointer(np.float64, flags="C_CONTIGUOUS")]
        u8p = np.ctypeslib.ndpointer(dtype=np.uint8, flags="C_CONTIGUOUS")
        lib.oracle_lower_bounding.argtypes = [ctypes.c_int32, ctypes.c_int64, i32p, i32p, ctypes.c_void_p,
                                              ctypes.c_int64, i32p, u8p, i64p]
        lib.oracle_bottom_up.argtypes = [ctypes.c_int32, ctypes.c_int64, i32p, i32p, i32p, u8p, ctypes.c_int32,
                                         ctypes.c_int64, i32p, i64p]
        for f in (lib.oracle_validate_edges, lib.oracle_validate_csr, lib.oracle_csr_to_edges,
                  lib.oracle_support_def, lib.oracle_support_fwd, lib.oracle_truss):
            f.restype = ctypes.c_int
        _lib = lib
    return _lib


class OracleError(RuntimeError):
    def __init__(self, code: int):
        super().__init__("oracle error code %d" % code)
        self.code = code


def _edges(src, dst):
    src = np.ascontiguousarray(src, dtype=np.int32)
    dst = np.ascontiguousarray(dst, dtype=np.int32)
    if src.shape != dst.shape or src.ndim != 1:
        raise ValueError("src/dst must be 1-D arrays of equal length")
    return src, dst


def validate_edges(n: int, src, dst) -> int:
    src, dst = _edges(src, dst)
    return _load().oracle_validate_edges(n, src.size, src, dst)


def validate_csr(n: int, m: int, row_ptr, col) -> int:
    row_ptr = np.ascontiguousarray(row_ptr, dtype=np.int64)
    col = np.ascontiguousarray(col, dtype=np.int32)
    if row_ptr.size != n + 1:
        return -INVAL
    if col.size == 0:
        col = np.zeros(1, dtype=np.int32)
    return _load().oracle_validate_csr(n, m, row_ptr, col)


def csr_to_edges(n: int, m: int, row_ptr, col):
    row_ptr = np.ascontiguousarray(row_ptr, dtype=np.int64)
    col = np.ascontiguousarray(col, dtype=np.int32)
    src = np.empty(max(m, 1), dtype=np.int32)
    dst = np.empty(max(m, 1), dtype=np.int32)
    if col.size == 0:
        col = np.zeros(1, dtype=np.int32)
    rc = _load().oracle_csr_to_edges(n, m, row_ptr, col, src, dst)
    if rc:
        raise OracleError(rc)
    return src[:m], dst[:m]


def _support(fn, n, src, dst):
    src, dst = _edges(src, dst)
    rc = _load().oracle_validate_edges(n, src.size, src, dst)
    if rc:
        raise OracleError(rc)
    sup = np.zeros(max(src.size, 1), dtype=np.int32)
    tri = ctypes.c_int64(0)
    if src.size:
        rc = fn(n, src.size, src, dst, sup, ctypes.byref(tri))
        if rc:
            raise OracleError(rc)
    return sup[: src.size], int(tri.value)


def support_def(n: int, src, dst):
    """(sup[m], triangle count) by full-adjacency merge per edge."""
    return _support(_load().oracle_support_def, n, src, dst)


def support_fwd(n: int, src, dst):
    """(sup[m], triangle count) by degree-oriented forward listing."""
    return _support(_load().oracle_support_fwd, n, src, dst)


def truss(n: int, src, dst):
    """(phi[m], kmax): truss number of every input edge by Algorithm 2."""
    src, dst = _edges(src, dst)
    rc = _load().oracle_validate_edges(n, src.size, src, dst)
    if rc:
        raise OracleError(rc)
    phi = np.zeros(max(src.size, 1), dtype=np.int32)
    kmax = ctypes.c_int32(0)
    if src.size:
        rc = _load().oracle_truss(n, src.size, src, dst, phi, ctypes.byref(kmax))
        if rc:
            raise OracleError(rc)
    return phi[: src.size], int(kmax.value)


def upper_bound(n: int, src, dst, sup=None):
    """psi[m]: min{sup(e), x_u, x_v} + 2 (Procedure 6) for every input edge."""
    src, dst = _edges(src, dst)
    if sup is None:
        sup, _ = support_fwd(n, src, dst)
    sup = np.ascontiguousarray(sup, dtype=np.int32)
    psi = np.zeros(max(src.size, 1), dtype=np.int32)
    if src.size:
        rc = _load().oracle_upper_bound(n, src.size, src, dst, sup, psi)
        if rc:
            raise OracleError(rc)
    return psi[: src.size]


def top_classes(phi, t: int):
    """The top-t k-classes (Algorithm 7's output) from the truss numbers:
    phi(e) where phi(e) > k_max - t, 0 elsewhere; and the lowest class kept."""
    phi = np.asarray(phi, dtype=np.int32)
    kmax = int(phi.max()) if phi.size else 0
    kmin = max(2, kmax - t + 1)
    return np.where(phi >= kmin, phi, 0).astype(np.int32), kmin


def core_numbers(n: int, src, dst):
    """(core[n], c_max): the core number of every vertex."""
    src, dst = _edges(src, dst)
    rc = _load().oracle_validate_edges(n, src.size, src, dst)
    if rc:
        raise OracleError(rc)
    core = np.zeros(max(n, 1), dtype=np.int32)
    cmax = ctypes.c_int32(0)
    rc = _load().oracle_core_numbers(n, src.size, src, dst, core, ctypes.byref(cmax))
    if rc:
        raise OracleError(rc)
    return core[:n], int(cmax.value)


def cohesion(n: int, src, dst, phi=None, core=None):
    """Table 6's columns: dict with V_T, E_T, kmax, CC_T, V_C, E_C, cmax, CC_C."""
    src, dst = _edges(src, dst)
    if phi is None:
        phi, _ = truss(n, src, dst)
    if core is None:
        core, _ = core_numbers(n, src, dst)
    out = np.zeros(8, dtype=np.float64)
    rc = _load().oracle_cohesion(n, src.size, src, dst, np.ascontiguousarray(phi, dtype=np.int32),
                                 np.ascontiguousarray(core, dtype=np.int32), out)
    if rc:
        raise OracleError(rc)
    keys = ["V_T", "E_T", "kmax", "CC_T", "V_C", "E_C", "cmax", "CC_C"]
    return {k: (float(v) if k.startswith("CC") else int(v)) for k, v in zip(keys, out)}


def lower_bounding(n: int, src, dst, cap: int, first_part=None):
    """Algorithm 3: (lb[m], phi2[m] as bool, info) where lb is the lower bound
    of every edge and phi2 marks the edges output as Phi_2.  cap = most edges
    a neighbourhood subgraph may hold; first_part (optional) = part id in
    [0, n) of every vertex with an edge, for the first pass (later passes
    use the sequential partition)."""
    src, dst = _edges(src, dst)
    rc = _load().oracle_validate_edges(n, src.size, src, dst)
    if rc:
        raise OracleError(rc)
    m = src.size
    lb = np.zeros(max(m, 1), dtype=np.int32)
    phi2 = np.zeros(max(m, 1), dtype=np.uint8)
    info = np.zeros(5, dtype=np.int64)
    fp = None
    if first_part is not None:
        fp = np.ascontiguousarray(first_part, dtype=np.int32)
        if fp.shape != (n,):
            raise ValueError("first_part must hold one part id per vertex")
    rc = _load().oracle_lower_bounding(n, m, src, dst, None if fp is None else fp.ctypes.data_as(ctypes.c_void_p),
                                       int(cap), lb, phi2, info)
    if rc:
        raise OracleError(rc)
    keys = ["passes", "subgraphs", "phi2_edges", "gnew_edges", "max_subgraph"]
    return lb[:m], phi2[:m].astype(bool), dict(zip(keys, map(int, info)))


def bottom_up(n: int, src, dst, cap: int, first_part=None):
    """Bottom-up truss decomposition (Algorithm 3, then Algorithm 4 with
    Procedure 5, or Procedure 9 when a candidate subgraph exceeds cap):
    (phi[m], lb[m], info)."""
    src, dst = _edges(src, dst)
    lb, phi2, info = lower_bounding(n, src, dst, cap, first_part)
    m = src.size
    phi = np.zeros(max(m, 1), dtype=np.int32)
    binfo = np.zeros(5, dtype=np.int64)
    kstart = 3 if info["passes"] <= 1 else 2
    rc = _load().oracle_bottom_up(n, m, src, dst, np.ascontiguousarray(lb, dtype=np.int32),
                                  np.ascontiguousarray(phi2, dtype=np.uint8), kstart, int(cap), phi, binfo)
    if rc:
        raise OracleError(rc)
    keys = ["candidates", "proc9_calls", "proc9_scans", "max_candidate", "kmax"]
    info.update(zip(keys, map(int, binfo)))
    info["kstart"] = kstart
    return phi[:m], lb, info
