"""Helpers for the GPU tests: move seeded inputs to the device, call the C ABI
through the binding, and bring results back as numpy arrays."""
import sys

import numpy as np

import graphgen


def say(*a):
    print(*a, flush=True)
    sys.stdout.flush()


def lib():
    import paper_1205_6693_amd as T
    T.load_library()
    return T


def dev(x, dtype=None):
    import torch
    t = torch.from_numpy(np.ascontiguousarray(x))
    if dtype is not None:
        t = t.to(dtype)
    return t.to("cuda:0")


def edges_graph(n, s, d):
    import torch
    T = lib()
    return T.Graph.from_edges(n, dev(s, torch.int32), dev(d, torch.int32))


def csr_graph(n, s, d):
    """CSR graph of a canonical edge list; output order = canonical (s, d) order."""
    import torch
    T = lib()
    rp, col = graphgen.to_csr(n, s, d)
    return T.Graph.from_csr(n, dev(rp, torch.int64), dev(col, torch.int32))


def gpu_truss(g, **opt):
    T = lib()
    o = T.make_options(**opt) if opt else None
    out, st = T.truss_decompose(g, o)
    return out.cpu().numpy(), st


def gpu_support(g):
    T = lib()
    out, tri = T.truss_support(g)
    return out.cpu().numpy(), tri


def canonical_sorted(s, d):
    """Canonical (u < v) edge list sorted by (u, v)."""
    a = np.minimum(s, d).astype(np.int64)
    b = np.maximum(s, d).astype(np.int64)
    order = np.lexsort((b, a))
    return a[order].astype(np.int32), b[order].astype(np.int32), order
