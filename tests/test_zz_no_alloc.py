"""truss_decompose_noalloc (scratch in the library's fixed device array)
against truss_decompose with a caller workspace, through the C ABI: two calls
in a row, the second on a smaller graph, so the second runs over the array
the first call left behind.  Outputs must be bit-identical (truss numbers are
unique, Definition 2) and equal to the oracle's."""
import ctypes

import numpy as np
import pytest

import graphgen
import oracle
from gpu_util import csr_graph, edges_graph, lib, say

pytestmark = pytest.mark.gpu


def _run_both(T, g, opts=None):
    import torch
    ref, _ = T.truss_decompose(g, opts)
    out = torch.full((g.m,), -7, dtype=torch.int32, device=g.device)
    got, st = T.truss_decompose_noalloc(g, out, opts)
    assert got.data_ptr() == out.data_ptr()
    assert st["ms_total"] == 0.0 and st["ms_peel_kernel"] == 0.0  # no timing events in this entry point
    return got.cpu().numpy(), ref.cpu().numpy(), st


def test_noalloc_matches_workspace_entry_point_twice():
    T = lib()
    from paper_1205_6693_amd import sched
    cases = []
    n, s, d = graphgen.rmat(14, 16, 9)  # about 190K edges, edge list in shuffled order
    s2, d2 = graphgen.shuffle(s, d, 4)
    cases.append(("rmat14 edge list", n, s2, d2, edges_graph(n, s2, d2)))
    n, s, d = graphgen.er_small(2)  # about 20K edges, CSR: smaller than the first
    cases.append(("er2000 csr", n, s, d, csr_graph(n, s, d)))
    sizes = []
    for name, n, s, d, g in cases:
        say(f"case: noalloc {name} n={n} m={s.size}")
        want, kmax = oracle.truss(n, s, d)
        for opts in (None, T.make_options(scheduler=T.SCHED_LEARNED, model=sched.load_model())):
            got, ref, st = _run_both(T, g, opts)
            np.testing.assert_array_equal(got, ref)
            np.testing.assert_array_equal(got, want)
            assert st["kmax"] == kmax and st["m"] == s.size
        sizes.append(T.truss_workspace_size(g))
    assert sizes[1] < sizes[0] <= T.NOALLOC_SCRATCH_BYTES


def test_noalloc_refuses_graphs_beyond_the_array():
    T = lib()
    rawlib = T.load_library()
    g = T._Graph()
    g.n, g.m, g.fmt = 1 << 20, 4 << 20, T.FMT_EDGES
    g.src = g.dst = 4096  # never dereferenced: refused before any device work
    st = T.Stats()
    rc = rawlib.truss_decompose_noalloc(ctypes.byref(g), ctypes.c_void_p(4096), None, ctypes.byref(st), None)
    assert rc == T.E_WORKSPACE
    assert b"fixed array" in rawlib.truss_last_error()
