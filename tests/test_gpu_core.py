"""GPU tests of the core numbers and of the cohesion statistics of the
k_max-truss and the c_max-core (Section 7, Table 6) against the oracle: core
numbers bit-exact, vertex and edge counts exact, mean clustering coefficients
to 1e-12 relative (the device sums them in a tree order, the oracle in vertex
order; each term is the same correctly rounded fp64 quotient)."""
import itertools

import numpy as np
import pytest

import golden_io
import graphgen
import oracle
from gpu_util import canonical_sorted, csr_graph, edges_graph, lib, say

pytestmark = pytest.mark.gpu

CC_RTOL = 1e-12


def _graphs():
    n, s, d, _ = golden_io.fig2()
    out = [("example2", n, s, d)]
    k = 9
    cs, cd = map(np.array, zip(*itertools.combinations(range(k), 2)))
    out.append(("K9", k, cs.astype(np.int32), cd.astype(np.int32)))
    out.append(("star", 70, np.zeros(69, np.int32), np.arange(1, 70, dtype=np.int32)))
    # a path and a triangle with isolated vertices around them (ids 0, 4, 9 unused)
    out.append(("sparse", 10, np.array([1, 2, 5, 5, 6], np.int32), np.array([2, 3, 6, 7, 7], np.int32)))
    out.append(("er2000", *graphgen.er_small(4)))
    out.append(("rmat13", *graphgen.rmat(13, 16, 8)))
    out.append(("chunglu", *graphgen.chung_lu(30000, 2.1, 20.0, 3000.0, 6, 20, 90, 9)))
    return out


def _check_cohesion(got, ref):
    for key in ("V_T", "E_T", "kmax", "V_C", "E_C", "cmax"):
        assert got[key] == ref[key], (key, got, ref)
    for key in ("CC_T", "CC_C"):
        assert got[key] == pytest.approx(ref[key], rel=CC_RTOL, abs=1e-15), (key, got, ref)


def test_core_numbers_match_oracle():
    T = lib()
    for name, n, s, d in _graphs():
        say(f"case: core numbers on {name}")
        ref, rmax = oracle.core_numbers(n, s, d)
        ss, dd = graphgen.shuffle(s, d, 11)
        got, cmax = T.truss_core_numbers(edges_graph(n, ss, dd))
        np.testing.assert_array_equal(got.cpu().numpy(), ref)
        assert cmax == rmax
        cs, cd, _ = canonical_sorted(s, d)
        got, cmax = T.truss_core_numbers(csr_graph(n, cs, cd))
        np.testing.assert_array_equal(got.cpu().numpy(), ref)
        assert cmax == rmax


def test_core_numbers_degenerate():
    T = lib()
    say("case: core numbers, no edges")
    got, cmax = T.truss_core_numbers(edges_graph(5, np.zeros(0, np.int32), np.zeros(0, np.int32)))
    np.testing.assert_array_equal(got.cpu().numpy(), np.zeros(5, np.int32))
    assert cmax == 0
    say("case: core numbers, no vertices")
    got, cmax = T.truss_core_numbers(edges_graph(0, np.zeros(0, np.int32), np.zeros(0, np.int32)))
    assert got.numel() == 0 and cmax == 0
    say("case: core numbers, one edge")
    got, cmax = T.truss_core_numbers(edges_graph(2, np.array([1], np.int32), np.array([0], np.int32)))
    np.testing.assert_array_equal(got.cpu().numpy(), [1, 1])
    assert cmax == 1


def test_core_numbers_reject_invalid_graphs():
    T = lib()
    say("case: core numbers, invalid inputs")
    with pytest.raises(T.TrussError):
        T.truss_core_numbers(edges_graph(4, np.array([0, 1], np.int32), np.array([0, 2], np.int32)))  # self-loop
    with pytest.raises(T.TrussError):
        T.truss_core_numbers(edges_graph(4, np.array([0, 1], np.int32), np.array([1, 0], np.int32)))  # duplicate
    with pytest.raises(T.TrussError):
        T.truss_core_numbers(edges_graph(4, np.array([0], np.int32), np.array([4], np.int32)))  # out of range


def test_cohesion_matches_oracle():
    T = lib()
    for name, n, s, d in _graphs():
        say(f"case: cohesion on {name}")
        ref = oracle.cohesion(n, s, d)
        ss, dd = graphgen.shuffle(s, d, 12)
        _check_cohesion(T.truss_cohesion(edges_graph(n, ss, dd)), ref)
        cs, cd, _ = canonical_sorted(s, d)
        _check_cohesion(T.truss_cohesion(csr_graph(n, cs, cd)), ref)


def test_cohesion_example2():
    """The graph of Example 2: its 5-truss and its 4-core are both the clique
    on vertices 0..4 (10 edges, clustering coefficient 1)."""
    T = lib()
    n, s, d, _ = golden_io.fig2()
    got = T.truss_cohesion(edges_graph(n, s, d))
    assert got == {"V_T": 5, "E_T": 10, "kmax": 5, "CC_T": 1.0, "V_C": 5, "E_C": 10, "cmax": 4, "CC_C": 1.0}


def test_cohesion_degenerate():
    T = lib()
    say("case: cohesion, no edges")
    got = T.truss_cohesion(edges_graph(6, np.zeros(0, np.int32), np.zeros(0, np.int32)))
    assert got == {"V_T": 0, "E_T": 0, "kmax": 0, "CC_T": 0.0, "V_C": 0, "E_C": 0, "cmax": 0, "CC_C": 0.0}
    say("case: cohesion, a matching (no triangles)")
    got = T.truss_cohesion(edges_graph(6, np.array([0, 2, 4], np.int32), np.array([1, 3, 5], np.int32)))
    assert got == {"V_T": 6, "E_T": 3, "kmax": 2, "CC_T": 0.0, "V_C": 6, "E_C": 3, "cmax": 1, "CC_C": 0.0}


FULL = {"er2000": lambda: graphgen.er_small(1), "rmat16": lambda: graphgen.rmat(16, 16, 1),
        "rmat20": lambda: graphgen.rmat20(1), "chunglu4m": lambda: graphgen.chung_lu4m(1),
        "rmat24": lambda: graphgen.rmat24(1)}


@pytest.mark.parametrize("name", list(FULL))
def test_core_and_cohesion_full_size(name):
    rec = golden_io.oracle_record(name)
    if rec is None or "core_sha256" not in rec:
        pytest.skip("no core record for " + name)
    T = lib()
    say(f"case: core numbers and cohesion, full size {name}")
    n, s, d = FULL[name]()
    g = csr_graph(n, s, d)
    core, cmax = T.truss_core_numbers(g)
    assert golden_io.int32_digest(core.cpu().numpy()) == rec["core_sha256"]
    assert cmax == rec["cmax"]
    if "cohesion" in rec:  # the R-MAT 24 record holds the core numbers only
        _check_cohesion(T.truss_cohesion(g), rec["cohesion"])


def test_truss_inside_core_at_size():
    """Every edge of the k-truss lies in the (k-1)-core: phi(e) - 1 <= core(u)
    and core(v), on R-MAT 20 (both sides checked against the oracle's digests
    elsewhere)."""
    import torch
    T = lib()
    say("case: k-truss inside the (k-1)-core, R-MAT 20")
    n, s, d = graphgen.rmat20(1)
    g = csr_graph(n, s, d)
    phi, _ = T.truss_decompose(g)
    core, _ = T.truss_core_numbers(g)
    u = torch.from_numpy(s.astype(np.int64)).cuda()
    v = torch.from_numpy(d.astype(np.int64)).cuda()
    lo = torch.minimum(core[u], core[v])
    assert bool((phi - 1 <= lo).all())
