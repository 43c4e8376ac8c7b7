"""GPU tests of the bottom-up decomposition of a graph in host memory
(Section 5: LowerBounding, Algorithm 4, Procedures 5 and 9) against the
oracle: truss numbers and lower bounds bit-exact, and the same partitions,
subgraph counts and Procedure 9 scans."""
import numpy as np
import pytest

import golden_io
import graphgen
import oracle
from gpu_util import lib, say

pytestmark = pytest.mark.gpu

STAT_KEYS = ["passes", "subgraphs", "phi2_edges", "gnew_edges", "max_subgraph", "candidates", "proc9_calls",
             "proc9_scans", "max_candidate", "kmax", "kstart"]


def _compare(T, name, n, s, d, cap, first_part=None):
    say(f"case: bottom-up {name} m={s.size} cap={cap}")
    phi_ref, lb_ref, info = oracle.bottom_up(n, s, d, cap, first_part)
    phi, lb, st = T.truss_bottomup(n, s, d, cap, first_part)
    np.testing.assert_array_equal(lb, lb_ref)
    np.testing.assert_array_equal(phi, phi_ref)
    for k in STAT_KEYS:
        assert st[k] == info[k], (k, st[k], info[k])
    return st


def test_example3():
    T = lib()
    n, s, d, phi_paper = golden_io.fig2()
    ex = golden_io.example3()
    part = np.array([ex["part"][v] - 1 for v in range(n)], np.int32)
    st = _compare(T, "example3", n, s, d, 1000, part)
    phi, lb, _ = T.truss_bottomup(n, s, d, 1000, part)
    np.testing.assert_array_equal(phi, phi_paper)
    assert st["phi2_edges"] == 1 and st["passes"] == 2


@pytest.mark.parametrize("cap", [10, 12, 15, 20, 26, 60])
def test_example2_graph_budgets(cap):
    T = lib()
    n, s, d, phi_paper = golden_io.fig2()
    _compare(T, "example2", n, s, d, cap)


def _medium():
    return [("er2000", graphgen.er_small(4)), ("rmat11", graphgen.rmat(11, 8, 3)),
            ("chunglu", graphgen.chung_lu(6000, 2.1, 10.0, 600.0, 3, 10, 30, 9))]


def test_medium_graphs():
    T = lib()
    used9 = 0
    for name, (n, s, d) in _medium():
        ss, dd = graphgen.shuffle(s, d, 21)
        for cap in (ss.size // 3, 2 * ss.size):
            st = _compare(T, name, n, ss, dd, cap)
            used9 += st["proc9_calls"] > 0
    assert used9 > 0


def test_tight_budget_many_subgraphs():
    """A budget of twice the largest degree: many passes, many small
    subgraphs, Procedure 9 on every large candidate."""
    T = lib()
    n, s, d = graphgen.rmat(11, 8, 3)
    dmax = int(np.bincount(np.concatenate([s, d])).max())
    st = _compare(T, "rmat11 tight", n, s, d, 2 * dmax)
    assert st["passes"] > 5 and st["proc9_scans"] > 100


def test_errors():
    T = lib()
    n, s, d, _ = golden_io.fig2()
    say("case: bottom-up errors")
    with pytest.raises(T.TrussError):  # vertex d has degree 7
        T.truss_bottomup(n, s, d, 6)
    bad = np.zeros(n, np.int32)
    bad[3] = -1
    with pytest.raises(T.TrussError):  # a vertex with edges and no part
        T.truss_bottomup(n, s, d, 1000, bad)
    big = np.zeros(n, np.int32)
    big[0] = n
    with pytest.raises(T.TrussError):  # a part id outside [0, n)
        T.truss_bottomup(n, s, d, 1000, big)
    with pytest.raises(T.TrussError):  # a part whose subgraph exceeds the budget
        T.truss_bottomup(n, s, d, 20, np.zeros(n, np.int32))
    with pytest.raises(T.TrussError):  # self-loop
        T.truss_bottomup(4, np.array([0, 2], np.int32), np.array([1, 2], np.int32), 10)
    with pytest.raises(T.TrussError):  # duplicate pair
        T.truss_bottomup(4, np.array([0, 1], np.int32), np.array([1, 0], np.int32), 10)
    phi, lb, st = T.truss_bottomup(5, np.zeros(0, np.int32), np.zeros(0, np.int32), 10)
    assert phi.size == 0 and st["passes"] == 0 and st["kmax"] == 0


def test_rmat16_full_size():
    """R-MAT 16 (909,729 edges) with a budget of a quarter of the edges: the
    truss numbers match the oracle's stored digest."""
    rec = golden_io.oracle_record("rmat16")
    T = lib()
    n, s, d = graphgen.rmat(16, 16, 1)
    cap = s.size // 4
    say(f"case: bottom-up rmat16 cap={cap}")
    phi, lb, st = T.truss_bottomup(n, s, d, cap)
    say("stats", st)
    assert golden_io.int32_digest(phi) == rec["truss_sha256"]
    assert st["passes"] > 1 and st["max_subgraph"] <= cap and (lb <= phi).all()
