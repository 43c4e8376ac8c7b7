"""Pins of the oracle's bottom-up truss decomposition (Section 5: LowerBounding,
Algorithm 3; Algorithm 4 with Procedures 5 and 9) against Example 3, Lemma 1,
the one-part closed form and brute force."""
import numpy as np
import pytest

import brute
import golden_io
import oracle


def _pairs(s, d):
    return [(min(int(a), int(b)), max(int(a), int(b))) for a, b in zip(s, d)]


def _example3():
    n, s, d, phi_paper = golden_io.fig2()
    ex = golden_io.example3()
    part = np.array([ex["part"][v] - 1 for v in range(n)], np.int32)
    return n, s, d, phi_paper, ex, part


def test_example3_lower_bounds():
    """The bounds and the 2-class that Example 3 states for the partition
    {a,b,c,l}, {d,e,f,g}, {h,i,j,k}."""
    n, s, d, _, ex, part = _example3()
    lb, phi2, info = oracle.lower_bounding(n, s, d, cap=1000, first_part=part)
    pairs = _pairs(s, d)
    for i, e in enumerate(pairs):
        if e in ex["phi2"]:
            assert phi2[i]
        else:
            assert not phi2[i], e
            assert lb[i] == ex["bound"][e], (e, lb[i])
    assert info["phi2_edges"] == len(ex["phi2"]) == 1
    assert info["gnew_edges"] == len(pairs) - 1
    # the first pass takes one neighbourhood subgraph per part; the edges
    # between parts need a second pass
    assert info["passes"] == 2 and info["subgraphs"] == 4


def test_example3_classes():
    """Stage 2 of Example 3: Phi_3 and Phi_4 as listed, and the truss numbers of
    Example 2 for every edge."""
    n, s, d, phi_paper, ex, part = _example3()
    phi, lb, info = oracle.bottom_up(n, s, d, cap=1000, first_part=part)
    np.testing.assert_array_equal(phi, phi_paper)
    pairs = _pairs(s, d)
    for k, edges in ex["classes"].items():
        assert sorted(e for i, e in enumerate(pairs) if phi[i] == k) == sorted(edges)
    assert info["kmax"] == 5


def test_one_part_gives_exact_bounds():
    """cap >= 2m: one pass, one neighbourhood subgraph (the whole graph), so the
    bound is phi itself and Phi_2 is the set of edges of support 0."""
    rng = np.random.default_rng(3)
    for trial in range(20):
        n = int(rng.integers(5, 30))
        edges = brute.random_graph(rng, n, float(rng.uniform(0.1, 0.6)))
        if not edges:
            continue
        s, d = np.array(edges, np.int32).T.copy()
        phi_ref = brute.truss_by_peeling(n, edges)
        sup = brute.support_brute(n, edges)
        lb, phi2, info = oracle.lower_bounding(n, s, d, cap=2 * len(edges))
        assert info["passes"] == 1 and info["subgraphs"] == 1
        np.testing.assert_array_equal(phi2, sup == 0)
        np.testing.assert_array_equal(lb, phi_ref)
        phi, _, info = oracle.bottom_up(n, s, d, cap=2 * len(edges))
        assert info["kstart"] == 3
        np.testing.assert_array_equal(phi, phi_ref)


def test_tiny_graphs_against_subset_enumeration():
    """Every budget from the largest degree up: the truss numbers equal the
    exhaustive definition, the bounds obey Lemma 1 and every Phi_2 edge has
    support 0 (Theorem 2's argument for the 2-class)."""
    rng = np.random.default_rng(11)
    done = 0
    while done < 25:
        n = int(rng.integers(4, 9))
        edges = brute.random_graph(rng, n, 0.55)
        if not edges or len(edges) > 16:
            continue
        done += 1
        s, d = np.array(edges, np.int32).T.copy()
        ref = brute.truss_literal(n, edges)
        sup = brute.support_brute(n, edges)
        dmax = int(np.bincount(np.concatenate([s, d])).max())
        for cap in range(dmax, 2 * len(edges) + 1):
            try:
                phi, lb, info = oracle.bottom_up(n, s, d, cap=cap)
            except oracle.OracleError as e:
                assert -e.code == oracle.STALL  # budget too small for any progress
                continue
            np.testing.assert_array_equal(phi, ref)
            assert (lb <= ref).all()
            lb1, phi2, _ = oracle.lower_bounding(n, s, d, cap=cap)
            assert (sup[phi2] == 0).all()


def test_medium_graphs_with_procedure9():
    """Budgets small enough that candidate subgraphs overflow and Procedure 9
    runs: the truss numbers still equal an independent peeling."""
    rng = np.random.default_rng(5)
    used9 = 0
    for trial in range(6):
        n = 36
        edges = brute.random_graph(rng, n, 0.3)
        s, d = np.array(edges, np.int32).T.copy()
        ref = brute.truss_by_peeling(n, edges)
        dmax = int(np.bincount(np.concatenate([s, d])).max())
        for cap in (2 * dmax, 4 * dmax, len(edges) // 2, 2 * len(edges)):
            phi, lb, info = oracle.bottom_up(n, s, d, cap=cap)
            np.testing.assert_array_equal(phi, ref)
            assert (lb <= ref).all() and (lb >= 2).all()
            used9 += info["proc9_calls"] > 0
    assert used9 > 0


def test_budget_below_a_degree_is_refused():
    n, s, d, _ = golden_io.fig2()
    with pytest.raises(oracle.OracleError) as e:
        oracle.lower_bounding(n, s, d, cap=6)  # vertex d has degree 7
    assert -e.value.code == oracle.CAP


def test_part_ids_outside_range_are_refused():
    # the caller's partition names every vertex with an edge by a part id in
    # [0, n), as the library's boundary requires; vertices without edges are
    # not read
    n, s, d, _, _, part = _example3()
    for bad in (-1, n, n + 7):
        p = part.copy()
        p[int(s[0])] = bad
        with pytest.raises(oracle.OracleError) as e:
            oracle.lower_bounding(n, s, d, cap=40, first_part=p)
        assert -e.value.code == oracle.INVAL
    iso = np.concatenate([part, np.array([n + 5], np.int32)])  # an isolated vertex n
    lb, _, _ = oracle.lower_bounding(n + 1, s, d, cap=40, first_part=iso)
    lb0, _, _ = oracle.lower_bounding(n, s, d, cap=40, first_part=part)
    assert (lb == lb0).all()
