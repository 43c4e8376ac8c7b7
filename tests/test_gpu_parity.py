"""GPU parity: the HIP path (through the C ABI) against the CPU oracle, bit-exact.

Support and truss numbers are integers, so every comparison is exact
(element by element).  Truss numbers are unique (a union of subgraphs that
satisfy Definition 2 satisfies it), so any correct peeling order gives the same
array.
"""
import itertools

import numpy as np
import pytest

import golden_io
import graphgen
import oracle
from gpu_util import canonical_sorted, csr_graph, edges_graph, gpu_support, gpu_truss, lib, say

pytestmark = pytest.mark.gpu

# option sets: support strategy (1 hash, 2 bsearch, 3 merge), frontier mode
# (1 sparse, 2 dense), membership probe while peeling (1 hash table, 2 bsearch)
STRATS = [dict(support_strategy=1, peel_mode=1, peel_probe=1, peel_shape=1),
          dict(support_strategy=2, peel_mode=2, peel_probe=2, peel_shape=2),
          dict(support_strategy=3, peel_mode=1, peel_probe=2, peel_shape=1),
          dict(support_strategy=1, peel_mode=2, peel_probe=1, peel_shape=2),
          dict(support_strategy=2, peel_mode=1, peel_probe=2)]


def _both_formats(n, s, d, phi_ref, sup_ref=None, **opt):
    """Edge-list input (shuffled order/orientation) and CSR input."""
    ss, dd = graphgen.shuffle(s, d, 99)
    # edge list: outputs follow the shuffled input order
    ref_sh = oracle.truss(n, ss, dd)[0]
    got, st = gpu_truss(edges_graph(n, ss, dd), **opt)
    np.testing.assert_array_equal(got, ref_sh)
    # CSR: outputs follow canonical order
    cs, cd, order = canonical_sorted(s, d)
    got, st2 = gpu_truss(csr_graph(n, cs, cd), **opt)
    np.testing.assert_array_equal(got, phi_ref[order])
    if sup_ref is not None:
        sup, tri = gpu_support(csr_graph(n, cs, cd))
        np.testing.assert_array_equal(sup, sup_ref[order])
        assert tri == sup_ref.sum() // 3
    return st


def test_example2_fixture():
    n, s, d, phi_paper = golden_io.fig2()
    say("case: Example 2 fixture")
    sup_ref, _ = oracle.support_fwd(n, s, d)
    for o in STRATS:
        st = _both_formats(n, s, d, phi_paper, sup_ref, **o)
        assert st["kmax"] == 5
    got, _ = gpu_truss(edges_graph(n, s, d))
    np.testing.assert_array_equal(got, phi_paper)


@pytest.mark.parametrize("k", [3, 4, 5, 9, 17, 40, 70])
def test_cliques(k):
    say(f"case: K_{k}")
    s, d = map(np.array, zip(*itertools.combinations(range(k), 2)))
    s, d = s.astype(np.int32), d.astype(np.int32)
    sup, tri = gpu_support(edges_graph(k, s, d))
    assert (sup == k - 2).all() and tri == k * (k - 1) * (k - 2) // 6
    for o in STRATS:
        got, st = gpu_truss(edges_graph(k, s, d), **o)
        assert (got == k).all() and st["kmax"] == k


def test_triangle_free():
    say("case: trees, stars, cycles")
    rng = np.random.default_rng(3)
    n = 500
    cases = [np.array([(int(rng.integers(0, v)), v) for v in range(1, n)]),
             np.array([(0, v) for v in range(1, n)]),
             np.array([(v, (v + 1) % n) for v in range(n)])]
    for e in cases:
        s, d = e[:, 0].astype(np.int32), e[:, 1].astype(np.int32)
        got, st = gpu_truss(edges_graph(n, s, d))
        assert (got == 2).all() and st["triangles"] == 0


def test_empty_and_isolated():
    say("case: empty graph")
    s = np.zeros(0, np.int32)
    got, st = gpu_truss(edges_graph(10, s, s))
    assert got.size == 0
    sup, tri = gpu_support(edges_graph(10, s, s))
    assert sup.size == 0 and tri == 0
    say("case: isolated vertices")
    s = np.array([0, 0, 1, 7], np.int32)
    d = np.array([1, 2, 2, 8], np.int32)
    got, _ = gpu_truss(edges_graph(1000, s, d))
    np.testing.assert_array_equal(got, [3, 3, 3, 2])


def test_random_small_graphs():
    rng = np.random.default_rng(2024)
    for trial in range(40):
        n = int(rng.integers(5, 300))
        p = float(rng.choice([0.02, 0.08, 0.2, 0.5]))
        n, s, d = graphgen.er(n, p, 1000 + trial)
        say(f"case: ER trial {trial} n={n} m={s.size}")
        phi, _ = oracle.truss(n, s, d)
        sup, _ = oracle.support_fwd(n, s, d)
        _both_formats(n, s, d, phi, sup, **STRATS[trial % len(STRATS)])


@pytest.mark.parametrize("seed", [1, 2, 3, 4, 5])
def test_er_n2000_p001(seed):
    """Erdos-Renyi G(2000, 0.01), the small parity configuration."""
    n, s, d = graphgen.er_small(seed)
    say(f"case: ER(2000, 0.01) seed={seed} m={s.size}")
    phi, _ = oracle.truss(n, s, d)
    sup, _ = oracle.support_fwd(n, s, d)
    _both_formats(n, s, d, phi, sup)


@pytest.mark.parametrize("scale", [10, 13, 15])
def test_rmat_vs_oracle(scale):
    n, s, d = graphgen.rmat(scale, 16, 7)
    say(f"case: R-MAT scale={scale} m={s.size}")
    phi, kmax = oracle.truss(n, s, d)
    sup, _ = oracle.support_fwd(n, s, d)
    for o in STRATS[:3]:
        st = _both_formats(n, s, d, phi, sup, **o)
        assert st["kmax"] == kmax


def test_chung_lu_cliques_vs_oracle():
    n, s, d = graphgen.chung_lu(20000, 2.1, 10.0, 2000.0, 4, 20, 80, 11)
    say(f"case: Chung-Lu 20000 with cliques m={s.size}")
    phi, kmax = oracle.truss(n, s, d)
    sup, _ = oracle.support_fwd(n, s, d)
    st = _both_formats(n, s, d, phi, sup)
    assert st["kmax"] == kmax


def test_heavy_walks_big_clique():
    """K_2300: every frontier walk exceeds the split threshold and the piece list
    overflows its capacity, so both heavy paths run."""
    k = 2300
    say(f"case: K_{k} heavy walks")
    s, d = map(np.array, zip(*itertools.combinations(range(k), 2)))
    s, d = s.astype(np.int32), d.astype(np.int32)
    g = csr_graph(k, s, d)
    for mode in (1, 2):
        for probe in (1, 2):
            got, st = gpu_truss(g, peel_mode=mode, peel_probe=probe)
            assert (got == k).all() and st["kmax"] == k


def test_hub_graph_heavy_mixed():
    """Two hubs joined to everything plus sparse noise: long walks at low levels."""
    rng = np.random.default_rng(5)
    n = 6000
    e = set()
    for v in range(2, n):
        e.add((0, v))
        e.add((1, v))
    e.add((0, 1))
    for _ in range(20000):
        a, b = sorted(rng.integers(2, n, size=2).tolist())
        if a != b:
            e.add((a, b))
    arr = np.array(sorted(e), dtype=np.int32)
    s, d = arr[:, 0].copy(), arr[:, 1].copy()
    say(f"case: two hubs n={n} m={s.size}")
    phi, _ = oracle.truss(n, s, d)
    sup, _ = oracle.support_fwd(n, s, d)
    _both_formats(n, s, d, phi, sup)


def test_determinism_and_strategy_invariance():
    n, s, d = graphgen.rmat(14, 16, 21)
    say(f"case: determinism R-MAT 14 m={s.size}")
    g = edges_graph(n, s, d)
    ref, _ = gpu_truss(g)
    for _ in range(3):
        got, _ = gpu_truss(g)
        np.testing.assert_array_equal(got, ref)
    for sup_s in (1, 2, 3):
        for mode in (1, 2):
            for probe in (1, 2):
                got, _ = gpu_truss(g, support_strategy=sup_s, peel_mode=mode, peel_probe=probe)
                np.testing.assert_array_equal(got, ref)
    T = lib()
    for sched in (T.SCHED_PLAIN, T.SCHED_HEURISTIC, T.SCHED_LEARNED):
        got, st = gpu_truss(g, scheduler=sched)
        np.testing.assert_array_equal(got, ref)


def test_metamorphic_relabel_union():
    n1, s1, d1 = graphgen.rmat(11, 8, 5)
    n2, s2, d2 = graphgen.er(700, 0.02, 6)
    say("case: relabel + disjoint union")
    g1, _ = gpu_truss(edges_graph(n1, s1, d1))
    g2, _ = gpu_truss(edges_graph(n2, s2, d2))
    s = np.concatenate([s1, s2 + n1]).astype(np.int32)
    d = np.concatenate([d1, d2 + n1]).astype(np.int32)
    gu, _ = gpu_truss(edges_graph(n1 + n2, s, d))
    np.testing.assert_array_equal(gu, np.concatenate([g1, g2]))
    rs, rd = graphgen.relabel(n1, s1, d1, 8)
    gr, _ = gpu_truss(edges_graph(n1, rs, rd))
    np.testing.assert_array_equal(gr, g1)


def test_validation_errors():
    T = lib()
    say("case: validation error codes")

    def code_edges(n, e):
        a = np.array(e, dtype=np.int32).reshape(-1, 2)
        try:
            gpu_truss(edges_graph(n, a[:, 0].copy(), a[:, 1].copy()))
        except T.TrussError as ex:
            return ex.code
        return 0

    assert code_edges(3, [(0, 1), (1, 2)]) == 0
    assert code_edges(2, [(0, 1), (1, 2)]) == T.E_RANGE
    assert code_edges(3, [(0, 1), (1, 1)]) == T.E_SELFLOOP
    assert code_edges(3, [(0, 1), (1, 0)]) == T.E_DUP
    assert code_edges(3, [(1, 1), (0, 5), (0, 2), (2, 0)]) == T.E_RANGE
    assert code_edges(3, [(1, 1), (0, 2), (2, 0)]) == T.E_SELFLOOP
    assert code_edges(3, [(0, -1)]) == T.E_RANGE

    def code_csr(n, rp, col):
        import torch
        from gpu_util import dev
        try:
            T.truss_decompose(T.Graph.from_csr(n, dev(np.array(rp, np.int64)), dev(np.array(col, np.int32))))
        except T.TrussError as ex:
            return ex.code
        return 0

    assert code_csr(3, [0, 1, 3, 4], [1, 0, 2, 1]) == 0
    assert code_csr(3, [0, 1, 3, 5], [1, 0, 2, 1]) == T.E_ROWPTR
    assert code_csr(3, [0, 2, 1, 4], [1, 0, 2, 1]) == T.E_ROWPTR
    assert code_csr(3, [0, 1, 3, 4], [7, 0, 2, 1]) == T.E_RANGE
    assert code_csr(3, [0, 1, 3, 4], [1, 2, 0, 1]) == T.E_UNSORTED
    assert code_csr(3, [0, 1, 3, 4], [1, 0, 0, 1]) == T.E_DUP
    assert code_csr(3, [0, 1, 1, 2], [1, 0]) == T.E_ASYM
    assert code_csr(3, [0, 1, 2, 2], [1, 2]) == T.E_ASYM
    # workspace too small
    n, s, d = graphgen.er(100, 0.1, 1)
    g = edges_graph(n, s, d)
    import torch
    ws = torch.empty(16, dtype=torch.uint8, device="cuda:0")
    with pytest.raises(T.TrussError) as ex:
        T.truss_decompose(g, ws=ws)
    assert ex.value.code == T.E_WORKSPACE


def test_subround_cap_reports_internal():
    T = lib()
    n, s, d = graphgen.rmat(12, 16, 2)
    say("case: sub-round cap")
    with pytest.raises(T.TrussError) as ex:
        gpu_truss(edges_graph(n, s, d), max_subrounds=3)
    assert ex.value.code == T.E_INTERNAL


def test_batch_small():
    T = lib()
    graphs = graphgen.batch(24, seed=3, n_lo=16, n_hi=600, d_lo=2.0, d_hi=20.0)
    vo, eo, s, d = graphgen.pack(graphs)
    say(f"case: batch of {len(graphs)} graphs, {s.size} edges")
    import torch
    from gpu_util import dev
    out, st = T.truss_batch(vo, eo, dev(s, torch.int32), dev(d, torch.int32))
    ref = np.concatenate([oracle.truss(n, a, b)[0] for n, a, b in graphs])
    np.testing.assert_array_equal(out.cpu().numpy(), ref)
