"""Pins of the CPU oracle against what the paper and the mathematics fix.

Each test checks the oracle against something other than itself: the paper's
worked examples (tests/golden/), closed forms, brute force on tiny graphs, and
invariants that hold at any size.
"""
import itertools

import numpy as np
import pytest

import brute
import golden_io
import graphgen
import oracle


def _edges(edges):
    if not edges:
        return np.zeros(0, np.int32), np.zeros(0, np.int32)
    a = np.array(edges, dtype=np.int32)
    return a[:, 0].copy(), a[:, 1].copy()


# ---------------------------------------------------------------- worked examples

def test_example2_truss_numbers():
    """Example 2 (Figure 2): Phi_2..Phi_5 edge by edge, k_max = 5."""
    n, s, d, phi_paper = golden_io.fig2()
    phi, kmax = oracle.truss(n, s, d)
    assert kmax == 5
    np.testing.assert_array_equal(phi, phi_paper)
    # class sizes printed in Example 2: |Phi_2|=1, |Phi_3|=9, |Phi_4|=6, |Phi_5|=10
    assert np.bincount(phi, minlength=6)[2:].tolist() == [1, 9, 6, 10]


def test_example2_shuffled_and_reoriented():
    n, s, d, phi_paper = golden_io.fig2()
    for seed in range(5):
        rng = np.random.default_rng(seed)
        perm = rng.permutation(s.size)
        flip = rng.random(s.size) < 0.5
        s2 = np.where(flip, d[perm], s[perm]).astype(np.int32)
        d2 = np.where(flip, s[perm], d[perm]).astype(np.int32)
        phi, _ = oracle.truss(n, s2, d2)
        np.testing.assert_array_equal(phi, phi_paper[perm])


def test_example4_support():
    """Example 4: sup((d,g)) = 3."""
    n, s, d, _ = golden_io.fig2()
    sup_f, _ = oracle.support_fwd(n, s, d)
    sup_d, _ = oracle.support_def(n, s, d)
    for q, (u, v), _, val in golden_io.example4():
        if q == "sup":
            i = golden_io.edge_index(s, d, u, v)
            assert sup_f[i] == val and sup_d[i] == val


def test_example4_upper_bound():
    """Example 4: x_d = 3 and x_g = 2 for the edge (d,g), so psi((d,g)) = 4;
    every edge of the 5-class has psi = 5; Example 5: psi((e,d)) = 5."""
    n, s, d, phi = golden_io.fig2()
    psi = oracle.upper_bound(n, s, d)
    sup, _ = oracle.support_fwd(n, s, d)
    edges = list(zip(s.tolist(), d.tolist()))
    for q, (u, v), w, val in golden_io.example4():
        i = golden_io.edge_index(s, d, u, v)
        if q == "psi":
            assert psi[i] == val
        elif q == "x":
            assert brute.x_brute(n, edges, sup, i, w) == val
    assert (psi[phi == 5] == 5).all()


def test_example5_top_two_classes():
    """Example 5: the top-2 classes of the Figure 2 graph are the K_5 on
    {a,b,c,d,e} (the 5-class) and the K_4 on {f,h,i,j} (the 4-class)."""
    n, s, d, phi = golden_io.fig2()
    top, kmin = oracle.top_classes(oracle.truss(n, s, d)[0], 2)
    assert kmin == 4
    names = "abcdefghijkl"
    k5 = set(itertools.combinations("abcde", 2))
    k4 = set(itertools.combinations("fhij", 2))
    for i, (u, v) in enumerate(zip(s, d)):
        pair = tuple(sorted((names[u], names[v])))
        assert top[i] == (5 if pair in k5 else 4 if pair in k4 else 0)


def test_upper_bound_brute_and_lemma2():
    """psi by the oracle equals Procedure 6 evaluated by its words, and
    phi <= psi <= sup + 2 (Lemma 2) on random graphs."""
    rng = np.random.default_rng(17)
    for trial in range(120):
        n = int(rng.integers(3, 30))
        edges = brute.random_graph(rng, n, float(rng.uniform(0.1, 0.8)))
        if not edges:
            continue
        s, d = _edges(edges)
        sup, _ = oracle.support_fwd(n, s, d)
        psi = oracle.upper_bound(n, s, d)
        np.testing.assert_array_equal(psi, brute.psi_brute(n, edges, sup))
        phi, _ = oracle.truss(n, s, d)
        assert (phi <= psi).all() and (psi <= sup + 2).all() and (psi >= 2).all()


def test_upper_bound_closed_forms():
    """K_k: x = k-2 at both ends, psi = k = phi; a star: psi = 2."""
    for k in (3, 4, 7, 12):
        s, d = _edges(list(itertools.combinations(range(k), 2)))
        assert (oracle.upper_bound(k, s, d) == k).all()
    s, d = _edges([(0, v) for v in range(1, 40)])
    assert (oracle.upper_bound(40, s, d) == 2).all()


def test_core_numbers_brute_and_closed_forms():
    """Core numbers by the bucket method equal repeated min-degree deletion;
    K_k: k-1; cycles: 2; stars and paths: 1; and every k-truss lies in the
    (k-1)-core (phi(e) - 1 <= core of both ends)."""
    rng = np.random.default_rng(23)
    for trial in range(150):
        n = int(rng.integers(2, 40))
        edges = brute.random_graph(rng, n, float(rng.uniform(0.05, 0.7)))
        if not edges:
            continue
        s, d = _edges(edges)
        core, cmax = oracle.core_numbers(n, s, d)
        ref = brute.kcore_numbers(n, edges)
        np.testing.assert_array_equal(core, ref)
        assert cmax == ref.max()
        phi, _ = oracle.truss(n, s, d)
        assert (phi - 1 <= np.minimum(core[s], core[d])).all()
    k = 9
    s, d = _edges(list(itertools.combinations(range(k), 2)))
    assert (oracle.core_numbers(k, s, d)[0] == k - 1).all()
    s, d = _edges([(v, (v + 1) % 30) for v in range(30)])
    assert (oracle.core_numbers(30, s, d)[0] == 2).all()
    s, d = _edges([(0, v) for v in range(1, 30)] + [(30 + v, 31 + v) for v in range(20)])
    assert (oracle.core_numbers(51, s, d)[0] == 1).all()


def test_cohesion_statistics():
    """Table 6's columns: K_k gives V = k, E = k(k-1)/2, k_max = k, c_max = k-1
    and clustering 1 for both; a cycle has clustering 0; random graphs agree
    with a brute-force count of adjacent neighbour pairs; on the Example 2
    graph the 5-truss and the 4-core are both the K_5 on {a,b,c,d,e}."""
    k = 7
    s, d = _edges(list(itertools.combinations(range(k), 2)))
    st = oracle.cohesion(k, s, d)
    assert st == {"V_T": k, "E_T": k * (k - 1) // 2, "kmax": k, "CC_T": 1.0,
                  "V_C": k, "E_C": k * (k - 1) // 2, "cmax": k - 1, "CC_C": 1.0}
    s, d = _edges([(v, (v + 1) % 12) for v in range(12)])
    st = oracle.cohesion(12, s, d)
    assert st["CC_T"] == 0.0 and st["E_T"] == 12 and st["kmax"] == 2
    n, s, d, _ = golden_io.fig2()
    st = oracle.cohesion(n, s, d)
    assert (st["V_T"], st["E_T"], st["kmax"], st["V_C"], st["E_C"], st["cmax"]) == (5, 10, 5, 5, 10, 4)
    rng = np.random.default_rng(29)
    for trial in range(40):
        n = int(rng.integers(5, 35))
        edges = brute.random_graph(rng, n, float(rng.uniform(0.15, 0.8)))
        if not edges:
            continue
        s, d = _edges(edges)
        phi, kmax = oracle.truss(n, s, d)
        core, cmax = oracle.core_numbers(n, s, d)
        st = oracle.cohesion(n, s, d, phi, core)
        T = [e for e, p in zip(edges, phi) if p == kmax]
        C = [(u, v) for u, v in edges if core[u] == cmax and core[v] == cmax]
        vt, et, cct = brute.clustering_brute(n, T)
        vc, ec, ccc = brute.clustering_brute(n, C)
        assert (st["V_T"], st["E_T"], st["V_C"], st["E_C"]) == (vt, et, vc, ec)
        assert abs(st["CC_T"] - cct) < 1e-12 and abs(st["CC_C"] - ccc) < 1e-12


# ---------------------------------------------------------------- closed forms

@pytest.mark.parametrize("k", [3, 4, 5, 8, 13])
def test_clique_closed_form(k):
    """K_k: every edge lies in k-2 triangles and has truss number k."""
    edges = list(itertools.combinations(range(k), 2))
    s, d = _edges(edges)
    sup, tri = oracle.support_fwd(k, s, d)
    assert (sup == k - 2).all()
    assert tri == k * (k - 1) * (k - 2) // 6
    phi, kmax = oracle.truss(k, s, d)
    assert (phi == k).all() and kmax == k


def test_trees_cycles_stars():
    """Triangle-free graphs: sup = 0 and truss number 2 everywhere."""
    rng = np.random.default_rng(7)
    graphs = []
    n = 50
    graphs.append((n, [(int(rng.integers(0, v)), v) for v in range(1, n)]))   # random tree
    graphs.append((n, [(0, v) for v in range(1, n)]))                          # star
    graphs.append((n, [(v, (v + 1) % n) for v in range(n)]))                   # cycle C_50
    graphs.append((4, [(0, 1), (1, 2), (2, 3), (3, 0)]))                       # C_4
    for n, edges in graphs:
        s, d = _edges(edges)
        sup, tri = oracle.support_fwd(n, s, d)
        phi, _ = oracle.truss(n, s, d)
        assert tri == 0 and (sup == 0).all() and (phi == 2).all()


def test_empty_and_isolated():
    s, d = _edges([])
    phi, kmax = oracle.truss(5, s, d)
    assert phi.size == 0 and kmax == 0
    sup, tri = oracle.support_fwd(5, s, d)
    assert sup.size == 0 and tri == 0


# ---------------------------------------------------------------- brute force

def test_random_tiny_vs_definition_peeling():
    """Oracle == Definition 2 by repeated deletion, on random graphs n <= 40."""
    rng = np.random.default_rng(12345)
    for trial in range(300):
        n = int(rng.integers(2, 41))
        p = float(rng.choice([0.05, 0.15, 0.3, 0.5, 0.8]))
        edges = brute.random_graph(rng, n, p)
        s, d = _edges(edges)
        s, d = graphgen.shuffle(s, d, trial)
        e = list(zip(s.tolist(), d.tolist()))
        phi, _ = oracle.truss(n, s, d)
        np.testing.assert_array_equal(phi, brute.truss_by_peeling(n, e), err_msg=f"trial {trial}")
        sup_f, tri = oracle.support_fwd(n, s, d)
        sup_d, tri_d = oracle.support_def(n, s, d)
        sb = brute.support_brute(n, e)
        np.testing.assert_array_equal(sup_f, sb)
        np.testing.assert_array_equal(sup_d, sb)
        if n <= 25:
            assert tri == tri_d == brute.triangles_brute(n, e)
        assert sup_f.sum() == 3 * tri


def test_random_tiny_vs_literal_definition():
    """Oracle == literal Definition 2 (all edge subsets), m <= 16."""
    rng = np.random.default_rng(777)
    done = 0
    while done < 60:
        n = int(rng.integers(4, 9))
        edges = brute.random_graph(rng, n, float(rng.choice([0.4, 0.6, 0.9])))
        if not 1 <= len(edges) <= 16:
            continue
        s, d = _edges(edges)
        phi, _ = oracle.truss(n, s, d)
        np.testing.assert_array_equal(phi, brute.truss_literal(n, edges))
        done += 1


def test_literal_definition_on_named_graphs():
    # K_4 plus a pendant triangle sharing a vertex; the "bowtie"; K_5 minus an edge
    cases = [
        (6, [(0, 1), (0, 2), (0, 3), (1, 2), (1, 3), (2, 3), (3, 4), (3, 5), (4, 5)]),
        (5, [(0, 1), (0, 2), (1, 2), (2, 3), (2, 4), (3, 4)]),
        (5, [e for e in itertools.combinations(range(5), 2) if e != (0, 1)]),
    ]
    for n, edges in cases:
        s, d = _edges(edges)
        phi, _ = oracle.truss(n, s, d)
        np.testing.assert_array_equal(phi, brute.truss_literal(n, edges))


# ---------------------------------------------------------------- invariants at size

def _check_invariants(n, s, d, phi, sup):
    # 2 <= phi <= sup + 2 (Definition 2)
    assert (phi >= 2).all() and (phi <= sup + 2).all()
    # a k-truss is a (k-1)-core: each vertex on an edge of truss number >= k
    # has at least k-1 such edges
    kmax = int(phi.max()) if phi.size else 2
    for k in range(3, kmax + 1):
        sel = phi >= k
        deg = np.bincount(np.concatenate([s[sel], d[sel]]), minlength=n)
        touched = deg > 0
        assert (deg[touched] >= k - 1).all(), k


def _h_index_fixpoint(n, s, d, phi):
    """phi(e)-2 = the largest h such that at least h triangles on e have both
    other edges with truss number >= h+2 (necessary condition, Definition 2)."""
    nb = [dict() for _ in range(n)]
    for i, (u, v) in enumerate(zip(s.tolist(), d.tolist())):
        nb[u][v] = i
        nb[v][u] = i
    for i, (u, v) in enumerate(zip(s.tolist(), d.tolist())):
        vals = sorted((min(phi[nb[u][w]], phi[nb[v][w]]) - 2
                       for w in nb[u].keys() & nb[v].keys()), reverse=True)
        h = 0
        for j, x in enumerate(vals):
            if x >= j + 1:
                h = j + 1
        assert h == phi[i] - 2, (i, h, phi[i])


def test_invariants_rmat_small():
    n, s, d = graphgen.rmat(12, 16, 3)
    phi, kmax = oracle.truss(n, s, d)
    sup, tri = oracle.support_fwd(n, s, d)
    sup_d, _ = oracle.support_def(n, s, d)
    np.testing.assert_array_equal(sup, sup_d)
    assert sup.sum() == 3 * tri
    _check_invariants(n, s, d, phi, sup)
    _h_index_fixpoint(n, s, d, phi)
    # Lemma 1: truss numbers in any subgraph are at most those in G
    keep = np.random.default_rng(1).random(s.size) < 0.7
    phi_sub, _ = oracle.truss(n, s[keep], d[keep])
    assert (phi_sub <= phi[keep]).all()


def test_planted_cliques_and_union():
    """A clique of size c lies in a c-truss; a disjoint union decomposes into
    the concatenation of its parts' truss numbers; relabelling is harmless."""
    n1, s1, d1 = graphgen.chung_lu(3000, 2.1, 8.0, 300.0, 3, 10, 25, 5)
    sizes = graphgen.chung_lu_clique_sizes(3, 10, 25, 5)
    phi1, k1 = oracle.truss(n1, s1, d1)
    assert k1 >= sizes.max()
    n2, s2, d2 = graphgen.er(500, 0.03, 9)
    phi2, _ = oracle.truss(n2, s2, d2)
    s = np.concatenate([s1, s2 + n1]).astype(np.int32)
    d = np.concatenate([d1, d2 + n1]).astype(np.int32)
    phi, _ = oracle.truss(n1 + n2, s, d)
    np.testing.assert_array_equal(phi, np.concatenate([phi1, phi2]))
    rs, rd = graphgen.relabel(n1, s1, d1, 3)
    phir, _ = oracle.truss(n1, rs, rd)
    np.testing.assert_array_equal(phir, phi1)


# ---------------------------------------------------------------- validation

def test_validation_codes():
    E = oracle
    s, d = _edges([(0, 1), (1, 2)])
    assert E.validate_edges(3, s, d) == 0
    assert E.validate_edges(2, s, d) == -E.RANGE
    assert E.validate_edges(3, *_edges([(0, 1), (1, 1)])) == -E.SELFLOOP
    assert E.validate_edges(3, *_edges([(0, 1), (1, 0)])) == -E.DUP
    assert E.validate_edges(3, *_edges([(0, 1), (0, 1)])) == -E.DUP
    # smallest magnitude wins: range beats self-loop beats duplicate
    assert E.validate_edges(3, *_edges([(1, 1), (0, 5), (0, 2), (2, 0)])) == -E.RANGE
    assert E.validate_edges(3, *_edges([(1, 1), (0, 2), (2, 0)])) == -E.SELFLOOP
    assert E.validate_edges(-1, *_edges([])) == -E.INVAL
    # CSR
    rp, col = graphgen.to_csr(3, np.array([0, 1], np.int32), np.array([1, 2], np.int32))
    assert E.validate_csr(3, 2, rp, col) == 0
    assert E.validate_csr(3, 3, rp, col) == -E.ROWPTR
    bad = col.copy(); bad[0] = 7
    assert E.validate_csr(3, 2, rp, bad) == -E.RANGE
    # row 1 lists neighbour 0 twice
    assert E.validate_csr(3, 2, np.array([0, 1, 3, 4], np.int64), np.array([1, 0, 0, 1], np.int32)) == -E.DUP
    assert E.validate_csr(3, 2, np.array([0, 1, 3, 4], np.int64), np.array([1, 2, 0, 1], np.int32)) == -E.UNSORTED
    # asymmetric: 0->1 and 1->2 only listed one way
    assert E.validate_csr(3, 1, np.array([0, 1, 1, 2], np.int64), np.array([1, 0], np.int32)) == -E.ASYM


def test_csr_to_edges_canonical_order():
    n, s, d = graphgen.er(200, 0.05, 4)
    rp, col = graphgen.to_csr(n, s, d)
    assert oracle.validate_csr(n, s.size, rp, col) == 0
    s2, d2 = oracle.csr_to_edges(n, s.size, rp, col)
    np.testing.assert_array_equal(s2, s)
    np.testing.assert_array_equal(d2, d)


@pytest.mark.parametrize("name", ["er2000", "rmat16"])
def test_stored_oracle_records(name):
    """The stored full-size records (tests/golden/oracle_<name>.txt) are what
    the oracle computes today: the generator output is canonical and the
    digests, triangle count and class sizes match a fresh oracle run."""
    import golden_io
    rec = golden_io.oracle_record(name)
    assert rec is not None
    n, s, d = graphgen.er_small(1) if name == "er2000" else graphgen.rmat(16, 16, 1)
    assert n == rec["n"] and s.size == rec["m"]
    sup, tri = oracle.support_fwd(n, s, d)
    phi, kmax = oracle.truss(n, s, d)
    assert tri == rec["triangles"] and kmax == rec["kmax"]
    assert golden_io.int32_digest(sup) == rec["support_sha256"]
    assert golden_io.int32_digest(phi) == rec["truss_sha256"]
    assert golden_io.int32_digest(oracle.upper_bound(n, s, d, sup)) == rec["psi_sha256"]
    hist = np.bincount(phi)
    assert {k: int(c) for k, c in enumerate(hist) if c} == rec["class_sizes"]
