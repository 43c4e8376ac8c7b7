"""GPU tests of the upper bound psi (Procedure 6) and the top-down top-t
classes (Algorithm 7) against the oracle, bit-exact, plus Lemma 2 at size."""
import itertools

import numpy as np
import pytest

import golden_io
import graphgen
import oracle
from gpu_util import canonical_sorted, csr_graph, edges_graph, lib, say

pytestmark = pytest.mark.gpu


def _graphs():
    n, s, d, _ = golden_io.fig2()
    out = [("example2", n, s, d)]
    k = 9
    cs, cd = map(np.array, zip(*itertools.combinations(range(k), 2)))
    out.append(("K9", k, cs.astype(np.int32), cd.astype(np.int32)))
    out.append(("star", 70, np.zeros(69, np.int32), np.arange(1, 70, dtype=np.int32)))
    out.append(("er2000", *graphgen.er_small(4)))
    out.append(("rmat13", *graphgen.rmat(13, 16, 8)))
    out.append(("chunglu", *graphgen.chung_lu(30000, 2.1, 20.0, 3000.0, 6, 20, 90, 9)))
    return out


def test_upper_bound_matches_oracle():
    T = lib()
    for name, n, s, d in _graphs():
        say(f"case: psi on {name}")
        ss, dd = graphgen.shuffle(s, d, 5)
        ref = oracle.upper_bound(n, ss, dd)
        got = T.truss_upper_bound(edges_graph(n, ss, dd)).cpu().numpy()
        np.testing.assert_array_equal(got, ref)
        cs, cd, order = canonical_sorted(s, d)
        got = T.truss_upper_bound(csr_graph(n, cs, cd)).cpu().numpy()
        np.testing.assert_array_equal(got, oracle.upper_bound(n, cs, cd))


FULL = {"er2000": lambda: graphgen.er_small(1), "rmat16": lambda: graphgen.rmat(16, 16, 1),
        "rmat20": lambda: graphgen.rmat20(1), "chunglu4m": lambda: graphgen.chung_lu4m(1),
        "rmat24": lambda: graphgen.rmat24(1)}


@pytest.mark.parametrize("name", list(FULL))
def test_upper_bound_full_size(name):
    rec = golden_io.oracle_record(name)
    if rec is None or "psi_sha256" not in rec:
        pytest.skip("no psi record for " + name)
    T = lib()
    say(f"case: psi full size {name}")
    n, s, d = FULL[name]()
    got = T.truss_upper_bound(csr_graph(n, s, d)).cpu().numpy()
    assert golden_io.int32_digest(got) == rec["psi_sha256"]


def test_lemma2_at_size():
    """phi <= psi on R-MAT 20 (phi itself is checked against the oracle's
    digest in the full-size parity test)."""
    T = lib()
    say("case: Lemma 2 on R-MAT 20")
    n, s, d = graphgen.rmat20(1)
    g = csr_graph(n, s, d)
    psi = T.truss_upper_bound(g)
    phi, _ = T.truss_decompose(g)
    assert bool((phi <= psi).all())
    sup, _ = T.truss_support(g)
    assert bool((psi <= sup + 2).all())


@pytest.mark.parametrize("t", [1, 2, 3, 7, 1000])
def test_topdown_matches_oracle(t):
    T = lib()
    for name, n, s, d in _graphs():
        say(f"case: top-{t} classes on {name}")
        ss, dd = graphgen.shuffle(s, d, 6)
        phi, kmax = oracle.truss(n, ss, dd)
        ref, kmin = oracle.top_classes(phi, t)
        got, gmin, gmax, st = T.truss_topdown(edges_graph(n, ss, dd), t)
        assert (gmin, gmax) == (kmin, kmax)
        np.testing.assert_array_equal(got.cpu().numpy(), ref)
        cs, cd, _ = canonical_sorted(s, d)
        ref_c, _ = oracle.top_classes(oracle.truss(n, cs, cd)[0], t)
        got, gmin, gmax, st = T.truss_topdown(csr_graph(n, cs, cd), t)
        assert (gmin, gmax) == (kmin, kmax)
        np.testing.assert_array_equal(got.cpu().numpy(), ref_c)


def test_topdown_planted_cliques_small_subgraph():
    """With planted cliques the top classes come from a small subgraph:
    the last subgraph decomposed is a small part of the graph."""
    T = lib()
    n, s, d = graphgen.chung_lu(200000, 2.1, 20.0, 20000.0, 16, 60, 200, 11)
    say(f"case: top-3 on a Chung-Lu graph with cliques, m={s.size}")
    phi, kmax = oracle.truss(n, s, d)
    ref, kmin = oracle.top_classes(phi, 3)
    got, gmin, gmax, st = T.truss_topdown(csr_graph(n, s, d), 3)
    assert gmax == kmax and gmin == kmin
    np.testing.assert_array_equal(got.cpu().numpy(), ref)
    assert st["m"] < s.size // 10


@pytest.mark.parametrize("name", ["rmat20", "chunglu4m", "rmat24"])
def test_topdown_full_size(name):
    """The top-t classes at full size: the full decomposition is checked against
    the oracle's digest and class sizes, and the top-down output must equal its
    classes above k_max - t (zero elsewhere)."""
    import torch
    rec = golden_io.oracle_record(name)
    if rec is None:
        pytest.skip("no record for " + name)
    T = lib()
    n, s, d = FULL[name]()
    g = csr_graph(n, s, d)
    phi, st = T.truss_decompose(g)
    assert golden_io.int32_digest(phi.cpu().numpy()) == rec["truss_sha256"]
    for t in (1, 3, 10):
        say(f"case: top-{t} classes at full size, {name}")
        got, kmin, kmax, tst = T.truss_topdown(g, t)
        assert kmax == rec["kmax"] and kmin == max(2, kmax - t + 1)
        ref = torch.where(phi >= kmin, phi, torch.zeros_like(phi))
        assert torch.equal(got, ref)
        sizes = {k: int(c) for k, c in rec["class_sizes"].items() if k >= kmin}
        vals, cnts = torch.unique(got[got > 0], return_counts=True)
        assert dict(zip(vals.tolist(), cnts.tolist())) == sizes
