"""GPU tests of Algorithm 1 (Section 3.1) as a comparator: the same truss
numbers as the oracle (bit-exact), and the merge work it reports equals its
closed form, the sum over vertices of deg(v)^2 in each stage (every edge merges
its two full rows once to count support and once when it leaves)."""
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


def _sum_deg2(n, s, d):
    deg = np.bincount(np.concatenate([s, d]), minlength=n).astype(np.int64)
    return int((deg * deg).sum())


def test_cohen_matches_oracle_and_work_closed_form():
    T = lib()
    for name, n, s, d in _graphs():
        say(f"case: algorithm 1 on {name}")
        ref, kmax = oracle.truss(n, s, d)
        ss, dd = graphgen.shuffle(s, d, 31)
        out, st = T.truss_cohen(edges_graph(n, ss, dd))
        ref_s, _ = oracle.truss(n, ss, dd)
        np.testing.assert_array_equal(out.cpu().numpy(), ref_s)
        assert st["kmax"] == kmax
        cs, cd, _ = canonical_sorted(s, d)
        out, st = T.truss_cohen(csr_graph(n, cs, cd))
        np.testing.assert_array_equal(out.cpu().numpy(), oracle.truss(n, cs, cd)[0])
        w = _sum_deg2(n, s, d)
        assert st["support_work"] == w and st["peel_work"] == w


def test_cohen_degenerate():
    T = lib()
    say("case: algorithm 1, no edges and one edge")
    out, st = T.truss_cohen(edges_graph(4, np.zeros(0, np.int32), np.zeros(0, np.int32)))
    assert out.numel() == 0 and st["kmax"] == 0
    out, st = T.truss_cohen(edges_graph(2, np.array([1], np.int32), np.array([0], np.int32)))
    assert out.cpu().tolist() == [2] and st["kmax"] == 2


@pytest.mark.parametrize("name", ["rmat16", "rmat20"])
def test_cohen_full_size(name):
    rec = golden_io.oracle_record(name)
    T = lib()
    gen = {"rmat16": lambda: graphgen.rmat(16, 16, 1), "rmat20": lambda: graphgen.rmat20(1)}[name]
    n, s, d = gen()
    say(f"case: algorithm 1 full size {name}")
    out, st = T.truss_cohen(csr_graph(n, s, d))
    say("stats", {k: st[k] for k in ("kmax", "levels", "subrounds", "ms_support", "ms_peel", "ms_total")})
    assert golden_io.int32_digest(out.cpu().numpy()) == rec["truss_sha256"]
    w = _sum_deg2(n, s, d)
    assert st["support_work"] == w and st["peel_work"] == w
