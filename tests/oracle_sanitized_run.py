"""Child process of test_oracle_sanitized.py: imports the oracle package copy
given as argv[1] (whose shared library was built with AddressSanitizer and
UndefinedBehaviorSanitizer) and drives every entry point over seeded random
graphs, including the error paths, with the results checked against brute
force (Definition 2 by repeated deletion) and against each other.  Any
out-of-bounds access or undefined operation in the oracle aborts the process.
"""
import os
import sys

import numpy as np

sys.path.insert(0, sys.argv[1])
sys.path.insert(1, os.path.dirname(os.path.abspath(__file__)))

import brute  # noqa: E402
import oracle  # noqa: E402

assert os.path.dirname(oracle.__file__) == os.path.join(sys.argv[1], "oracle"), oracle.__file__


def main():
    rng = np.random.default_rng(20120501)
    cases = 0
    for _ in range(int(sys.argv[2]) if len(sys.argv) > 2 else 120):
        n = int(rng.integers(1, 40))
        edges = brute.random_graph(rng, n, float(rng.choice([0.05, 0.2, 0.5, 0.9])))
        m = len(edges)
        flip = rng.random(m) < 0.5  # either orientation of each input pair
        s = np.array([v if f else u for (u, v), f in zip(edges, flip)], np.int32)
        d = np.array([u if f else v for (u, v), f in zip(edges, flip)], np.int32)
        phi, kmax = oracle.truss(n, s, d)
        if m <= 120:
            ref = brute.truss_by_peeling(n, list(zip(s.tolist(), d.tolist())))
            assert [int(x) for x in phi] == [int(x) for x in ref], (n, m)
        sup, tri = oracle.support_fwd(n, s, d)
        sup2, tri2 = oracle.support_def(n, s, d)
        assert (sup == sup2).all() and tri == tri2
        psi = oracle.upper_bound(n, s, d, sup)
        assert (phi <= psi).all()
        core, _ = oracle.core_numbers(n, s, d)
        if m:
            oracle.cohesion(n, s, d, phi, core)
            deg = np.bincount(np.concatenate([s, d]), minlength=n)
            for cap in (int(deg.max()), int(deg.max()) + 3, m + 1):
                for fp in (None, rng.integers(0, max(1, n // 3), size=n).astype(np.int32)):
                    try:
                        phib, lb, _ = oracle.bottom_up(n, s, d, cap, first_part=fp)
                    except oracle.OracleError as ex:
                        assert -ex.code in (oracle.CAP, oracle.STALL), ex.code
                        continue
                    assert (phib == phi).all() and (lb <= phi).all(), (n, m, cap)
        # symmetric CSR round trip and a corrupted copy
        a = np.concatenate([s, d])
        b = np.concatenate([d, s])
        o = np.lexsort((b, a))
        a, b = a[o], b[o]
        rp = np.zeros(n + 1, np.int64)
        np.add.at(rp, a + 1, 1)
        rp = np.cumsum(rp)
        assert oracle.validate_csr(n, m, rp, b) == 0
        es, _ = oracle.csr_to_edges(n, m, rp, b)
        assert es.size == m
        if m:
            bad = b.copy()
            bad[int(rng.integers(0, bad.size))] = n + 3
            assert oracle.validate_csr(n, m, rp, bad) != 0
        cases += 1
    for n, s, d in [(3, [0, 0], [1, 1]), (3, [0], [0]), (3, [0], [5]), (3, [-1], [1])]:
        s = np.array(s, np.int32)
        d = np.array(d, np.int32)
        assert oracle.validate_edges(n, s, d) != 0
        for f in (oracle.truss, oracle.core_numbers):
            try:
                f(n, s, d)
                raise AssertionError("invalid graph accepted")
            except oracle.OracleError:
                pass
    print("sanitized oracle ok: %d graphs" % cases, flush=True)


if __name__ == "__main__":
    main()
