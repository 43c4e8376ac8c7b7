"""Writes the stored expected values of the full-size parity tests.

Calls only the CPU oracle (oracle/) on seeded synthetic inputs (graphgen/), never
the GPU library.  Each output file records, for one workload, the oracle's
truss numbers, supports and upper bounds in canonical edge order (u < v, sorted
by (u, v), which is also the library's CSR output order) and the core numbers
by vertex as SHA-256 digests of the int32 arrays, the triangle count, k_max,
c_max, the size of every k-class and the cohesion statistics of the k_max-truss
and the c_max-core (Table 6's columns).

Usage: python tests/golden/make_golden.py rmat20      (about 5 minutes, one core)
       python tests/golden/make_golden.py chunglu4m   (the 57M-edge Chung-Lu graph; about 8 minutes)
       python tests/golden/make_golden.py rmat24      (260M edges; hours, about 30 GB of RAM)
       python tests/golden/make_golden.py batch4096   (the 4096-graph batch; five processes)
       python tests/golden/make_golden.py --core rmat24  (core numbers only, added to an existing record)
       python tests/golden/make_golden.py --psi rmat24   (the upper bound only, likewise)
"""
import hashlib
import os
import sys
import time

HERE = os.path.dirname(os.path.abspath(__file__))
ROOT = os.path.dirname(os.path.dirname(HERE))
sys.path.insert(0, ROOT)

import numpy as np  # noqa: E402

import graphgen  # noqa: E402
import oracle  # noqa: E402

WORKLOADS = {
    "rmat20": lambda: graphgen.rmat20(1),
    "er2000": lambda: graphgen.er_small(1),
    "rmat16": lambda: graphgen.rmat(16, 16, 1),
    "chunglu4m": lambda: graphgen.chung_lu4m(1),
    "rmat24": lambda: graphgen.rmat24(1),
}


def digest(a):
    return hashlib.sha256(np.ascontiguousarray(a, dtype=np.int32).tobytes()).hexdigest()


def _batch_one(spec):
    n, s, d = graphgen.batch_graph(spec)
    phi, kmax = oracle.truss(n, s, d)
    return phi, kmax, s.size


def batch_main(workers=5):
    """The 4096-graph batch: truss numbers of every graph, concatenated in
    batch order, as one digest; per-graph k_max and edge counts alongside."""
    from multiprocessing import Pool
    specs = graphgen.batch_specs(4096, 1)
    t0 = time.time()
    with Pool(workers) as pool:
        res = pool.map(_batch_one, specs, chunksize=16)
    phi = np.concatenate([r[0] for r in res])
    kmax = [int(r[1]) for r in res]
    ms = [int(r[2]) for r in res]
    h = hashlib.sha256(np.ascontiguousarray(phi, dtype=np.int32).tobytes()).hexdigest()
    hist = np.bincount(phi)
    lines = [
        "# Oracle results for the batch of 4096 graphs (seed 1), edges in batch order.",
        "# Written by tests/golden/make_golden.py batch4096 from oracle.truss, one call per graph",
        "# (%.0f s on %d cores)." % (time.time() - t0, workers),
        "graphs: 4096",
        "m: %d" % phi.size,
        "kmax: %d" % max(kmax),
        "truss_sha256: %s" % h,
        "class_sizes: %s" % " ".join("%d:%d" % (k, c) for k, c in enumerate(hist) if c),
        "graph_kmax: %s" % " ".join(map(str, kmax)),
        "graph_m: %s" % " ".join(map(str, ms)),
    ]
    path = os.path.join(HERE, "oracle_batch4096.txt")
    with open(path, "w") as f:
        f.write("\n".join(lines) + "\n")
    print("\n".join(lines[:8]))


def main(name):
    n, s, d = WORKLOADS[name]()
    t0 = time.time()
    sup, tri = oracle.support_fwd(n, s, d)
    phi, kmax = oracle.truss(n, s, d)
    psi = oracle.upper_bound(n, s, d, sup)
    core, cmax = oracle.core_numbers(n, s, d)
    coh = oracle.cohesion(n, s, d, phi=phi, core=core)
    hist = np.bincount(phi, minlength=kmax + 1)
    lines = [
        "# Oracle results for workload %s (seed 1), canonical edge order." % name,
        "# Written by tests/golden/make_golden.py from oracle.support_fwd, oracle.truss, oracle.upper_bound,",
        "# oracle.core_numbers and oracle.cohesion",
        "# (%.0f s on one core)." % (time.time() - t0),
        "n: %d" % n,
        "m: %d" % s.size,
        "triangles: %d" % tri,
        "kmax: %d" % kmax,
        "truss_sha256: %s" % digest(phi),
        "support_sha256: %s" % digest(sup),
        "psi_sha256: %s" % digest(psi),
        "core_sha256: %s" % digest(core),
        "cmax: %d" % cmax,
        "cohesion: %s" % " ".join("%s=%r" % (k, v) for k, v in coh.items()),
        "class_sizes: %s" % " ".join("%d:%d" % (k, c) for k, c in enumerate(hist) if c),
    ]
    path = os.path.join(HERE, "oracle_%s.txt" % name)
    with open(path, "w") as f:
        f.write("\n".join(lines) + "\n")
    print("\n".join(lines))


def core_main(name):
    """Adds the core-number digest and c_max to an existing record (for
    records written before those fields existed; the truss numbers the
    cohesion statistics need are not recomputed)."""
    path = os.path.join(HERE, "oracle_%s.txt" % name)
    text = open(path).read()
    if "core_sha256:" in text:
        print("record already has core numbers")
        return
    n, s, d = WORKLOADS[name]()
    t0 = time.time()
    core, cmax = oracle.core_numbers(n, s, d)
    lines = ["# core numbers added by tests/golden/make_golden.py --core %s from oracle.core_numbers (%.0f s)"
             % (name, time.time() - t0), "core_sha256: %s" % digest(core), "cmax: %d" % cmax]
    with open(path, "a") as f:
        f.write("\n".join(lines) + "\n")
    print("\n".join(lines))


def psi_main(name):
    """Adds the upper-bound digest to an existing record (supports recomputed
    by the oracle and checked against the recorded digest first)."""
    path = os.path.join(HERE, "oracle_%s.txt" % name)
    text = open(path).read()
    if "psi_sha256:" in text:
        print("record already has psi")
        return
    n, s, d = WORKLOADS[name]()
    t0 = time.time()
    sup, _ = oracle.support_fwd(n, s, d)
    if "support_sha256: %s" % digest(sup) not in text:
        raise SystemExit("supports differ from the record")
    psi = oracle.upper_bound(n, s, d, sup)
    lines = ["# upper bound added by tests/golden/make_golden.py --psi %s from oracle.support_fwd and "
             "oracle.upper_bound (%.0f s)" % (name, time.time() - t0), "psi_sha256: %s" % digest(psi)]
    with open(path, "a") as f:
        f.write("\n".join(lines) + "\n")
    print("\n".join(lines))


if __name__ == "__main__":
    which = sys.argv[1] if len(sys.argv) > 1 else "rmat20"
    if which == "batch4096":
        batch_main()
    elif which == "--core":
        core_main(sys.argv[2])
    elif which == "--psi":
        psi_main(sys.argv[2])
    else:
        main(which)
