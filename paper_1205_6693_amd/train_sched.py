"""Trains the learned scheduler's model file (sched_model.json beside this file).

Training graphs are seeded synthetic graphs (seeds >= 1000): R-MAT (scales
14-23, edge factors 8-128; scale 23 with edge factor 20 is above 2^27 edges,
so its levels are timed on the wide peeling shape), Chung-Lu
power-law graphs with planted cliques (up to 2^21 vertices, cliques up to 4600
vertices) and Erdos-Renyi graphs.  For each, exhaustive timing (sched.exhaustive) records the time of
every action at every decision; both model parts are then fitted on the GPU by
the library's own forward, backward and Adam kernels.  Held-out graphs
(other seeds and shapes) report the regret of each scheduler against the
per-decision best.

usage (repository root, one GPU):
    python -m paper_1205_6693_amd.train_sched [--out PATH] [--save-tables NPZ]
                                              [--tables NPZ] [--steps N] [--hidden H]
"""
from __future__ import annotations

import argparse
import json
import os
import sys
import time

import numpy as np

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
if ROOT not in sys.path:
    sys.path.insert(0, ROOT)

import graphgen  # noqa: E402

from . import Graph, make_options, SCHED_HEURISTIC, SCHED_LEARNED, SCHED_PLAIN, truss_decompose  # noqa: E402
from . import sched, truss_decompose_traced  # noqa: E402

TRAIN = [
    ("rmat", 14, 16, 1000), ("rmat", 15, 8, 1001), ("rmat", 16, 16, 1002), ("rmat", 16, 32, 1003),
    ("rmat", 17, 16, 1004), ("rmat", 18, 16, 1005), ("rmat", 18, 8, 1006), ("rmat", 19, 16, 1007),
    ("rmat", 17, 32, 1008),
    ("cl", 1 << 16, 30, 16, 20, 120, 1010), ("cl", 1 << 18, 30, 32, 30, 250, 1011),
    ("cl", 1 << 19, 20, 32, 40, 300, 1012), ("cl", 1 << 20, 30, 64, 50, 500, 1013),
    ("cl", 1 << 17, 40, 8, 100, 400, 1014),
    # large planted cliques put vertices in the two high out-degree support bins
    ("cl", 1 << 16, 20, 4, 1100, 2000, 1015), ("cl", 1 << 17, 20, 1, 4300, 4600, 1016),
    ("rmat", 15, 128, 1009),
    ("er", 20000, 1e-3, 1020), ("er", 100000, 3e-4, 1021), ("er", 4000, 1e-2, 1022),
    # larger graphs (still below the R-MAT 24 and Chung-Lu 4M workloads)
    ("rmat", 20, 16, 1030), ("rmat", 21, 16, 1031), ("rmat", 22, 16, 1032), ("rmat", 21, 8, 1033),
    ("cl", 1 << 21, 30, 64, 50, 500, 1034),
    # above 2^27 edges, where the peeling kernel takes its wide shape
    ("rmat", 23, 20, 1035),
]
HELDOUT = [("rmat", 17, 16, 2000), ("cl", 1 << 19, 30, 48, 50, 400, 2001), ("rmat", 19, 12, 2002)]


def make_graph(spec):
    kind = spec[0]
    if kind == "rmat":
        _, scale, ef, seed = spec
        return graphgen.rmat(scale, ef, seed)
    if kind == "cl":
        _, n, mean, ncl, lo, hi, seed = spec
        return graphgen.chung_lu(n, 2.1, float(mean), float(min(200000, n // 4)), ncl, lo, hi, seed)
    _, n, p, seed = spec
    return graphgen.er(n, p, seed)


def to_device(n, s, d):
    import torch
    rp, col = graphgen.to_csr(n, s, d)
    return Graph.from_csr(n, torch.from_numpy(rp).cuda(), torch.from_numpy(col).cuda())


def collect(specs, repeats=2):
    tables = []
    for spec in specs:
        t0 = time.time()
        n, s, d = make_graph(spec)
        g = to_device(n, s, d)
        tab = sched.exhaustive(g, repeats=repeats)
        tab.pop("out")
        tab["spec"] = list(spec)
        tables.append(tab)
        print("traced %-40s m=%-9d levels=%-4d %.1fs" % (spec, s.size, tab["level_feat"].shape[0], time.time() - t0),
              flush=True)
    return tables


def save_tables(tables, path):
    arrs = {}
    for i, t in enumerate(tables):
        for k in ("level_feat", "level_ms", "sup_feat", "sup_ms"):
            arrs["%d_%s" % (i, k)] = np.asarray(t[k])
        arrs["%d_spec" % i] = np.array(json.dumps(t["spec"]))
    np.savez(path, **arrs)


def load_tables(path):
    z = np.load(path)
    n = len({k.split("_")[0] for k in z.files})
    return [{"level_feat": z["%d_level_feat" % i], "level_ms": z["%d_level_ms" % i],
             "sup_feat": z["%d_sup_feat" % i], "sup_ms": z["%d_sup_ms" % i],
             "spec": json.loads(str(z["%d_spec" % i]))} for i in range(n)]


def evaluate(model, specs, repeats=3):
    """Regret of each scheduler's choices against the exhaustive table, and
    end-to-end time per scheduler (median of `repeats`)."""
    rows = []
    for spec in specs:
        n, s, d = make_graph(spec)
        g = to_device(n, s, d)
        tab = sched.exhaustive(g, repeats=2)
        row = {"spec": spec, "m": int(s.size)}
        for name, kw in (("plain", dict(scheduler=SCHED_PLAIN)), ("heuristic", dict(scheduler=SCHED_HEURISTIC)),
                         ("learned", dict(scheduler=SCHED_LEARNED, model=model))):
            o = make_options(**kw)
            _, st, tr = truss_decompose_traced(g, o)
            row[name + "_peel_regret"] = sched.regret(tab["level_ms"], tr["level_action"])
            sm = tab["sup_ms"]
            acts = np.array(tr["sup_action"])
            row[name + "_sup_regret"] = sched.regret(sm, acts)
            ts = []
            for _ in range(repeats):
                _, st = truss_decompose(g, o)
                ts.append(st["ms_total"])
            row[name + "_ms"] = float(np.median(ts))
        row["oracle_peel_ms"] = float(np.min(tab["level_ms"], axis=1).sum())
        rows.append(row)
        print(json.dumps(row), flush=True)
    return rows


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--out", default=sched.MODEL_PATH)
    ap.add_argument("--save-tables", default=None)
    ap.add_argument("--tables", default=None, help="fit on saved tables instead of timing")
    ap.add_argument("--steps", type=int, default=4000)
    ap.add_argument("--hidden", type=int, default=32)
    ap.add_argument("--no-eval", action="store_true")
    a = ap.parse_args()
    tables = load_tables(a.tables) if a.tables else collect(TRAIN)
    if a.save_tables:
        save_tables(tables, a.save_tables)
    model, info = sched.fit(tables, H=a.hidden, steps=a.steps)
    meta = dict(info, hidden=a.hidden, steps=a.steps, train=[t["spec"] for t in tables])
    print(json.dumps(meta), flush=True)
    if not a.no_eval:
        meta["heldout"] = evaluate(model, HELDOUT)
    sched.save_model(model, a.out, meta)
    print("wrote", a.out, flush=True)


if __name__ == "__main__":
    main()
