"""Learned scheduler: exhaustive timing, model fitting and model files.

The scheduler picks, per support bin, the intersection method (LDS hash,
binary search, merge) and, per peeling level, the frontier mode (sparse
worklist or dense re-scan) and the membership probe (hash table or binary
search).  Every choice is exact, so the choice changes time, never results.

Exhaustive timing: one traced run per action with that action forced
everywhere.  The state at each level's decision (live edges, supports, row
compaction) does not depend on earlier choices, so the features of a level are
identical across the runs (checked) and the per-level times of different runs
can be compared: row i of the result holds the time of level i under every
action.  The best schedule is the per-row minimum; a scheduler's regret is
how much slower its choices are.

Fitting runs on the GPU through truss_sched_train (the library's own forward,
backward and Adam kernels); this module only stacks the traces.
"""
from __future__ import annotations

import json
import os

import numpy as np

from . import (PEEL_DENSE, PEEL_SPARSE, PROBE_BSEARCH, PROBE_HASH, SCHED_HEURISTIC, SCHED_PEEL_A,
               SCHED_SUP_A, SCHED_SUP_BINS, SUP_BSEARCH, SUP_HASH, SUP_MERGE, make_options,
               sched_part_floats, sched_train, truss_decompose_traced)

MODEL_PATH = os.path.join(os.path.dirname(os.path.abspath(__file__)), "sched_model.json")

# action a of a level: bit 0 = binary-search probe, bit 1 = dense frontier
PEEL_ACTIONS = [(PEEL_SPARSE, PROBE_HASH), (PEEL_SPARSE, PROBE_BSEARCH),
                (PEEL_DENSE, PROBE_HASH), (PEEL_DENSE, PROBE_BSEARCH)]
SUP_ACTIONS = [SUP_HASH, SUP_BSEARCH, SUP_MERGE]


def exhaustive(graph, repeats: int = 2, level_cap: int = 8192):
    """Times every action at every decision of one graph.

    Returns a dict with level_feat (L x 8), level_ms (L x 4), sup_feat (4 x 6),
    sup_ms (4 x 3, 0 where a method does not apply), and the truss output of
    the first run (for the caller's checks).  Times are the minimum over
    `repeats` runs."""
    feat = None
    lms = None
    sfeat = None
    sms = np.zeros((SCHED_SUP_BINS, SCHED_SUP_A))
    first_out = None
    for a, (mode, probe) in enumerate(PEEL_ACTIONS):
        sup = SUP_ACTIONS[a] if a < SCHED_SUP_A else SUP_HASH
        opts = make_options(support_strategy=sup, peel_mode=mode, peel_probe=probe, scheduler=SCHED_HEURISTIC)
        best_l = None
        best_s = None
        for _ in range(repeats):
            out, st, tr = truss_decompose_traced(graph, opts, level_cap=level_cap)
            if first_out is None:
                first_out = out.cpu().numpy()
            if feat is None:
                feat = tr["level_feat"].copy()
                lms = np.zeros((tr["levels"], SCHED_PEEL_A))
                sfeat = np.array(tr["sup_feat"])
            elif not np.array_equal(feat, tr["level_feat"]):
                raise RuntimeError("level features differ between actions")
            if not np.all(tr["level_action"] == a):
                raise RuntimeError("forced action not taken")
            best_l = tr["level_ms"] if best_l is None else np.minimum(best_l, tr["level_ms"])
            s_ms = np.array(tr["sup_ms"])
            best_s = s_ms if best_s is None else np.minimum(best_s, s_ms)
        lms[:, a] = best_l
        if a < SCHED_SUP_A:
            sms[:, a] = best_s
    # the last bin has no hash method (it falls back to binary search)
    sms[SCHED_SUP_BINS - 1, 0] = 0.0
    return {"level_feat": feat, "level_ms": lms, "sup_feat": sfeat, "sup_ms": sms, "out": first_out}


def regret(times, actions):
    """Time of the chosen actions over the per-row best (>= 1.0) for one
    exhaustive table (rows x actions; entries <= 0 are not allowed)."""
    t = np.where(times > 0, times, np.inf)
    chosen = t[np.arange(len(actions)), actions]
    return float(chosen.sum() / t.min(axis=1).sum())


def fit(tables, H: int = 32, steps: int = 4000, lr: float = 1e-2, seed: int = 1, device="cuda:0"):
    """Fits both model parts on a list of exhaustive() tables; returns
    (model float32 tensor, {"peel_loss", "sup_loss"})."""
    import torch
    Xp = np.concatenate([t["level_feat"] for t in tables]).astype(np.float32)
    Tp = np.concatenate([t["level_ms"] for t in tables]).astype(np.float32)
    Xs = np.concatenate([t["sup_feat"] for t in tables]).astype(np.float32)
    Ts = np.concatenate([t["sup_ms"] for t in tables]).astype(np.float32)
    keep = Xs[:, 0] > 0  # empty bins: nothing to decide
    Xs, Ts = Xs[keep], Ts[keep]
    n0, n1 = sched_part_floats(0, H), sched_part_floats(1, H)
    model = torch.empty(n0 + n1, dtype=torch.float32, device=device)
    _, lp = sched_train(0, torch.from_numpy(Xp).to(device), torch.from_numpy(Tp).to(device), H=H, steps=steps,
                        lr=lr, seed=seed, out=model[:n0])
    _, ls = sched_train(1, torch.from_numpy(Xs).to(device), torch.from_numpy(Ts).to(device), H=H, steps=steps,
                        lr=lr, seed=seed + 1, out=model[n0:])
    return model, {"peel_loss": lp, "sup_loss": ls, "peel_rows": int(len(Xp)), "sup_rows": int(len(Xs))}


def save_model(model, path: str = MODEL_PATH, meta: dict | None = None):
    vals = model.detach().cpu().numpy().astype(np.float32)
    with open(path, "w") as f:
        json.dump({"format": "truss-sched-1", "meta": meta or {},
                   "floats": [float(v) for v in vals]}, f, indent=0)


def load_model(path: str = MODEL_PATH, device="cuda:0"):
    """The model tensor for truss_options.model (device float32)."""
    import torch
    with open(path) as f:
        d = json.load(f)
    if d.get("format") != "truss-sched-1":
        raise ValueError("not a scheduler model file: %s" % path)
    return torch.tensor(np.array(d["floats"], dtype=np.float32), device=device)


def model_meta(path: str = MODEL_PATH) -> dict:
    with open(path) as f:
        return json.load(f).get("meta", {})
