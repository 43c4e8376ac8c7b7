"""GPU tests of the learned scheduler: the network kernels against the float64
reference (oracle/mlp_oracle.py), the decisions against the network, the
invariance of results under every decision, and the exhaustive-timing record.
"""
import numpy as np
import pytest

import graphgen
import oracle
from gpu_util import csr_graph, dev, edges_graph, lib, say
from oracle import mlp_oracle as M

pytestmark = pytest.mark.gpu


def _torch():
    import torch
    return torch


@pytest.mark.parametrize("F,H,O,B", [(8, 32, 4, 1000), (6, 17, 3, 257), (3, 64, 8, 1), (16, 5, 1, 600)])
def test_forward_backward_match_reference(F, H, O, B):
    say(f"case: network F={F} H={H} O={O} B={B}")
    T = lib()
    rng = np.random.default_rng(F * 100 + H)
    p = rng.normal(0, 0.4, M.param_count(F, H, O)).astype(np.float32)
    X = rng.normal(0, 1.5, (B, F)).astype(np.float32)
    dY = rng.normal(0, 1, (B, O)).astype(np.float32)
    Y = T.mlp_forward(dev(p), dev(X), H, O).cpu().numpy()
    Yr, _ = M.forward(p.astype(np.float64), X.astype(np.float64), F, H, O)
    scale = np.abs(Yr).max() + 1e-30
    assert np.abs(Y - Yr).max() <= 1e-4 * scale
    g = T.mlp_backward(dev(p), dev(X), dev(dY), H).cpu().numpy()
    gr = M.backward(p.astype(np.float64), X.astype(np.float64), dY.astype(np.float64), F, H, O)
    assert np.abs(g - gr).max() <= 1e-4 * (np.abs(gr).max() + 1e-30)


def test_adam_steps_match_reference():
    say("case: Adam steps")
    T = lib()
    torch = _torch()
    F, H, O, B = 8, 24, 4, 700
    rng = np.random.default_rng(11)
    p = rng.normal(0, 0.4, M.param_count(F, H, O)).astype(np.float32)
    X = rng.normal(0, 1, (B, F)).astype(np.float32)
    Tg = rng.normal(0, 1, (B, O)).astype(np.float32)
    Wt = rng.uniform(0, 1, (B, O)).astype(np.float32)
    Wt[rng.uniform(size=(B, O)) < 0.2] = 0
    pd, md, vd = dev(p), torch.zeros(p.size, device="cuda:0"), torch.zeros(p.size, device="cuda:0")
    lr = 1e-3
    loss = T.mlp_train(pd, md, vd, dev(X), dev(Tg), dev(Wt), H, steps=3, step0=0, lr=lr)
    loss2 = T.mlp_train(pd, md, vd, dev(X), dev(Tg), dev(Wt), H, steps=2, step0=3, lr=lr)
    p64, m64, v64 = M.adam_train(p.astype(np.float64), np.zeros(p.size), np.zeros(p.size), X, Tg, Wt, F, H, O,
                                 5, 0, lr)
    got = pd.cpu().numpy()
    # every coordinate moves by about lr per step; compare the moves
    np.testing.assert_allclose(got - p, p64 - p, rtol=1e-3, atol=2e-3 * lr)
    np.testing.assert_allclose(md.cpu().numpy(), m64, rtol=1e-3, atol=1e-7)
    assert abs(loss2 - M.loss(p64, X, Tg, Wt, F, H, O)) <= 1e-4 * M.loss(p64, X, Tg, Wt, F, H, O)
    assert loss2 < loss


def test_sched_train_normalisation_and_fit():
    say("case: model fitting")
    T = lib()
    rng = np.random.default_rng(5)
    B = 900
    X = rng.normal(3, 2, (B, 8)).astype(np.float32)
    X[:, 6] = 0.5  # a constant feature
    # times with a clear structure: action 1 is best when feature 0 is large
    base = np.exp2(0.3 * X[:, 1:2])
    Tm = np.concatenate([base * (1 + (X[:, 0:1] > 3)), base * (1 + (X[:, 0:1] <= 3)), base * 3, base * 4],
                        axis=1).astype(np.float32)
    Tm[::7, 3] = 0  # unmeasured
    part, loss = T.sched_train(0, dev(X), dev(Tm), H=16, steps=1500, lr=1e-2, seed=3)
    part = part.cpu().numpy()
    assert part[0] == 1205 and tuple(part[1:4]) == (8, 16, 4)
    mu, isd, _, Y, Wt = M.sched_prep(X, Tm)
    np.testing.assert_allclose(part[4:12], mu, rtol=1e-5, atol=1e-5)
    np.testing.assert_allclose(part[12:20], isd, rtol=1e-4)
    # the reported loss is the reference loss of the fitted parameters
    params = part[20:].astype(np.float64)
    ref = M.loss(params, (X - part[4:12]) * part[12:20], Y, Wt, 8, 16, 4)
    assert abs(loss - ref) <= 1e-3 * ref + 1e-6
    # and the fitted network ranks the actions as the data do
    sc = M.model_scores(part, X)
    best = np.argmin(np.where(Tm > 0, Tm, np.inf), axis=1)
    assert (np.argmin(sc, axis=1) == best).mean() > 0.8


def _random_model(seed, H=8, scale=3.0):
    T = lib()
    rng = np.random.default_rng(seed)
    parts = []
    for F, A in ((8, 4), (6, 3)):
        mu = rng.normal(0, 1, F)
        isd = rng.uniform(0.2, 1, F)
        p = rng.normal(0, scale, M.param_count(F, H, A))
        parts.append(np.concatenate([[1205.0, F, H, A], mu, isd, p]))
    blob = np.concatenate(parts).astype(np.float32)
    assert blob.size == T.load_library().truss_sched_model_floats(H)
    return blob


def test_results_do_not_depend_on_decisions():
    T = lib()
    graphs = [("er2000", graphgen.er_small(2)), ("rmat14", graphgen.rmat(14, 16, 3)),
              ("chunglu", graphgen.chung_lu(20000, 2.1, 20.0, 2000.0, 4, 10, 40, 7))]
    for name, (n, s, d) in graphs:
        ref, _ = oracle.truss(n, s, d)
        g = edges_graph(n, s, d)
        seen = set()
        for seed in range(6):
            say(f"case: {name} random model {seed}")
            model = dev(_random_model(seed))
            o = T.make_options(scheduler=T.SCHED_LEARNED, model=model)
            out, st, tr = T.truss_decompose_traced(g, o)
            assert st["sched_fallback"] == 0
            np.testing.assert_array_equal(out.cpu().numpy(), ref)
            seen.update(tr["level_action"].tolist())
            # the device's choices are the network's argmin over the recorded features
            blob = _random_model(seed)
            n0 = T.sched_part_floats(0, 8)
            sc = M.model_scores(blob[:n0], tr["level_feat"])
            srt = np.sort(sc, axis=1)
            clear = srt[:, 1] - srt[:, 0] > 1e-3 * (1 + np.abs(srt[:, 0]))
            assert np.array_equal(np.argmin(sc, axis=1)[clear], tr["level_action"][clear])
            # support bins: the network's method when it beats the heuristic's
            # (hash; binary search in the last bin) by more than 0.25 in log2 ms
            ssc = M.model_scores(blob[n0:], np.array(tr["sup_feat"]))
            for b in range(4):
                allowed = [0, 1, 2] if b < 3 else [1, 2]
                s_b = ssc[b, allowed]
                if np.sort(s_b)[1] - np.sort(s_b)[0] <= 1e-3 * (1 + abs(s_b.min())):
                    continue
                best = allowed[int(np.argmin(s_b))]
                pref = 0 if b < 3 else 1
                gap = ssc[b, pref] - 0.25 - ssc[b, best]
                if abs(gap) > 1e-3 * (1 + abs(ssc[b, best])):
                    assert tr["sup_action"][b] == (best if gap > 0 else pref)
        assert len(seen) >= 2, "random models should exercise several level actions"


def test_malformed_model_falls_back():
    say("case: malformed model")
    T = lib()
    n, s, d = graphgen.er_small(3)
    ref, _ = oracle.truss(n, s, d)
    bad = _random_model(1)
    good = bad.copy()
    bad[0] = 7.0
    # valid headers but fewer floats than they ask for: the binding passes the
    # tensor's length and the library must not read past it
    truncated = (good[:4].copy(), good[:-1].copy(), np.concatenate([good, np.zeros(3, good.dtype)]))
    for model in (None, dev(bad)) + tuple(dev(t) for t in truncated):
        o = T.make_options(scheduler=T.SCHED_LEARNED, model=model)
        out, st = T.truss_decompose(edges_graph(n, s, d), o)
        assert st["sched_fallback"] == 1
        np.testing.assert_array_equal(out.cpu().numpy(), ref)


def test_exhaustive_record_is_consistent():
    """Level features are identical under every forced action (checked inside
    exhaustive()), each table row has a time for every action, and the
    per-level times add up to no more than the peeling time."""
    from paper_1205_6693_amd import sched
    T = lib()
    n, s, d = graphgen.rmat(15, 16, 4)
    ref, kmax = oracle.truss(n, s, d)
    g = csr_graph(n, s, d)
    say("case: exhaustive timing, R-MAT 15")
    tab = sched.exhaustive(g, repeats=1)
    np.testing.assert_array_equal(tab["out"], ref)
    L = tab["level_feat"].shape[0]
    assert L == len(np.unique(ref)) and L >= 3
    assert np.all(tab["level_ms"] > 0)
    assert np.all(tab["sup_ms"][:3] > 0) and tab["sup_ms"][3, 0] == 0
    # features: log2(k) rises with the level; live edges fall
    assert np.all(np.diff(tab["level_feat"][:, 3]) > 0)
    assert np.all(np.diff(tab["level_feat"][:, 0]) < 0)
    for a in range(4):
        assert sched.regret(tab["level_ms"], np.full(L, a)) >= 1.0
    assert sched.regret(tab["level_ms"], np.argmin(tab["level_ms"], axis=1)) == 1.0


def test_learned_scheduler_gain():
    """What the trained network (the committed model file) gains over the
    method without it, on held-out graphs (seeds and shapes not used in
    training): the learned form beats the plain form end to end, reaches at
    least the heuristic's speed within noise, and its per-level choices stay
    within 10% of the exhaustive per-level best.  Outputs stay bit-exact."""
    import os
    from paper_1205_6693_amd import sched, train_sched
    T = lib()
    assert os.path.exists(sched.MODEL_PATH), "scheduler model file missing"
    model = sched.load_model()
    for spec in [("rmat", 17, 16, 3000), ("cl", 1 << 18, 30, 32, 50, 400, 3001)]:
        say(f"case: gain on {spec}")
        n, s, d = train_sched.make_graph(spec)
        ref, _ = oracle.truss(n, s, d)
        g = csr_graph(n, s, d)
        med = {}
        for name, kw in (("plain", dict(scheduler=T.SCHED_PLAIN)), ("heuristic", dict(scheduler=T.SCHED_HEURISTIC)),
                         ("learned", dict(scheduler=T.SCHED_LEARNED, model=model))):
            o = T.make_options(**kw)
            ts = []
            for _ in range(7):
                out, st = T.truss_decompose(g, o)
                ts.append(st["ms_total"])
                assert st["sched_fallback"] == 0
            np.testing.assert_array_equal(out.cpu().numpy(), ref)
            med[name] = float(np.median(ts[1:]))
        tab = sched.exhaustive(g, repeats=2)
        _, _, tr = T.truss_decompose_traced(g, T.make_options(scheduler=T.SCHED_LEARNED, model=model))
        reg = sched.regret(tab["level_ms"], tr["level_action"])
        say(f"  median ms {med}; learned per-level regret {reg:.3f}")
        assert med["learned"] < 0.95 * med["plain"]
        assert med["learned"] < 1.05 * med["heuristic"]
        assert reg <= 1.10
