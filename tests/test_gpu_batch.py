"""GPU tests of the batched path (truss_batch, batch plans, the autotuner):
every graph of a packed batch must get exactly the oracle's truss numbers of
that graph alone (triangles never cross graphs), for every built shape."""
import itertools

import numpy as np
import pytest

import golden_io
import graphgen
import oracle
from gpu_util import dev, lib, say

pytestmark = pytest.mark.gpu

SHAPES = [(b, i) for b in (256, 512, 1024) for i in (1, 2, 4)]


def _clique(k):
    s, d = map(np.array, zip(*itertools.combinations(range(k), 2)))
    return k, s.astype(np.int32), d.astype(np.int32)


def _mixed_batch(seed, count=40, n_hi=1500):
    gs = graphgen.batch(count, seed, n_lo=16, n_hi=n_hi, d_lo=2.0, d_hi=40.0)
    n2, s2, d2, _ = golden_io.fig2()
    extra = [(5, np.zeros(0, np.int32), np.zeros(0, np.int32)),   # no edges
             (2, np.array([1], np.int32), np.array([0], np.int32)),  # one edge
             _clique(5), _clique(33), (n2, s2, d2),
             (1, np.zeros(0, np.int32), np.zeros(0, np.int32)),
             (0, np.zeros(0, np.int32), np.zeros(0, np.int32))]
    gs = extra[:3] + gs[:count // 2] + extra[3:] + gs[count // 2:]
    # random edge orientation and order inside each graph
    out = []
    for i, (n, s, d) in enumerate(gs):
        ss, dd = graphgen.shuffle(s, d, 100 + i) if s.size else (s, d)
        out.append((n, ss, dd))
    return out


def _expected(gs):
    return np.concatenate([oracle.truss(n, s, d)[0] if s.size else np.zeros(0, np.int32) for n, s, d in gs])


def _run(T, gs, **opt):
    vo, eo, s, d = graphgen.pack(gs)
    o = T.make_options(**opt) if opt else None
    out, st = T.truss_batch(vo, eo, dev(s), dev(d), o)
    return out.cpu().numpy(), st


def test_batch_every_shape_matches_oracle():
    T = lib()
    gs = _mixed_batch(7)
    ref = _expected(gs)
    for blk, lanes in SHAPES:
        say(f"case: batch shape {blk}x{lanes}, {len(gs)} graphs")
        got, st = _run(T, gs, batch_block=blk, batch_ilp=lanes)
        np.testing.assert_array_equal(got, ref)
        assert st["m"] == ref.size and st["kmax"] == max(33, int(ref.max()))
        assert st["triangles"] == sum(oracle.support_fwd(n, s, d)[1] for n, s, d in gs if s.size)


def test_batch_errors_report_first_failing_graph():
    T = lib()
    gs = _mixed_batch(8, count=10, n_hi=200)
    bad = list(gs)
    n, s, d = bad[6]
    bad[6] = (n, np.append(s, s[0]), np.append(d, d[0]))            # duplicate edge
    n, s, d = bad[9]
    bad[9] = (n, np.append(s, 1).astype(np.int32), np.append(d, 1).astype(np.int32))  # self-loop
    n, s, d = bad[11]
    bad[11] = (n, np.append(s, n).astype(np.int32), np.append(d, 0).astype(np.int32))  # out of range
    say("case: batch errors")
    with pytest.raises(T.TrussError) as ei:
        _run(T, bad)
    assert ei.value.code == T.E_DUP
    with pytest.raises(T.TrussError) as ei:
        _run(T, [gs[0], gs[1]] + bad[9:])
    assert ei.value.code == T.E_SELFLOOP
    with pytest.raises(T.TrussError) as ei:
        _run(T, bad[11:])
    assert ei.value.code == T.E_RANGE


def test_plan_replays_match_oracle():
    torch = pytest.importorskip("torch")
    T = lib()
    gs = _mixed_batch(9, count=30)
    ref = _expected(gs)
    vo, eo, s, d = graphgen.pack(gs)
    plan = T.BatchPlan(vo, eo, dev(s), dev(d), T.make_options(batch_block=512, batch_ilp=4))
    for rep in range(4):
        say(f"case: plan replay {rep}")
        plan.out.fill_(-1)          # eager work between replays
        torch.cuda.synchronize()
        out, st = plan.run()
        np.testing.assert_array_equal(out.cpu().numpy(), ref)
        assert st["launches"] == 1
    plan.close()


def test_big_graph_takes_device_wide_path():
    T = lib()
    n, s, d = graphgen.rmat(17, 20, 5)
    assert s.size > (1 << 21)
    gs = _mixed_batch(10, count=6, n_hi=300)
    gs = gs[:4] + [(n, s, d)] + gs[4:]
    say(f"case: batch with a {s.size}-edge graph")
    ref = _expected(gs)
    got, st = _run(T, gs)
    np.testing.assert_array_equal(got, ref)
    assert st["launches"] == 2


def test_autotune_returns_a_built_shape():
    T = lib()
    gs = _mixed_batch(11, count=60, n_hi=3000)
    vo, eo, s, d = graphgen.pack(gs)
    say("case: autotune")
    blk, lanes, ms = T.truss_batch_autotune(vo, eo, dev(s), dev(d))
    assert (blk, lanes) in SHAPES and ms > 0
    got, _ = _run(T, gs, batch_block=blk, batch_ilp=lanes)
    np.testing.assert_array_equal(got, _expected(gs))


def test_batch_4096_full_size():
    """The 4096-graph batch at full size: the concatenated truss numbers'
    digest against the stored oracle record, plus per-graph k_max."""
    rec = golden_io.oracle_record("batch4096")
    if rec is None:
        pytest.skip("oracle record for the 4096-graph batch not generated")
    T = lib()
    say("case: 4096-graph batch, generating")
    gs = graphgen.batch(4096, 1)
    vo, eo, s, d = graphgen.pack(gs)
    assert int(eo[-1]) == rec["m"]
    say("case: 4096-graph batch, running")
    out, st = T.truss_batch(vo, eo, dev(s), dev(d))
    got = out.cpu().numpy()
    kmax = [int(got[eo[g]:eo[g + 1]].max(initial=0)) for g in range(4096)]
    assert kmax == rec["graph_kmax"]
    assert golden_io.int32_digest(got) == rec["truss_sha256"]
