"""CPU checks of the benchmark's host logic: the unit counts of its byte
models agree between the CSR and edge-list forms and with their definitions
on small graphs, the merge-form support count equals the sum over edges of
the smaller degree, the recorded-traffic lookup refuses a summary taken on
other sources, and --gpus N > 1 stops before touching a GPU."""
import itertools
import os
import subprocess
import sys

import numpy as np

import graphgen

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
sys.path.insert(0, ROOT)
import bench  # noqa: E402


def _brute_counts(n, s, d):
    deg = np.bincount(np.concatenate([s, d]), minlength=n)
    before = lambda a, b: (deg[a], a) < (deg[b], b)  # noqa: E731
    out = {a: set() for a in range(n)}
    for a, b in zip(s.tolist(), d.tolist()):
        if before(a, b):
            out[a].add(b)
        else:
            out[b].add(a)
    pairs = sum(len(out[b]) for a in range(n) for b in out[a])
    merge = sum(len(out[a]) + len(out[b]) for a in range(n) for b in out[a])
    mn = sum(min(deg[a], deg[b]) for a, b in zip(s, d))
    lg = sum(min(deg[a], deg[b]) * int(np.ceil(np.log2(max(deg[a], deg[b], 1)))) for a, b in zip(s, d))
    return {"support_pairs": pairs, "merge_elems": merge, "sum_min_deg": mn, "sum_min_deg_log": lg}


def test_models_match_definitions():
    rng = np.random.default_rng(4)
    for trial in range(10):
        n = int(rng.integers(5, 40))
        pairs = [(a, b) for a, b in itertools.combinations(range(n), 2) if rng.random() < 0.3]
        if not pairs:
            continue
        s, d = np.array(pairs, np.int32).T.copy()
        ref = _brute_counts(n, s, d)
        e = bench.edge_work_model(n, s, d)
        rp, col = graphgen.to_csr(n, s, d)
        c = bench.host_work_model(n, rp, col)
        for k, v in ref.items():
            assert e[k] == v and c[k] == v, (k, e[k], c[k], v)
        assert e["merge_elems"] == e["sum_min_deg"]  # each oriented a->b: min degree = d+(a) + d-(a)


def test_models_agree_on_rmat():
    n, s, d = graphgen.rmat(12, 8, 3)
    rp, col = graphgen.to_csr(n, s, d)
    c = bench.host_work_model(n, rp, col)
    e = bench.edge_work_model(n, s, d)
    for k in ("support_pairs", "oriented_edges", "merge_elems", "sum_min_deg", "sum_min_deg_log"):
        assert c[k] == e[k], k
    sup, peel = bench.method_bytes(e, s.size, 1000)
    assert sup == 4 * e["merge_elems"] + 16 * 1000 + 20 * s.size
    # one 16-byte hash-table slot per membership test (the method's E_G)
    assert peel == 28 * s.size + 8 * e["sum_min_deg"] + 16 * e["sum_min_deg"] + 8 * 1000
    _, peel_bs = bench.method_bytes(e, s.size, 1000, probe="bsearch")
    assert peel_bs == 28 * s.size + 8 * e["sum_min_deg"] + 4 * e["sum_min_deg_log"] + 8 * 1000


def test_traffic_lookup_needs_matching_sources(tmp_path, monkeypatch):
    monkeypatch.setattr(bench, "PROFILES", str(tmp_path))
    f = tmp_path / "traffic_k_peel_demo.txt"
    f.write_text("hbm_bytes_per_launch: 1.5e+09\nsource_digest: 0000000000000000\n")
    assert bench.measured_traffic("demo", "k_peel", 1) is None
    f.write_text("hbm_bytes_per_launch: 1.5e+09\nsource_digest: %s\n" % bench.source_digest("k_peel"))
    assert bench.measured_traffic("demo", "k_peel", 1) == 1500000000


def test_more_than_one_gpu_is_refused():
    r = subprocess.run([sys.executable, os.path.join(ROOT, "bench.py"), "--gpus", "2"], capture_output=True,
                       text=True, timeout=120, env=dict(os.environ, HIP_VISIBLE_DEVICES=""))
    assert r.returncode != 0
    assert "--gpus 1" in r.stderr


def test_digest_ignores_comments_only(tmp_path, monkeypatch):
    import shutil
    pkg = tmp_path / "paper_1205_6693_amd"
    shutil.copytree(os.path.join(ROOT, "paper_1205_6693_amd", "csrc"), pkg / "csrc")
    shutil.copy(os.path.join(ROOT, "paper_1205_6693_amd", "sched_model.json"), pkg / "sched_model.json")
    (tmp_path / "include").mkdir()
    shutil.copy(os.path.join(ROOT, "include", "truss.h"), tmp_path / "include" / "truss.h")
    monkeypatch.setattr(bench, "ROOT", str(tmp_path))
    base, batch = bench.source_digest("k_peel"), bench.source_digest("k_batch")
    peel = pkg / "csrc" / "peel.hip"
    text = peel.read_text()
    peel.write_text(text + "\n// a comment\n/* another\n comment */\n")
    assert bench.source_digest("k_peel") == base
    peel.write_text(text.replace("kMinChunk = 64", "kMinChunk = 32"))
    assert bench.source_digest("k_peel") != base
    assert bench.source_digest("k_batch") == batch  # the batch kernel does not depend on peel.hip


def test_device_work_model_matches_host_model():
    """The torch form of the counts (run on the GPU at full size) equals the
    numpy form; here both run on the CPU."""
    import torch
    for scale, ef, seed in ((10, 8, 1), (12, 16, 2)):
        n, s, d = graphgen.rmat(scale, ef, seed)
        rp, col = graphgen.to_csr(n, s, d)
        h = bench.host_work_model(n, rp, col)
        t = bench.device_work_model(n, torch.from_numpy(rp), torch.from_numpy(col))
        for k in ("support_pairs", "oriented_edges", "max_outdeg", "merge_elems", "sum_min_deg", "sum_min_deg_log"):
            assert h[k] == t[k], k


def test_verify_output_against_the_stored_record():
    """bench.py's check of a timed output: the oracle's own truss numbers of
    the ER workload match the stored digest, in canonical order and through a
    shuffle's ordering; a single changed value does not."""
    import oracle
    n, s, d = graphgen.er_small(1)
    phi, _ = oracle.truss(n, s, d)
    ok, secs = bench.verify_output("er2000", phi)
    assert ok is True
    bad = phi.copy()
    bad[17] += 1
    assert bench.verify_output("er2000", bad)[0] is False
    s2, d2 = graphgen.shuffle(s, d, 12345)
    phi2, _ = oracle.truss(n, s2, d2)
    lo, hi = np.minimum(s2, d2).astype(np.int64), np.maximum(s2, d2).astype(np.int64)
    assert bench.verify_output("er2000", phi2, np.lexsort((hi, lo)))[0] is True
    assert bench.verify_output("no_such_workload", phi) == (None, None)
    assert bench.verify_output("rmat24", phi)[1] == 11210
