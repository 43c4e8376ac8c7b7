#!/usr/bin/env python3
"""Benchmark: truss-decomposed edges/s on one MI355X, plain vs learned-scheduled.

A step is one truss_decompose call on the resident input graph: validation,
CSR build, support counting, peeling, output.  Inputs are generated on the host
from a seed and copied to HBM before the timed region; the timed region covers
exactly K steps bracketed by device synchronisation.  The default workload is
R-MAT scale 24 (260M edges, CSR).  The headline value is the learned-scheduled
form (the committed model); the plain and heuristic forms are timed afterwards
with fewer steps (--compare-steps) for comparison.  The output of the last
timed step is hashed and compared with the oracle's stored digest for the
workload ("verified" in the JSON line).

Prints one JSON line with the metric, the roofline of the dominant kernel
(measured with HIP events on the library's stream) and the CPU oracle timed on a
bounded sample of the same generator family.
"""
from __future__ import annotations

import argparse
import json
import os
import sys
import time

import numpy as np

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

HBM_PEAK_GBS = 8000.0
PROFILES = os.path.join(ROOT, "profiles")

WORKLOADS = {
    "rmat20": "R-MAT scale 20, edge factor 16, (a,b,c,d)=(.57,.19,.19,.05), symmetrised, deduplicated, int32 CSR",
    "er2000": "Erdos-Renyi G(n=2000, p=0.01), int32 edge list",
    "chunglu4m": "Chung-Lu n=4M, exponent 2.1, mean degree 30, cap 200k, 64 planted cliques U{50..500}, int32 CSR",
    "rmat24": "R-MAT scale 24, edge factor 16, same (a,b,c,d), int32 ids / int64 offsets CSR",
    "batch4096": "4096 graphs, n ~ U{64..8192}, mean degree ~ U[4,64], even ER / odd R-MAT (.57,.19,.19,.05), "
                 "packed int32 edge lists with int64 offsets",
}


def make_graph(name: str, seed: int):
    import graphgen
    if name == "rmat20":
        return graphgen.rmat20(seed), "csr"
    if name == "er2000":
        return graphgen.er_small(seed), "edges"
    if name == "chunglu4m":
        return graphgen.chung_lu4m(seed), "csr"
    if name == "rmat24":
        return graphgen.rmat24(seed), "csr"
    raise SystemExit("unknown workload " + name)


def host_work_model(n, row_ptr, col):
    """Unit counts of the algorithmic byte models, from the graph itself:
    oriented (b, c) pairs and edges (support as walked), sum over oriented
    edges of d+(a) + d+(b) (the merge-form reference count of support), and
    over the edges of min(deg u, deg v) and min(deg) * ceil(log2 max(deg)) (the
    walk of the smaller endpoint's full row and its binary-search probes in
    Algorithm 2)."""
    deg = np.diff(row_ptr).astype(np.int64)
    rows = np.repeat(np.arange(n, dtype=np.int64), deg)
    c = col.astype(np.int64)
    before = (deg[rows] < deg[c]) | ((deg[rows] == deg[c]) & (rows < c))
    dplus = np.bincount(rows[before], minlength=n).astype(np.int64)
    pairs = int(dplus[c[before]].sum())  # sum over a->b of d+(b)
    upper = rows < c  # every undirected edge once
    du, dv = deg[rows[upper]], deg[c[upper]]
    mn, mx = np.minimum(du, dv), np.maximum(du, dv)
    lg = np.ceil(np.log2(np.maximum(mx, 1).astype(np.float64))).astype(np.int64)
    return {"support_pairs": pairs, "oriented_edges": int(before.sum()), "max_outdeg": int(dplus.max(initial=0)),
            "merge_elems": int((dplus * dplus).sum()) + pairs, "sum_min_deg": int(mn.sum()),
            "sum_min_deg_log": int((mn * lg).sum())}


def device_work_model(n, row_ptr, col):
    """host_work_model's counts computed with torch on the GPU (the same
    formulas; R-MAT 24's 520M row entries take seconds there, minutes in
    numpy).  row_ptr, col: the CSR tensors on the device."""
    import torch
    deg = row_ptr[1:] - row_ptr[:-1]
    rows = torch.repeat_interleave(torch.arange(n, device=col.device, dtype=torch.int64), deg)
    c = col.to(torch.int64)
    dr, dc = deg[rows], deg[c]
    before = (dr < dc) | ((dr == dc) & (rows < c))
    dplus = torch.bincount(rows[before], minlength=n).to(torch.int64)
    pairs = int(dplus[c[before]].sum().item())
    oriented = int(before.sum().item())
    del before
    upper = rows < c
    du, dv = dr[upper], dc[upper]
    del rows, c, dr, dc, upper
    mn, mx = torch.minimum(du, dv), torch.maximum(du, dv)
    del du, dv
    lg = torch.ceil(torch.log2(mx.clamp(min=1).to(torch.float64))).to(torch.int64)
    out = {"support_pairs": pairs, "oriented_edges": oriented, "max_outdeg": int(dplus.max().item()) if n else 0,
           "merge_elems": int((dplus * dplus).sum().item()) + pairs, "sum_min_deg": int(mn.sum().item()),
           "sum_min_deg_log": int((mn * lg).sum().item())}
    del mn, mx, lg
    if col.is_cuda:
        torch.cuda.empty_cache()
    return out


def verify_output(workload, out_host, order=None):
    """Compares the truss numbers of a timed step with the oracle's stored
    record for the workload (tests/golden/oracle_<workload>.txt: SHA-256 of the
    int32 truss numbers in canonical edge order, written from the oracle
    alone).  order: index array that puts out_host into canonical order (None:
    already canonical).  Truss numbers are unique (Definition 2), so the
    comparison is exact.  Returns (verified or None when no record exists,
    the record's oracle seconds or None)."""
    import hashlib
    import re
    path = os.path.join(ROOT, "tests", "golden", "oracle_%s.txt" % workload)
    if not os.path.exists(path):
        return None, None
    want, secs = None, None
    for line in open(path):
        if line.startswith("truss_sha256:"):
            want = line.split(":", 1)[1].strip()
        mt = re.search(r"\((\d+) s on one core\)", line)
        if mt and secs is None:
            secs = int(mt.group(1))
    if want is None:
        return None, secs
    a = out_host if order is None else out_host[order]
    got = hashlib.sha256(np.ascontiguousarray(a, dtype=np.int32).tobytes()).hexdigest()
    return got == want, secs


def edge_work_model(n, s, d):
    """host_work_model's counts from an edge list (each undirected edge once)."""
    s = s.astype(np.int64)
    d = d.astype(np.int64)
    deg = np.bincount(np.concatenate([s, d]), minlength=n).astype(np.int64)
    fwd = (deg[s] < deg[d]) | ((deg[s] == deg[d]) & (s < d))
    a = np.where(fwd, s, d)
    b = np.where(fwd, d, s)
    dplus = np.bincount(a, minlength=n).astype(np.int64)
    mn = np.minimum(deg[s], deg[d])
    mx = np.maximum(deg[s], deg[d])
    lg = np.ceil(np.log2(np.maximum(mx, 1).astype(np.float64))).astype(np.int64)
    return {"support_pairs": int(dplus[b].sum()), "oriented_edges": int(s.size),
            "merge_elems": int((dplus[a] + dplus[b]).sum()), "sum_min_deg": int(mn.sum()),
            "sum_min_deg_log": int((mn * lg).sum())}


def method_bytes(model, m, triangles, probe="hash"):
    """Algorithmic bytes of support and peeling for the method (see main).
    The membership test of each walked entry is priced as the method keeps
    E_G: one 16-byte hash-table slot (Section 3.2), or, with probe="bsearch",
    4 bytes per step of a binary search of the longer row."""
    sup = 4 * model["merge_elems"] + 16 * triangles + 20 * m
    probes = 16 * model["sum_min_deg"] if probe == "hash" else 4 * model["sum_min_deg_log"]
    peel = 16 * m + 8 * model["sum_min_deg"] + probes + 8 * triangles + 4 * m + 8 * m
    return sup, peel


# sources that decide what a profiled kernel does on the benchmark's input: its
# own translation unit and headers, and what builds its input and drives it
_DIGEST_FILES = {
    "k_peel": ["csrc/peel.hip", "csrc/common.hpp", "csrc/internal.hpp", "csrc/mlp.hpp", "csrc/build.hip",
               "csrc/scan.hip", "csrc/support.hip", "csrc/api.hip", "sched_model.json"],
    "k_sup": ["csrc/support.hip", "csrc/common.hpp", "csrc/internal.hpp", "csrc/mlp.hpp", "csrc/build.hip",
              "csrc/scan.hip", "csrc/api.hip", "sched_model.json"],
    "k_batch": ["csrc/batch.hip", "csrc/common.hpp", "csrc/internal.hpp", "csrc/api.hip"],
}


def source_digest(kernel="k_peel"):
    """Digest of the code behind `kernel` (and the C ABI header), comments
    left out; recorded traffic is valid only for the same code."""
    import hashlib
    import re
    h = hashlib.sha256()
    pkg = os.path.join(ROOT, "paper_1205_6693_amd")
    for f in sorted(_DIGEST_FILES[kernel]) + ["../include/truss.h"]:
        with open(os.path.join(pkg, f), "rb") as fh:
            text = fh.read()
        if not f.endswith(".json"):
            text = re.sub(rb"/\*.*?\*/", b"", text, flags=re.S)
            text = re.sub(rb"//[^\n]*", b"", text)
            text = b"\n".join(line.rstrip() for line in text.splitlines() if line.strip())
        h.update(f.encode() + text)
    return h.hexdigest()[:16]


def measured_traffic(workload, kernel, launches):
    """HBM bytes per launch of `kernel` from the committed rocprofv3 counter
    summary (FETCH_SIZE + WRITE_SIZE scaled by the copy-kernel calibration), or
    None if there is none for these sources."""
    path = os.path.join(PROFILES, "traffic_%s_%s.txt" % (kernel, workload))
    if not os.path.exists(path):
        return None
    kv = {}
    for line in open(path):
        if ":" in line:
            a, b = line.split(":", 1)
            kv[a.strip()] = b.strip()
    if kv.get("source_digest") != source_digest(kernel):
        return None
    try:
        return int(float(kv["hbm_bytes_per_launch"]))
    except (KeyError, ValueError):
        return None


def traffic_fields(traffic, launch_ms):
    """Counter-measured bytes per launch, and the bandwidth they give over the
    launch time, when a record exists."""
    if not traffic:
        return {"traffic": None}
    gbs = traffic / (launch_ms * 1e-3) / 1e9
    return {"traffic": traffic, "traffic_GB/s": round(gbs, 2), "traffic_frac": round(gbs / HBM_PEAK_GBS, 5)}


def calibrate_copy(nbytes):
    """A plain device copy of known size, for scaling the PMC byte counters."""
    import torch
    a = torch.ones(nbytes // 4, dtype=torch.int32, device="cuda:0")
    b = torch.empty_like(a)
    for _ in range(5):
        torch.add(a, 0, out=b)
    torch.cuda.synchronize()
    print(json.dumps({"calibration_copy_bytes_read": a.numel() * 4, "bytes_written": b.numel() * 4,
                      "dispatches": 5}))


def _short(name):
    name = name.replace("(anonymous namespace)::", "").replace("void ", "").replace("truss::", "")
    return name.split("(")[0] if "(" in name else name


def summarize_db(path):
    """Kernel durations (and PMC counters, when the run collected them) from a
    rocprofv3 SQLite output file."""
    import sqlite3
    out = []
    c = sqlite3.connect(path)
    rows = c.execute("select name, count(*), sum(duration), avg(duration) from kernels group by name "
                     "order by sum(duration) desc").fetchall()
    out.append("kernel stats: " + os.path.basename(path))
    for name, calls, tot, avg in rows:
        out.append("  %-60s calls=%d total_ns=%d avg_ns=%.0f" % (_short(name)[:60], calls, tot, avg))
    try:
        cnt = c.execute("select kernel_name, counter_name, count(distinct dispatch_id), sum(value) "
                        "from counters_collection group by kernel_name, counter_name").fetchall()
    except sqlite3.Error:
        cnt = []
    if cnt:
        out.append("counters: " + os.path.basename(path))
        for name, cname, disp, val in cnt:
            out.append("  %-50s %-12s dispatches=%d total=%.6g per_dispatch=%.6g"
                       % (_short(name)[-50:], cname, disp, val, val / max(1, disp)))
    return out


def summarize(prof_dir):
    """Text summary of rocprofv3 output (kernel stats and counters), CSV or
    SQLite."""
    import csv
    import glob
    out = []
    for f in sorted(glob.glob(os.path.join(prof_dir, "**", "*.db"), recursive=True)):
        out.extend(summarize_db(f))
    for f in sorted(glob.glob(os.path.join(prof_dir, "**", "*kernel_stats.csv"), recursive=True)):
        out.append("kernel stats: " + os.path.relpath(f, prof_dir))
        for r in csv.DictReader(open(f)):
            name = r.get("Name", r.get("KERNEL_NAME", "?")).replace("(anonymous namespace)::", "").replace("void ", "")
            out.append("  %-60s calls=%s total_ns=%s avg_ns=%s" % (name[:60], r.get("Calls"), r.get("TotalDurationNs"),
                                                                  r.get("AverageNs")))
    for f in sorted(glob.glob(os.path.join(prof_dir, "**", "*counter_collection.csv"), recursive=True)):
        agg = {}
        for r in csv.DictReader(open(f)):
            name = r["Kernel_Name"].replace("(anonymous namespace)::", "").replace("void ", "").split("(")[0]
            key = (name, r["Counter_Name"])
            a = agg.setdefault(key, [0.0, set()])
            a[0] += float(r["Counter_Value"])
            a[1].add(r["Dispatch_Id"])
        out.append("counters: " + os.path.relpath(f, prof_dir))
        for (name, cname), (val, disp) in sorted(agg.items()):
            out.append("  %-50s %-12s dispatches=%d total=%.6g per_dispatch=%.6g" % (name[-50:], cname, len(disp), val,
                                                                                  val / max(1, len(disp))))
    print("\n".join(out))


def host_info():
    """The host the oracle was timed on: CPU model and logical CPUs."""
    model = "unknown"
    try:
        with open("/proc/cpuinfo") as f:
            for line in f:
                if line.startswith("model name"):
                    model = line.split(":", 1)[1].strip()
                    break
    except OSError:
        pass
    return {"cpu": model, "logical_cpus": os.cpu_count()}


def cpu_baseline(sample_scale: int, seed: int):
    import graphgen
    import oracle
    n, s, d = graphgen.rmat(sample_scale, 16, seed)
    oracle.build()
    times = []
    for _ in range(3):
        t0 = time.perf_counter()
        oracle.truss(n, s, d)
        times.append(time.perf_counter() - t0)
    t = float(np.median(times))
    return {"value": s.size / t, "unit": "edges/s", "cores": 1, "kind": "oracle",
            "sample": "serial C oracle (support + Algorithm 2 bin-sort peeling), one thread, on R-MAT scale %d "
                      "edge factor 16 (same generator, m=%d): median of 3 runs, %.1f s each; full-size oracle "
                      "runs take minutes" % (sample_scale, s.size, t), "host": host_info()}


def bench_batch(args):
    """The batch workload: one persistent batch kernel in a replayed HIP graph
    (shape from the autotuner) against one truss_decompose call per graph."""
    import torch
    import graphgen
    import paper_1205_6693_amd as T
    T.load_library()
    torch.cuda.set_device(0)
    print("generating batch4096 seed %d" % args.seed, file=sys.stderr, flush=True)
    gs = graphgen.batch(4096, args.seed)
    vo, eo, s, d = graphgen.pack(gs)
    m = int(eo[-1])
    S, D = torch.from_numpy(s).cuda(), torch.from_numpy(d).cuda()
    del gs
    t = time.perf_counter()
    if args.batch_shape:
        blk, lanes = args.batch_shape
        tune_ms = None
    else:
        blk, lanes, tune_ms = T.truss_batch_autotune(vo, eo, S, D)
        print("autotune: %d threads x %d entries in flight (%.1f ms on the batch; tuning took %.1f s)"
              % (blk, lanes, tune_ms, time.perf_counter() - t), file=sys.stderr, flush=True)
    plan = T.BatchPlan(vo, eo, S, D, T.make_options(batch_block=blk, batch_ilp=lanes))
    for i in range(args.warmup):
        _, st = plan.run()
        print("warmup %d: %.2f ms" % (i, st["ms_total"]), file=sys.stderr, flush=True)
    stats = []
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    for i in range(args.steps):
        _, st = plan.run()
        stats.append(st)
        print("step %d: %.2f ms" % (i, st["ms_total"]), file=sys.stderr, flush=True)
    torch.cuda.synchronize()
    ms_per_step = (time.perf_counter() - t0) * 1e3 / args.steps
    st = stats[-1]
    kms = float(np.mean([x["ms_peel_kernel"] for x in stats]))
    # algorithmic bytes of the batch kernel: the method's support and peeling
    # bytes of every graph (the per-unit figures of the single-graph bench)
    # plus 56 B per edge for the per-graph build (input, canonical pair, CSR
    # build and sort, output); beside them the bytes as walked here: 56 B per
    # edge, 8 B per support walk entry, 16 B per peeling walk entry
    alg = 56 * m
    for g in range(4096):
        ng = int(vo[g + 1] - vo[g])
        sg, dg = s[eo[g]:eo[g + 1]], d[eo[g]:eo[g + 1]]
        if sg.size:
            mdl = edge_work_model(ng, sg, dg)
            alg += sum(method_bytes(mdl, int(sg.size), 0))
    alg += 24 * st["triangles"]  # the triangle terms of both stages (16 + 8 B per triangle)
    walked = 56 * m + 8 * st["support_work"] + 16 * st["peel_work"]
    achieved = alg / (kms * 1e-3) / 1e9
    per_graph = None
    if not args.no_compare:
        o = T.make_options()
        out = torch.empty(m, dtype=torch.int32, device="cuda:0")
        graphs = [T.Graph.from_edges(int(vo[g + 1] - vo[g]), S[eo[g]:eo[g + 1]], D[eo[g]:eo[g + 1]])
                  for g in range(4096)]
        ws = torch.empty(max(T.truss_workspace_size(g, o) for g in graphs), dtype=torch.uint8, device="cuda:0")
        for g in range(8):
            T.truss_decompose(graphs[g], o, out=out[eo[g]:eo[g + 1]], ws=ws)
        torch.cuda.synchronize()
        t1 = time.perf_counter()
        for g in range(4096):
            T.truss_decompose(graphs[g], o, out=out[eo[g]:eo[g + 1]], ws=ws)
            if g % 512 == 511:
                print("per-graph launches: %d graphs done" % (g + 1), file=sys.stderr, flush=True)
        torch.cuda.synchronize()
        pg = time.perf_counter() - t1
        per_graph = {"edges_per_s": m / pg, "ms_per_batch": pg * 1e3, "calls": 4096}
        same = bool(torch.equal(out, plan.out))
        per_graph["same_output"] = same
    result = {
        "metric": "truss-decomposed edges/s + HBM GB/s, plain vs learned-scheduled, 1 MI355X",
        "value": m / (ms_per_step * 1e-3), "unit": "edges/s", "n_gpus": 1, "steps": args.steps,
        "warmup": args.warmup, "ms_per_step": ms_per_step, "higher_is_better": True, "scaling": "weak",
        "vs_baseline": None, "dtype": "int32", "data": "synthetic",
        "config": {"workload": "batch4096", "description": WORKLOADS["batch4096"], "seed": args.seed,
                   "graphs": 4096, "m": m, "batch_block": blk, "batch_ilp": lanes},
        "kmax": st["kmax"], "levels": st["levels"], "subrounds": st["subrounds"], "triangles": st["triangles"],
        "support_work": st["support_work"], "peel_work": st["peel_work"], "batch_kernel_ms": kms,
        "autotune_ms": tune_ms,
        "roofline": {"bound": "hbm", "achieved": round(achieved, 2), "peak": HBM_PEAK_GBS, "unit": "GB/s",
                     "frac": round(achieved / HBM_PEAK_GBS, 5),
                     "traffic": measured_traffic("batch4096", "k_batch", 1), "kernel": "k_batch",
                     "launches_per_step": 1, "avg_launch_ms": round(kms, 4), "bytes_per_launch": int(alg),
                     "achieved_walked": round(walked / (kms * 1e-3) / 1e9, 2),
                     "frac_walked": round(walked / (kms * 1e-3) / 1e9 / HBM_PEAK_GBS, 5),
                     "walked_bytes_per_launch": int(walked)},
        "per_graph_launches": per_graph,
    }
    if per_graph:
        result["batched_over_per_graph"] = result["value"] / per_graph["edges_per_s"]
    if not args.no_cpu_baseline:
        print("timing the CPU oracle on a sample", file=sys.stderr, flush=True)
        result["cpu_baseline"] = cpu_baseline_batch(args.seed)
    print(json.dumps(result), flush=True)


def cpu_baseline_batch(seed: int):
    """The oracle on the first 256 graphs of the batch spec list (serial)."""
    import graphgen
    import oracle
    oracle.build()
    specs = graphgen.batch_specs(4096, seed)[:256]
    tot, m = 0.0, 0
    for sp in specs:
        n, s, d = graphgen.batch_graph(sp)
        t0 = time.perf_counter()
        oracle.truss(n, s, d)
        tot += time.perf_counter() - t0
        m += s.size
    return {"value": m / tot, "unit": "edges/s", "cores": 1, "kind": "oracle",
            "sample": "serial C oracle, one thread, on the first 256 graphs of the batch (m=%d) in %.1f s"
                      % (m, tot), "host": host_info()}


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=10)
    ap.add_argument("--warmup", type=int, default=2)
    ap.add_argument("--workload", default="rmat24", choices=sorted(WORKLOADS))
    ap.add_argument("--compare-steps", type=int, default=3,
                    help="timed steps of each comparison form (after one warm-up step)")
    ap.add_argument("--seed", type=int, default=1)
    ap.add_argument("--scheduler", default="learned", choices=["plain", "heuristic", "learned"])
    ap.add_argument("--no-compare", action="store_true", help="skip timing the other scheduler forms")
    ap.add_argument("--topdown", type=int, default=0, metavar="T",
                    help="also time the top-T k-classes (upper bound + top-down) against the full decomposition")
    ap.add_argument("--bottomup", type=float, default=0.0, metavar="FRACTION",
                    help="also run the bottom-up decomposition from host memory with a device budget of "
                         "FRACTION * m edges per subgraph")
    ap.add_argument("--cohen", action="store_true",
                    help="also time Algorithm 1 (the comparator of Table 3) on the workload")
    ap.add_argument("--cohen-sweep", action="store_true",
                    help="Table 3's shape: Algorithm 1 against the learned Algorithm 2 path on Chung-Lu graphs "
                         "of growing maximum degree")
    ap.add_argument("--cohesion", action="store_true",
                    help="also time the core numbers and the cohesion statistics of Table 6")
    ap.add_argument("--batch-shape", type=int, nargs=2, default=None, metavar=("THREADS", "ILP"),
                    help="batch4096: use this shape instead of the autotuner's")
    ap.add_argument("--probe", default="auto", choices=["auto", "hash", "bsearch"])
    ap.add_argument("--peel-mode", default="auto", choices=["auto", "sparse", "dense"])
    ap.add_argument("--support", default="auto", choices=["auto", "hash", "bsearch", "merge"])
    ap.add_argument("--cpu-sample-scale", type=int, default=17)
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--calibrate-copy", type=int, default=0, help="run a plain copy of this many bytes and exit")
    ap.add_argument("--summarize", default="", help="summarise a rocprofv3 output directory and exit")
    args = ap.parse_args()
    if args.summarize:
        summarize(args.summarize)
        return
    if args.calibrate_copy:
        calibrate_copy(args.calibrate_copy)
        return
    if args.gpus != 1:
        print("bench.py measures one GPU only: the library has no multi-GPU path "
              "(run with --gpus 1)", file=sys.stderr)
        sys.exit(2)

    if args.workload == "batch4096":
        bench_batch(args)
        return
    import torch
    import paper_1205_6693_amd as T
    T.load_library()
    torch.cuda.set_device(0)

    print("generating %s seed %d" % (args.workload, args.seed), file=sys.stderr, flush=True)
    (n, s, d), fmt = make_graph(args.workload, args.seed)
    import graphgen
    m = s.size
    model = None
    canon_order = None  # puts the output into canonical edge order
    if fmt == "csr":
        row_ptr, col = graphgen.to_csr(n, s, d)
        g = T.Graph.from_csr(n, torch.from_numpy(row_ptr).cuda(), torch.from_numpy(col).cuda())
        del row_ptr, col
        model = device_work_model(n, g.row_ptr, g.col)
        host_edges = (s, d)  # canonical order = the CSR output order
    else:
        s2, d2 = graphgen.shuffle(s, d, 12345)
        g = T.Graph.from_edges(n, torch.from_numpy(s2).cuda(), torch.from_numpy(d2).cuda())
        host_edges = (s2, d2)
        lo, hi = np.minimum(s2, d2).astype(np.int64), np.maximum(s2, d2).astype(np.int64)
        canon_order = np.lexsort((hi, lo))
        row_ptr, col = graphgen.to_csr(n, s, d)
        model = host_work_model(n, row_ptr, col)
    sched_ids = {"plain": T.SCHED_PLAIN, "heuristic": T.SCHED_HEURISTIC, "learned": T.SCHED_LEARNED}
    from paper_1205_6693_amd import sched as S
    sched_model = S.load_model() if os.path.exists(S.MODEL_PATH) else None

    def form_options(name):
        if name == "learned" and sched_model is None:
            raise SystemExit("learned scheduler requested but %s is missing" % S.MODEL_PATH)
        return T.make_options(scheduler=sched_ids[name], model=sched_model if name == "learned" else None,
                              peel_probe={"auto": 0, "hash": 1, "bsearch": 2}[args.probe],
                              peel_mode={"auto": 0, "sparse": 1, "dense": 2}[args.peel_mode],
                              support_strategy={"auto": 0, "hash": 1, "bsearch": 2, "merge": 3}[args.support])

    opts = form_options(args.scheduler)
    ws = T.workspace(g, opts)
    out = torch.empty(m, dtype=torch.int32, device="cuda:0")
    torch.cuda.synchronize()
    print("n=%d m=%d workspace=%.2f GB" % (n, m, ws.numel() / 1e9), file=sys.stderr, flush=True)

    for i in range(args.warmup):
        _, st = T.truss_decompose(g, opts, out=out, ws=ws)
        print("warmup %d: %.2f ms (build %.2f support %.2f peel %.2f) kmax %d subrounds %d fallback %d"
              % (i, st["ms_total"], st["ms_build"], st["ms_support"], st["ms_peel"], st["kmax"],
                 st["subrounds"], st["sched_fallback"]), file=sys.stderr, flush=True)
        if args.scheduler == "learned" and st["sched_fallback"]:
            raise SystemExit("the learned model was rejected by the library")
    stats = []
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    for i in range(args.steps):
        _, st = T.truss_decompose(g, opts, out=out, ws=ws)
        stats.append(st)
        print("step %d: %.2f ms" % (i, st["ms_total"]), file=sys.stderr, flush=True)
    torch.cuda.synchronize()
    wall = time.perf_counter() - t0
    ms_per_step = wall * 1e3 / args.steps
    print("timed %d steps: %.3f ms/step" % (args.steps, ms_per_step), file=sys.stderr, flush=True)
    verified, oracle_secs = verify_output(args.workload, out.cpu().numpy(), canon_order)
    print("output of the last timed step equals the oracle record: %s" % verified, file=sys.stderr, flush=True)

    def avg(key):
        return float(np.mean([x[key] for x in stats]))

    ms_sup, ms_peel, ms_build = avg("ms_support"), avg("ms_peel"), avg("ms_build")
    ms_peel_kernel = avg("ms_peel_kernel")
    st = stats[-1]
    launches = max(1, st["launches"])
    # algorithmic bytes: the per-unit figures of the byte model for the method
    # (support, merge form: 4 B per list element compared, 16 B per triangle,
    # 20 B per edge; peeling: per edge 16 B + 8 B per entry of the smaller
    # endpoint's row + one 16 B hash-table slot per membership test, 8 B per
    # triangle, 4 B truss and 8 B of frontier per edge), and beside them the
    # bytes of what the kernels walk here (after row compaction)
    T3 = st["triangles"]
    sup_bytes, peel_bytes = method_bytes(model, m, T3)
    _, peel_bytes_bs = method_bytes(model, m, T3, probe="bsearch")
    sup_walked = 4 * model["support_pairs"] + 24 * model["oriented_edges"] + 8 * T3
    peel_walked = 16 * st["peel_work"] + 44 * m
    kernels = {
        "support": {"bytes": sup_bytes, "walked": sup_walked, "ms": ms_sup, "launches": 1,
                    "name": "k_sup"},
        "peel": {"bytes": peel_bytes, "walked": peel_walked, "ms": ms_peel_kernel, "launches": launches,
                 "name": "k_peel"},
    }
    dom = max(kernels, key=lambda k: kernels[k]["ms"])
    kd = kernels[dom]
    achieved = kd["bytes"] / (kd["ms"] * 1e-3) / 1e9
    walked = kd["walked"] / (kd["ms"] * 1e-3) / 1e9
    traffic = measured_traffic(args.workload, kd["name"], kd["launches"])
    roofline = {"bound": "hbm", "achieved": round(achieved, 2), "peak": HBM_PEAK_GBS, "unit": "GB/s",
                "frac": round(achieved / HBM_PEAK_GBS, 5), "traffic": traffic, "kernel": kd["name"],
                "traffic_GBs": round(traffic / (kd["ms"] / kd["launches"] * 1e-3) / 1e9, 2) if traffic else None,
                "traffic_frac": round(traffic / (kd["ms"] / kd["launches"] * 1e-3) / 1e9 / HBM_PEAK_GBS, 5)
                if traffic else None,
                "launches_per_step": kd["launches"], "avg_launch_ms": round(kd["ms"] / kd["launches"], 4),
                "bytes_per_launch": int(kd["bytes"] / kd["launches"]),
                "achieved_walked": round(walked, 2), "frac_walked": round(walked / HBM_PEAK_GBS, 5),
                "walked_bytes_per_launch": int(kd["walked"] / kd["launches"])}
    result = {
        "metric": "truss-decomposed edges/s + HBM GB/s, plain vs learned-scheduled, 1 MI355X",
        "value": m / (ms_per_step * 1e-3), "unit": "edges/s",
        "n_gpus": 1, "steps": args.steps, "warmup": args.warmup, "ms_per_step": ms_per_step,
        "higher_is_better": True, "scaling": "weak", "vs_baseline": None, "dtype": "int32",
        "data": "synthetic",
        "config": {"workload": args.workload, "description": WORKLOADS[args.workload], "seed": args.seed,
                   "n": n, "m": m, "scheduler": args.scheduler, "probe": args.probe,
                   "peel_mode": args.peel_mode, "support": args.support},
        "verified": verified,
        "phases_ms": {"build": ms_build, "support": ms_sup, "peel": ms_peel},
        "kmax": st["kmax"], "levels": st["levels"], "subrounds": st["subrounds"],
        "triangles": st["triangles"], "peel_work": st["peel_work"], "launches": st["launches"],
        "heavy_rounds": st["heavy_rounds"], "frontier_hist": st["frontier_hist"],
        "peel_phase_ms": dict(zip(["sweep", "start", "rounds", "pieces", "dense"], st["ms_phase"][:5])),
        "roofline": roofline,
        "roofline_all": {k: dict({"GB/s": round(v["bytes"] / (v["ms"] * 1e-3) / 1e9, 2), "ms": round(v["ms"], 3),
                                  "frac": round(v["bytes"] / (v["ms"] * 1e-3) / 1e9 / HBM_PEAK_GBS, 5),
                                  "bytes": v["bytes"],
                                  "walked_GB/s": round(v["walked"] / (v["ms"] * 1e-3) / 1e9, 2),
                                  "walked_bytes": v["walked"]},
                                 **traffic_fields(measured_traffic(args.workload, v["name"], v["launches"]),
                                                  v["ms"] / v["launches"]))
                         for k, v in kernels.items()},
        "peel_kernel_ms": ms_peel_kernel,
        "peel_bytes_bsearch_probes": peel_bytes_bs,
    }
    forms = {args.scheduler: {"edges_per_s": result["value"], "ms_per_step": ms_per_step, "steps": args.steps,
                              "warmup": args.warmup, "verified": verified}}
    if not args.no_compare:
        for name in ("plain", "heuristic", "learned"):
            if name in forms:
                continue
            o = form_options(name)
            T.truss_decompose(g, o, out=out, ws=ws)
            torch.cuda.synchronize()
            t1 = time.perf_counter()
            for _ in range(args.compare_steps):
                T.truss_decompose(g, o, out=out, ws=ws)
            torch.cuda.synchronize()
            ms = (time.perf_counter() - t1) * 1e3 / args.compare_steps
            ok, _ = verify_output(args.workload, out.cpu().numpy(), canon_order)
            forms[name] = {"edges_per_s": m / (ms * 1e-3), "ms_per_step": ms, "steps": args.compare_steps,
                           "warmup": 1, "verified": ok}
            print("form %s: %.3f ms/step (output equals the oracle record: %s)" % (name, ms, ok),
                  file=sys.stderr, flush=True)
    result["forms"] = forms
    if "plain" in forms and "learned" in forms:
        result["learned_over_plain"] = forms["learned"]["edges_per_s"] / forms["plain"]["edges_per_s"]
    if args.topdown > 0:
        tws = None
        for _ in range(args.warmup):
            top, kmin, kmax, tst = T.truss_topdown(g, args.topdown, opts, ws=tws)
        torch.cuda.synchronize()
        t1 = time.perf_counter()
        for _ in range(args.steps):
            top, kmin, kmax, tst = T.truss_topdown(g, args.topdown, opts, ws=tws)
        torch.cuda.synchronize()
        td_ms = (time.perf_counter() - t1) * 1e3 / args.steps
        t1 = time.perf_counter()
        T.truss_upper_bound(g, ws=ws)
        torch.cuda.synchronize()
        ub_ms = (time.perf_counter() - t1) * 1e3
        result["topdown"] = {"t": args.topdown, "ms_per_call": td_ms, "kmin": kmin, "kmax": kmax,
                             "subgraph_m": tst["m"], "decompositions": tst["launches"],
                             "edges_in_top_classes": int((top > 0).sum().item()),
                             "full_over_topdown": ms_per_step / td_ms, "upper_bound_ms": ub_ms}
        print("top-%d classes: %.2f ms (k %d..%d, last subgraph %d edges, %d decompositions)"
              % (args.topdown, td_ms, kmin, kmax, tst["m"], tst["launches"]), file=sys.stderr, flush=True)
    if args.cohesion:
        result["cohesion"] = time_cohesion(T, torch, g, opts, args)
    if args.bottomup > 0:
        result["bottomup"] = time_bottomup(T, n, host_edges[0], host_edges[1], opts, out, args)
    if args.cohen:
        result["cohen"] = time_cohen(T, torch, g, out, ms_per_step, args)
    if args.cohen_sweep:
        result["cohen_sweep"] = cohen_sweep(T, torch, opts)
    if not args.no_cpu_baseline:
        print("timing the CPU oracle on a sample", file=sys.stderr, flush=True)
        result["cpu_baseline"] = cpu_baseline(args.cpu_sample_scale, args.seed)
        if oracle_secs:
            result["cpu_baseline"]["recorded_full_size"] = {
                "workload": args.workload, "seconds": oracle_secs, "edges_per_s": m / oracle_secs, "cores": 1,
                "note": "the oracle on the whole workload graph (support + Algorithm 2), timed once when its "
                        "stored digests were written, on the build host's CPU, not this one"}
    print(json.dumps(result), flush=True)


def time_bottomup(T, n, s, d, opts, out, args):
    """One bottom-up run (Section 5) from host memory with a budget of
    FRACTION * m edges per device subgraph; checked against the in-memory
    decomposition just timed (same canonical edge order)."""
    cap = max(1, int(args.bottomup * s.size))
    phi, lb, st = T.truss_bottomup(n, s, d, cap, opts=opts)
    same = bool((phi == out.cpu().numpy()).all())
    print("bottom-up, budget %d edges: %.1f ms (lower bounding %.1f, bottom-up %.1f), %d passes, %d subgraphs, "
          "%d candidates, %d by procedure 9 (%d scans), %d device calls, %.2f GB to the device; "
          "equal to the in-memory result: %s"
          % (cap, st["ms_total"], st["ms_lower"], st["ms_bottomup"], st["passes"], st["subgraphs"],
             st["candidates"], st["proc9_calls"], st["proc9_scans"], st["device_calls"], st["bytes_h2d"] / 1e9,
             same), file=sys.stderr, flush=True)
    return dict(st, budget_edges=cap, equal_to_in_memory=same)


def time_cohen(T, torch, g, out, ms_alg2, args):
    """Algorithm 1 on the workload graph, checked against the output just timed."""
    reps = max(1, min(args.steps, 3))
    res, st = T.truss_cohen(g)
    same = bool(torch.equal(res, out))
    torch.cuda.synchronize()
    t1 = time.perf_counter()
    for _ in range(reps):
        res, st = T.truss_cohen(g)
    torch.cuda.synchronize()
    ms = (time.perf_counter() - t1) * 1e3 / reps
    print("algorithm 1: %.1f ms (support %.1f, peel %.1f), %.3g row entries merged; algorithm 2 path %.1f ms "
          "(%.1fx); equal: %s" % (ms, st["ms_support"], st["ms_peel"], st["support_work"] + st["peel_work"],
                                  ms_alg2, ms / ms_alg2, same), file=sys.stderr, flush=True)
    return {"ms_per_call": ms, "ms_support": st["ms_support"], "ms_peel": st["ms_peel"],
            "entries_merged": st["support_work"] + st["peel_work"], "alg2_ms": ms_alg2,
            "alg1_over_alg2": ms / ms_alg2, "equal": same}


def cohen_sweep(T, torch, opts):
    """Chung-Lu graphs, n = 2^18, mean degree 30, weight cap 10^5, no cliques,
    seed 7, with the power-law exponent falling from 3.5 to 2.1 (so the degree
    skew and the largest degree grow, at about 3.3-3.9 M edges): the time of
    Algorithm 1 over that of the Algorithm 2 path (Table 3 reports 2.2x to
    73.2x on four real graphs, growing with the largest degree)."""
    import graphgen
    rows = []
    for gamma in (3.5, 3.0, 2.6, 2.3, 2.1):
        n, s, d = graphgen.chung_lu(1 << 18, gamma, 30.0, 100000.0, 0, 0, 0, 7)
        row_ptr, col = graphgen.to_csr(n, s, d)
        g = T.Graph.from_csr(n, torch.from_numpy(row_ptr).cuda(), torch.from_numpy(col).cuda())
        deg = np.diff(row_ptr)
        times = {}
        for name, fn in (("alg2", lambda: T.truss_decompose(g, opts)), ("alg1", lambda: T.truss_cohen(g))):
            fn()
            torch.cuda.synchronize()
            t1 = time.perf_counter()
            for _ in range(3):
                o, st = fn()
            torch.cuda.synchronize()
            times[name] = (time.perf_counter() - t1) * 1e3 / 3
            times[name + "_out"] = o
        same = bool(torch.equal(times.pop("alg1_out"), times.pop("alg2_out")))
        row = {"exponent": gamma, "m": int(s.size), "d_max": int(deg.max()),
               "sum_deg2_over_m": float((deg.astype(np.float64) ** 2).sum() / max(1, s.size)),
               "alg1_ms": times["alg1"], "alg2_ms": times["alg2"], "speedup": times["alg1"] / times["alg2"],
               "equal": same}
        print("sweep: d_max %d, sum deg^2/m %.0f: algorithm 1 %.1f ms, algorithm 2 path %.1f ms, %.1fx, equal %s"
              % (row["d_max"], row["sum_deg2_over_m"], row["alg1_ms"], row["alg2_ms"], row["speedup"], same),
              file=sys.stderr, flush=True)
        rows.append(row)
    return rows


def time_cohesion(T, torch, g, opts, args):
    """Core numbers and Table 6's statistics (both include their own build;
    the statistics include a full decomposition, the core numbers and the
    support of the two subgraphs)."""
    reps = max(1, min(args.steps, 3))
    core, cmax = T.truss_core_numbers(g)
    torch.cuda.synchronize()
    t1 = time.perf_counter()
    for _ in range(reps):
        core, cmax = T.truss_core_numbers(g)
    torch.cuda.synchronize()
    core_ms = (time.perf_counter() - t1) * 1e3 / reps
    st = T.truss_cohesion(g, opts)
    torch.cuda.synchronize()
    t1 = time.perf_counter()
    for _ in range(reps):
        st = T.truss_cohesion(g, opts)
    torch.cuda.synchronize()
    coh_ms = (time.perf_counter() - t1) * 1e3 / reps
    print("core numbers %.2f ms (c_max %d); cohesion statistics %.2f ms: %s" % (core_ms, cmax, coh_ms, st),
          file=sys.stderr, flush=True)
    return dict(st, core_ms=core_ms, cohesion_ms=coh_ms)


if __name__ == "__main__":
    main()
