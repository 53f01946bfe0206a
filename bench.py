#!/usr/bin/env python3
"""Benchmark of the alignment hot path on one MI355X: GCUPS, checked against stored oracle results.

  python bench.py [--steps K] [--warmup W] [--workload NAME] [--no-cpu-baseline] [--no-serve]

One step is one call of the library on one batch of synthetic, device-resident input (every pass of
the path the workload needs: planning, the DP relaxation, optimum selection, 16/32-bit redo, and the
traceback when the workload asks for CIGARs).  Prints one JSON line.

Workloads (synth/__init__.py has the recipes):
  protein  65,536 protein pairs, lengths log-uniform 64..16384, local affine (-11/-1), score-only     [default]
           The line also carries the same batch as one captured HIP graph, as one call per length bin,
           and one pair per call (the "plain" form), and, unless --no-serve, a "serve" record: the
           request stream below at 20,000 requests/s with p50/p99 latency per class.
  reads    1,048,576 read/window pairs, semi-global affine (-5/-2, +1/-4), CIGAR for every pair
  long     1 pair 262144 x 262144 DNA, local affine (-3/-1, +2/-3), score + end cell
  long_tb  the same pair with its CIGAR, a 4-bit code stored per cell (34 GB; --linear-space: the library's
           default for pairs above 2^24 cells, checkpoints and tiles relaxed again)
  long_tb_393216  a 393216 x 393216 pair made the same way, with its CIGAR: its 4-bit codes would take 72 GiB,
           so the traceback runs in linear space
  nw1k     1 pair 1000 x 1000 DNA, global linear (+2/-1, gap -1), CIGAR
  serve    only the request stream through the continuous-batching server (paper_2002_04561_amd/serve.py):
           a Poisson stream of 80% read/window pairs with CIGARs, 19% protein pairs (lengths log-uniform
           64..16384) and 1% local DNA pairs of 65536 x 65536; GCUPS over the run and p50/p99 latency per class
"""
import argparse
import json
import os
import sys
import time

import numpy as np

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

# Integer VALU peak of MI355X (256 CUs x 4 SIMDs at 2.4 GHz), in 2-input ops: a SIMD retires at most 32 a
# cycle -- a 32-bit add takes 2 cycles per wave64 instruction, a 3-input max (two ops) or a packed 16-bit
# instruction (two lanes) takes 4, and a 2-input max, a bit-field extract or a DPP move takes 4 for one op
# a lane.  A microbenchmark of independent chains at 8 waves per SIMD measured 63 T lane-ops/s for
# v_add_u32 (70 T for v_add_f32), 38 T instructions for v_max_i32, v_max3_i32, v_bfe_i32 and v_pk_add_u16.
# 256 x 4 x 32 x 2.4e9 = 78.64 T ops/s bounds every mix of adds and maxes, in 32 or in packed 16 bits.
PEAK_I32_TOPS = 256 * 4 * 32 * 2.4e9 / 1e12
PEAK_I16_TOPS = PEAK_I32_TOPS

# Algorithmic integer ops per DP cell (each 2-input add/sub/max and the substitution lookup count 1):
# linear: sigma, diagonal add, up+g, left+g, max3 (2) = 5 ... as in Eqs. (1)-(5).
OPS_PER_CELL = {("global", "linear"): 5, ("semiglobal", "linear"): 5, ("local", "linear"): 7,
                ("global", "affine"): 10, ("semiglobal", "affine"): 10, ("local", "affine"): 12}
MODE_NAME = {0: "global", 1: "local", 2: "semiglobal"}


def make_workload(name, pairs=None):
    import synth
    if name == "long":
        return synth.long_dna_local()
    if name == "long_tb":
        import dataclasses
        return dataclasses.replace(synth.long_dna_local(), traceback=True)
    if name == "long_tb_393216":
        import dataclasses
        return dataclasses.replace(synth.long_dna_local(n=393216), traceback=True)
    if name == "reads":
        return synth.reads_semiglobal(n_pairs=pairs or (1 << 20))
    if name == "protein":
        return synth.protein_uneven(n_pairs=pairs or 65536)
    if name == "nw1k":
        return synth.long_dna_global_1k()
    raise SystemExit("unknown workload %s" % name)


def _measured_traffic(kernel, workload):
    """HBM bytes per launch of `kernel` on `workload` from a committed PMC summary, or None.

    profiles/traffic_*.json hold FETCH_SIZE / WRITE_SIZE per dispatch scaled by what the same counters
    read for a copy of known size; a summary counts only while the kernel's source file still has the
    hash it was taken at."""
    import glob
    import hashlib
    for path in sorted(glob.glob(os.path.join(ROOT, "profiles", "traffic_*.json"))):
        with open(path) as fh:
            rec = json.load(fh)
        if rec.get("kernel") != kernel or rec.get("workload") != workload:
            continue
        src = os.path.join(ROOT, rec["source"])
        if not os.path.exists(src):
            continue
        with open(src, "rb") as fh:
            digest = hashlib.sha256(fh.read()).hexdigest()[:16]
        if digest == rec.get("source_sha256_16"):
            return float(rec["traffic_bytes_per_launch"])
    return None


def _oracle_scoring(w):
    import oracle
    return oracle.Scoring.matrix(w.mode, w.sigma_table(), w.gap_open, w.gap_extend)


def run_cpu_baseline(w, budget_s=20.0):
    """The oracle as it stands, on a bounded sample of the workload, on the host's cores."""
    import oracle
    threads = len(os.sched_getaffinity(0))
    sc = _oracle_scoring(w)
    n, m = w.lengths()
    cells = n.astype(np.int64) * m.astype(np.int64)
    if w.n_pairs == 1:
        # one long pair: the oracle runs on one thread; sample = the first rows of the matrix
        a, b = w.pair(0)
        rows = max(1, min(len(a), int(1e10 / max(len(b), 1))))
        t0 = time.perf_counter()
        oracle.align(sc, a[:rows], b, traceback=w.traceback, impl="affine" if w.traceback else "linspace")
        dt = time.perf_counter() - t0
        return {"value": rows * len(b) / dt / 1e9, "unit": "GCUPS", "cores": 1, "kind": "oracle",
                "sample": "first %d rows x %d columns of the pair (%.1f s)" % (rows, len(b), dt)}
    # batches: pairs in order until the measured time reaches the budget, calibrated on a prefix of
    # about a second (a prefix of a few pairs keeps few cores busy and understates the rate)
    csum = np.cumsum(cells)
    k, dt = min(w.n_pairs, 64), 0.0
    while True:
        t0 = time.perf_counter()
        sub = w.subset(np.arange(k))
        oracle.align_batch(sc, sub.q, sub.q_off, sub.s, sub.s_off, traceback=w.traceback, threads=threads)
        dt = max(time.perf_counter() - t0, 1e-3)
        if dt > 1.0 or k == w.n_pairs:
            break
        k = min(w.n_pairs, k * 4)
    rate = cells[:k].sum() / dt
    target = rate * budget_s
    k2 = int(min(w.n_pairs, max(k, np.searchsorted(csum, target))))
    sub = w.subset(np.arange(k2))
    t0 = time.perf_counter()
    oracle.align_batch(sc, sub.q, sub.q_off, sub.s, sub.s_off, traceback=w.traceback, threads=threads)
    dt = time.perf_counter() - t0
    return {"value": float(csum[k2 - 1]) / dt / 1e9, "unit": "GCUPS", "cores": threads, "kind": "oracle",
            "sample": "first %d of %d pairs, %.3g cells, %s (%.1f s)" % (
                k2, w.n_pairs, float(csum[k2 - 1]), "with traceback" if w.traceback else "score-only", dt)}


GOLDEN = {"long_dna_local_262144": "long_local_262144.json", "long_dna_local_393216": "long_local_393216.json",
          "long_dna_global_1k": "global_1k.json",
          "reads_semiglobal": "reads_sample.json", "protein_uneven": "protein_sample.json"}


def _cigar_string(runs):
    return "".join("%d%s" % (n, "MID"[op]) for n, op in runs)


def golden_pairs(w):
    """Indices of the pairs whose expected results tests/golden/ holds for this workload (written there by
    tests/golden/make_golden.py from the oracle), or None."""
    path = os.path.join(ROOT, "tests", "golden", GOLDEN.get(w.name, "-"))
    if not os.path.exists(path):
        return None, None
    g = json.load(open(path))
    if "pairs" in g:
        if g["n_pairs"] != w.n_pairs or bool(g["traceback"]) != bool(w.traceback):
            return None, None
        return [p["k"] for p in g["pairs"]], g["pairs"]
    return [0], [dict(g, k=0)]


def spot_check(w, res, cigars, idx, expect):
    """Compares pairs bit-exactly with the oracle's stored results (score, end cell, and the begin cell and
    CIGAR when traced back)."""
    if expect is None:
        return "not checked (no stored oracle values for this workload)"
    for e in expect:
        k = int(e["k"])
        g = (int(res["score"][k]), int(res["q_end"][k]), int(res["s_end"][k]))
        o = (e["score"], e["q_end"], e["s_end"])
        if g != o:
            return "MISMATCH pair %d" % k
        if w.traceback and "cigar" in e:
            g = (int(res["q_begin"][k]), int(res["s_begin"][k]), _cigar_string(cigars[k]))
            if g != (e["q_begin"], e["s_begin"], e["cigar"]):
                return "MISMATCH pair %d (CIGAR)" % k
    return "bit-exact vs the stored oracle values of %d pair(s)" % len(expect)


DIGESTS = {"reads_semiglobal": "reads_digest.json", "protein_uneven": "protein_digest.json"}


def digest_check(w, ba, res):
    """Every pair of a full batch against the oracle: chunk digests of all results (tests/golden/digest.py)
    compared with the stored digests of the oracle's results."""
    path = os.path.join(ROOT, "tests", "golden", DIGESTS.get(w.name, "-"))
    if not os.path.exists(path):
        return None
    g = json.load(open(path))
    if g["n_pairs"] != w.n_pairs or bool(g["traceback"]) != bool(w.traceback):
        return None
    sys.path.insert(0, os.path.join(ROOT, "tests", "golden"))
    import digest
    if w.traceback:
        d = digest.chunk_digests(res, True, ba.cigar.to("cpu").numpy().view(np.uint32), ba.cigar_off.to("cpu").numpy())
    else:
        d = digest.chunk_digests(res, False)
    bad = sum(1 for x, y in zip(d, g["digests"]) if x != y) + abs(len(d) - len(g["digests"]))
    if bad:
        return "MISMATCH in %d of %d chunks of all pairs' digests" % (bad, len(g["digests"]))
    return "all %d pairs bit-exact vs the oracle's digests (%d chunks)" % (w.n_pairs, len(d))


def time_graph(ba, stream, steps):
    """The batch call captured once in a HIP graph and replayed `steps` times; ms per replay."""
    import torch
    g = torch.cuda.CUDAGraph()
    side = torch.cuda.Stream()
    side.wait_stream(stream)
    with torch.cuda.stream(side):
        with torch.cuda.graph(g):
            ba.run()
    stream.wait_stream(side)
    torch.cuda.synchronize()
    with torch.cuda.stream(stream):
        g.replay()
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        for _ in range(steps):
            g.replay()
        torch.cuda.synchronize()
    return (time.perf_counter() - t0) * 1e3 / steps, g


def _sub_aligner(w, idx, flags, config=None):
    import paper_2002_04561_amd as aln
    sub = w.subset(np.asarray(idx))
    n, m = sub.lengths()
    q, qo, s, so = aln.to_device(sub)
    return aln.BatchAligner(aln.scoring_of(sub), q, qo, s, so, max(int(n.max()), 1), max(int(m.max()), 1), flags,
                            config=config), sub


def time_per_bin(w, flags, stream, steps, config=None, tune_each=False):
    """One aln_align_batch call per length bin (bins of log2 max(n, m)), run back to back on one stream: with
    the given config, or (tune_each) with each bin's own config from the autotuner.  Returns (ms per pass,
    number of calls, the bins' configs)."""
    import torch
    n, m = w.lengths()
    key = np.log2(np.maximum(np.maximum(n, m), 1)).astype(int)
    calls = [_sub_aligner(w, np.nonzero(key == b)[0], flags, config)[0] for b in np.unique(key)]
    cfgs = []
    if tune_each:
        from paper_2002_04561_amd import tune
        for ba in calls:
            cfg, _ = tune.tune(ba, stream)
            cfgs.append(dict(cfg.__dict__))
    for ba in calls:
        ba.run(stream)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    for _ in range(steps):
        for ba in calls:
            ba.run(stream)
    torch.cuda.synchronize()
    return (time.perf_counter() - t0) * 1e3 / steps, len(calls), cfgs


def time_plain(w, flags, stream, count, seed=1):
    """One pair per call: a seeded random sample of the batch's pairs, each its own aln_align_batch call with
    n_pairs = 1 (the same kernels as the batched call, one pair per launch), all enqueued back to back on one
    stream with one synchronisation at the end; GCUPS = sample cells / elapsed time."""
    import torch

    import paper_2002_04561_amd as aln
    rng = np.random.default_rng(seed)
    idx = np.sort(rng.choice(w.n_pairs, size=min(count, w.n_pairs), replace=False))
    n, m = w.lengths()
    sc = aln.scoring_of(w)
    q, qo, s, so = aln.to_device(w)
    sizes = [aln.aln_batch_workspace_size(sc, 1, int(n[k]), int(m[k]), int(n[k]), int(m[k]), flags) for k in idx]
    ws = torch.empty(max(max(sizes), 256), dtype=torch.uint8, device="cuda")
    calls = []
    for k in idx:
        k = int(k)
        # the pair's offsets are absolute positions in the whole batch's arrays; its lengths bound the totals
        calls.append(aln.BatchAligner(sc, q, qo[k:k + 2], s, so[k:k + 2], int(n[k]), int(m[k]), flags,
                                      total_q=int(n[k]), total_s=int(m[k]), workspace=ws))
    for ba in calls[:8]:
        ba.run(stream)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    for ba in calls:
        ba.run(stream)
    torch.cuda.synchronize()
    dt = time.perf_counter() - t0
    cells = float(np.sum(n[idx].astype(np.int64) * m[idx]))
    res = np.concatenate([ba.results() for ba in calls])
    return {"gcups": round(cells / dt / 1e9, 2), "pairs": len(idx), "cells": cells, "seconds": round(dt, 4),
            "sample": "%d seeded random pairs, one aln_align_batch call (n_pairs = 1) per pair, enqueued back to "
                      "back on one stream, one synchronisation" % len(idx)}, idx, res


def check_plain(res_plain, idx, res_batched):
    """The one-pair calls must give the batched call's results."""
    same = all(np.array_equal(res_plain[f], res_batched[f][idx]) for f in ("score", "q_end", "s_end", "flags"))
    return "identical to the batched call on all %d pairs" % len(idx) if same else "DIFFERS from the batched call"


SERVE_GOLDEN = "serve_sample.json"


def serve_requests(n_req, rate_hz, seed=5, long_len=65536):
    """The serving workload's request stream (synth.serve_stream) as server requests."""
    import synth
    from paper_2002_04561_amd.serve import Request
    items, sig = synth.serve_stream(n_req, rate_hz, seed=seed, long_len=long_len)
    # the 65536^2 pairs go through batched calls: the bands of all a call's pairs share one queue
    reqs = [Request(it.rid, it.klass, it.q, it.s, it.arrival, traceback=synth.SERVE_CLASSES[it.klass]["traceback"])
            for it in items]
    return reqs, sig


def serve_check(srv, n_req, seed):
    """Compares the served results of the requests whose oracle results tests/golden/ holds (the first
    requests of each class of the seed-5, 200,000-request stream) bit-exactly."""
    path = os.path.join(ROOT, "tests", "golden", SERVE_GOLDEN)
    if not os.path.exists(path) or n_req != 200000 or seed != 5:
        return "not checked (no stored oracle values for this stream)"
    g = json.load(open(path))
    got = {c.rid: c for c in srv.completed}
    count = 0
    for klass, rows in g["classes"].items():
        for e in rows:
            c = got.get(e["rid"])
            if c is None:
                return "MISSING request %d" % e["rid"]
            score, qb, qe, sb, se, flags = c.result
            if (score, qe, se, flags) != (e["score"], e["q_end"], e["s_end"], 0):
                return "MISMATCH request %d (%s)" % (e["rid"], klass)
            if "cigar" in e and ((qb, sb) != (e["q_begin"], e["s_begin"]) or _cigar_string(c.cigar) != e["cigar"]):
                return "MISMATCH request %d (%s, CIGAR)" % (e["rid"], klass)
            count += 1
    return "bit-exact vs the stored oracle values of %d requests (%s)" % (
        count, ", ".join("%d %s" % (len(v), k) for k, v in g["classes"].items()))


def run_serve(args, log=None):
    """The request stream through the continuous-batching server; returns the record."""
    import torch

    import paper_2002_04561_amd as aln
    import synth
    from paper_2002_04561_amd.serve import AlignServer
    t0 = time.perf_counter()
    reqs, sig = serve_requests(args.requests, args.rate)
    if log:
        log("serve: %d requests generated in %.1f s" % (len(reqs), time.perf_counter() - t0))
    sc = {k: aln.Scoring(c["mode"], c["alphabet_size"], c["gap_open"], c["gap_extend"], match=c.get("match", 0),
                         mismatch=c.get("mismatch", 0), subst=sig if k == "protein" else None)
          for k, c in synth.SERVE_CLASSES.items()}
    torch.cuda.set_device(0)
    warm, _ = serve_requests(64, 1e6, seed=99, long_len=4096)
    AlignServer(sc, budget_bytes=args.budget_gb << 30).run(warm, realtime=False)
    long_cfg = aln.BatchConfig(wf_waves_per_cu=args.serve_long_waves) if args.serve_long_waves else None
    prot_cfg = aln.BatchConfig(wf_min_cells=args.serve_protein_min_cells) if args.serve_protein_min_cells else None
    srv = AlignServer(sc, budget_bytes=args.budget_gb << 30, streams=args.serve_streams, max_pairs=8192,
                      class_max_pairs={"long": args.serve_long_batch}, class_configs={"long": long_cfg, "protein": prot_cfg},
                      class_max_streams={"long": args.serve_long_streams} if args.serve_long_streams else None)
    t_run = time.perf_counter()
    st = srv.run(reqs, realtime=True)
    if log:
        log("serve: %d requests in %.1f s" % (st["requests"], time.perf_counter() - t_run))
    check = serve_check(srv, args.requests, 5)
    if log:
        log("serve parity:", check)
    return {"gcups": round(st["gcups"], 2), "wall_s": round(st["wall_s"], 3), "requests": len(reqs),
            "rate_per_s": args.rate, "cells": st["cells"], "latency_ms": st["classes"],
            "int32_redo_requests": st["int32_redo"], "parity": check, "budget_bytes": st["budget_bytes"],
            "peak_bytes": st["peak_bytes"], "streams": args.serve_streams, "long_batch": args.serve_long_batch,
            "protein_min_cells": args.serve_protein_min_cells,
            "what": "Poisson stream: 80% read/window pairs with CIGARs, 19% protein pairs (64..16384), 1% "
                    "65536 x 65536 local DNA pairs; latency = completion - arrival"}


def print_serve_line(args):
    rec = run_serve(args, lambda *a: print("[bench]", *a, file=sys.stderr, flush=True))
    out = {
        "metric": "GCUPS (batched vs plain, bit-exact) on one MI355X; p50/p99 request latency",
        "value": rec["gcups"], "unit": "GCUPS", "n_gpus": 1, "steps": 1, "warmup": 1,
        "ms_per_step": round(rec["wall_s"] * 1e3, 1), "higher_is_better": True, "scaling": "weak",
        "vs_baseline": None, "dtype": "int16+int32", "data": "synthetic (seeded generator)",
        "config": {"workload": "serve", "requests": rec["requests"], "rate_per_s": args.rate},
        "parity": rec["parity"], "serve": rec,
    }
    print(json.dumps(out), flush=True)


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=10)
    ap.add_argument("--warmup", type=int, default=2)
    ap.add_argument("--workload", default="protein", choices=["long", "long_tb", "long_tb_393216", "reads", "protein", "nw1k", "serve"])
    ap.add_argument("--no-serve", action="store_true", help="protein: leave out the serving record")
    ap.add_argument("--plain-pairs", type=int, default=2048, help="pairs timed one per call (the plain form)")
    ap.add_argument("--requests", type=int, default=200000, help="serve: number of requests")
    ap.add_argument("--rate", type=float, default=20000.0, help="serve: Poisson arrival rate (requests/s)")
    ap.add_argument("--budget-gb", type=int, default=64, help="serve: device memory budget (GiB)")
    ap.add_argument("--serve-streams", type=int, default=4, help="serve: batches in flight (one HIP stream each)")
    ap.add_argument("--serve-long-batch", type=int, default=8, help="serve: most 65536^2 pairs in one batch call")
    ap.add_argument("--serve-protein-min-cells", type=int, default=1,
                    help="serve: wf_min_cells of the protein calls (0 = the library's default, 2^16)")
    ap.add_argument("--serve-long-streams", type=int, default=0,
                    help="serve: most 65536^2-pair batches in flight at once (0 = no limit)")
    ap.add_argument("--serve-long-waves", type=int, default=0,
                    help="serve: wf_waves_per_cu for the 65536^2 pairs' calls (0 = the library's default)")
    ap.add_argument("--copy-calibration", action="store_true",
                    help="run only a plain 1 GiB device-to-device copy (scale for rocprofv3 FETCH_SIZE/WRITE_SIZE)")
    ap.add_argument("--pairs", type=int, default=None, help="override the pair count of a batch workload")
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--no-tune", action="store_true", help="batch workloads: library defaults instead of autotuning")
    ap.add_argument("--config", default=None,
                    help="batch workloads: a fixed aln_batch_config_t as JSON (no autotuning), e.g. "
                         "'{\"wf_min_cells\": 1, \"wf_waves_per_cu\": 32, \"wf_orient\": 2}'")
    ap.add_argument("--no-compare", action="store_true",
                    help="batch workloads: skip the graph / per-length-bin / one-pair-per-call comparisons")
    ap.add_argument("--no-check", action="store_true")
    ap.add_argument("--linear-space", action="store_true",
                    help="long_tb: trace back in linear space (checkpoints, tiles relaxed again), the library's "
                         "default above 2^24 cells, instead of storing the 4-bit code of every cell")
    args = ap.parse_args()
    if args.gpus != 1:
        print("bench.py runs on one GPU only: the library has no multi-GPU path", file=sys.stderr)
        sys.exit(2)

    if args.copy_calibration:
        import torch
        x = torch.ones(1 << 28, dtype=torch.int32, device="cuda")
        y = torch.empty_like(x)
        torch.cuda.synchronize()
        y.copy_(x)
        torch.cuda.synchronize()
        print(json.dumps({"copy_bytes_read": 1 << 30, "copy_bytes_written": 1 << 30}))
        return
    if args.workload == "serve":
        print_serve_line(args)
        return

    import torch

    import paper_2002_04561_amd as aln

    def log(*a):
        print("[bench]", *a, file=sys.stderr, flush=True)

    torch.cuda.set_device(0)
    t0 = time.time()
    w = make_workload(args.workload, args.pairs)
    n, m = w.lengths()
    cells = w.cells()
    log("workload %s: %d pairs, %.4g cells, generated in %.1f s" % (w.name, w.n_pairs, cells, time.time() - t0))
    stream = torch.cuda.Stream()
    flags = aln.TRACEBACK if w.traceback else aln.SCORE_ONLY
    # a single pair runs through aln_align_long, unless an explicit batch config asks for the batch API
    long_path = (w.n_pairs == 1) and not args.config
    with torch.cuda.stream(stream):
        q, qo, s, so = aln.to_device(w)
        if long_path:
            if args.linear_space:
                flags |= aln.LINEAR_SPACE
            elif flags & aln.TRACEBACK:
                flags |= aln.STORED_CODES  # a code per cell (while it fits), as the workload's name says
            ba = aln.LongAligner(aln.scoring_of(w), q[:int(n[0])], s[:int(m[0])], flags)
        else:
            ba = aln.BatchAligner(aln.scoring_of(w), q, qo, s, so, int(n.max()), int(m.max()), flags)
    torch.cuda.synchronize()
    log("device buffers ready; workspace %.3g GB" % (ba.ws_bytes / 1e9))
    tuned = None
    if not long_path and args.config:
        ba.config = aln.BatchConfig(**json.loads(args.config))
        tuned = {"config": ba.config.__dict__, "seconds": 0.0, "candidates": 0, "fixed": True}
    elif not long_path and not args.no_tune:
        from paper_2002_04561_amd import tune
        t0 = time.perf_counter()
        cfg, table = tune.tune(ba, stream, log=log)
        tuned = {"config": cfg.__dict__, "seconds": round(time.perf_counter() - t0, 2), "candidates": len(table)}
        log("tuned config %s in %.1f s" % (cfg, tuned["seconds"]))
    for _ in range(args.warmup):
        ba.run(stream)
    torch.cuda.synchronize()
    aln.aln_profile_enable(True)
    aln.aln_profile_reset()
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    for _ in range(args.steps):
        ba.run(stream)
    torch.cuda.synchronize()
    t1 = time.perf_counter()
    prof = aln.aln_profile_read()
    aln.aln_profile_enable(False)
    ms = (t1 - t0) * 1e3 / args.steps
    gcups = cells / (ms * 1e-3) / 1e9
    log("%.3f ms/step, %.1f GCUPS; kernels %s" % (ms, gcups, prof))

    res = ba.result().reshape(1) if long_path else ba.results()
    idx, expect = golden_pairs(w)
    idx = idx or []
    if long_path:
        cigars = {0: ba.cigar_runs()} if w.traceback else None
    else:
        cigars = ba.cigars(idx) if w.traceback else None
    check = "skipped" if args.no_check else spot_check(w, res, cigars, idx, expect)
    if not args.no_check and not long_path and not check.startswith("MISMATCH"):
        dcheck = digest_check(w, ba, res)
        if dcheck:
            check = dcheck if dcheck.startswith("MISMATCH") else "%s; %s" % (dcheck, check)
    log("parity:", check)

    gap = "linear" if w.gap_open == 0 else "affine"
    opc = OPS_PER_CELL[(MODE_NAME[w.mode], gap)]
    dom = max(((k, v) for k, v in prof.items() if k != "plan"), key=lambda kv: kv[1][1]) if prof else None
    dtype = "int16" if (dom and ("i16" in dom[0] or "p16" in dom[0])) else "int32"
    peak = PEAK_I32_TOPS if dtype == "int32" else PEAK_I16_TOPS
    roof = None
    if dom:
        per_launch_ms = dom[1][1] / max(dom[1][0], 1)
        launches_per_step = dom[1][0] / args.steps
        cells_per_launch = cells / max(launches_per_step, 1e-9)
        # the step's cells are attributed to the dominant kernel; when other DP kernels also took a share of
        # them (pairs split between the band wavefront and one pair per lane), their time is added, so that
        # the rate is never credited with work another kernel did
        others = sum(v[1] for k, v in prof.items() if k not in ("plan", dom[0]))
        if others > 0.01 * dom[1][1]:
            per_launch_ms = (dom[1][1] + others) / max(dom[1][0], 1)
        achieved = opc * cells_per_launch / (per_launch_ms * 1e-3) / 1e12
        roof = {"bound": "alu", "achieved": round(achieved, 3), "peak": round(peak, 2), "unit": "Tops/s",
                "frac": round(achieved / peak, 4), "traffic": _measured_traffic(dom[0], w.name), "kernel": dom[0],
                "kernel_ms": round(per_launch_ms, 4), "ops_per_cell": opc,
                "kernels_ms_per_step": {k: round(v[1] / args.steps, 4) for k, v in prof.items()}}
    out = {
        "metric": "GCUPS (batched vs plain, bit-exact) on one MI355X; p50/p99 request latency",
        "value": round(gcups, 2), "unit": "GCUPS", "n_gpus": 1, "steps": args.steps, "warmup": args.warmup,
        "ms_per_step": round(ms, 4), "higher_is_better": True, "scaling": "weak", "vs_baseline": None,
        "dtype": dtype, "data": "synthetic (seeded generator, synth/__init__.py)",
        "config": {"workload": w.name, "pairs": w.n_pairs, "cells": cells, "mode": MODE_NAME[w.mode], "gap": gap,
                   "gap_open": w.gap_open, "gap_extend": w.gap_extend, "traceback": bool(w.traceback),
                   "linear_space": bool(flags & aln.LINEAR_SPACE) or bool(
                       flags & aln.TRACEBACK and w.n_pairs == 1 and (int(n[0]) + 256) // 2 * int(m[0]) > (64 << 30))},
        "parity": check,
        "roofline": roof,
    }
    if tuned:
        out["tuned"] = tuned
    if not long_path and not args.no_compare:
        gms, _ = time_graph(ba, stream, args.steps)
        out["graph"] = {"ms_per_step": round(gms, 4), "gcups": round(cells / (gms * 1e-3) / 1e9, 2),
                        "what": "the same call captured once in a HIP graph, replayed"}
        log("graph replay: %.3f ms" % gms)
        bms, nbins, _ = time_per_bin(w, flags, stream, max(1, min(args.steps, 3)), ba.config)
        out["per_length_bin"] = {"ms_per_step": round(bms, 4), "gcups": round(cells / (bms * 1e-3) / 1e9, 2),
                                 "calls": nbins, "what": "one call per bin of log2 max(n, m), back to back"}
        log("per length bin: %.3f ms in %d calls" % (bms, nbins))
        if not args.no_tune and not args.config:
            tms, nbins, bcfgs = time_per_bin(w, flags, stream, max(1, min(args.steps, 3)), None, tune_each=True)
            out["per_length_bin_tuned"] = {
                "ms_per_step": round(tms, 4), "gcups": round(cells / (tms * 1e-3) / 1e9, 2), "calls": nbins,
                "configs": bcfgs, "what": "one call per bin, each bin with its own autotuned config"}
            log("per length bin, tuned per bin: %.3f ms" % tms)
        plain, pidx, pres = time_plain(w, flags, stream, args.plain_pairs)
        plain["parity"] = check_plain(pres, pidx, res)
        out["plain"] = plain
        out["batched_vs_plain"] = round(gcups / plain["gcups"], 2)
        log("plain: %s" % plain)
    if args.workload == "protein" and not args.no_serve:
        out["serve"] = run_serve(args, log)
    if not args.no_cpu_baseline:
        log("timing the oracle on a host sample ...")
        out["cpu_baseline"] = run_cpu_baseline(w)
    print(json.dumps(out), flush=True)


if __name__ == "__main__":
    main()
