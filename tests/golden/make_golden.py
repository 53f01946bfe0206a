"""Writes the stored expected values under tests/golden/ by calling only the oracle.

Every value here comes from oracle/ (plain scalar C, pinned by brute force in
tests/test_oracle_pins.py) run on the seeded synthetic workloads of synth/.
Usage: python tests/golden/make_golden.py [name ...]
"""
import json
import os
import sys
import time

HERE = os.path.dirname(os.path.abspath(__file__))
ROOT = os.path.dirname(os.path.dirname(HERE))
sys.path.insert(0, ROOT)

import oracle  # noqa: E402
import synth  # noqa: E402


def _sc(w):
    return oracle.Scoring.matrix(w.mode, w.sigma_table(), w.gap_open, w.gap_extend)


def long_local_262144():
    """The 262144 x 262144 local affine DNA pair (score and end cell), oracle in two rows of memory."""
    w = synth.long_dna_local(seed=2, n=262144)
    a, b = w.pair(0)
    t0 = time.time()
    r = oracle.align(_sc(w), a, b, impl="linspace")
    return {"workload": "long_dna_local(seed=2, n=262144)", "mode": "local", "gap_open": -3, "gap_extend": -1,
            "match": 2, "mismatch": -3, "score": r.score, "q_end": r.q_end, "s_end": r.s_end,
            "oracle_seconds": round(time.time() - t0, 1)}


def long_local_393216():
    """The 393216 x 393216 local affine DNA pair (score and end cell): its 4-bit codes would take 72 GiB, so
    its traceback runs in linear space."""
    w = synth.long_dna_local(seed=2, n=393216)
    a, b = w.pair(0)
    t0 = time.time()
    r = oracle.align(_sc(w), a, b, impl="linspace")
    return {"workload": "long_dna_local(seed=2, n=393216)", "mode": "local", "gap_open": -3, "gap_extend": -1,
            "match": 2, "mismatch": -3, "score": r.score, "q_end": r.q_end, "s_end": r.s_end,
            "oracle_seconds": round(time.time() - t0, 1)}


def long_local_262144_cigar():
    """The canonical CIGAR of the 262144 x 262144 local affine pair, from the oracle's linear-space traceback
    (every 512th row kept, one block of full matrices at a time): begin and end cells, the run count and
    the SHA-256 of the CIGAR words (little-endian uint32, (length << 4) | op), with the first and last runs."""
    import hashlib
    import numpy as np
    w = synth.long_dna_local(seed=2, n=262144)
    a, b = w.pair(0)
    t0 = time.time()
    r = oracle.align(_sc(w), a, b, traceback=True, impl="checkpointed", block_rows=512)
    words = np.array([(L << 4) | op for L, op in r.cigar], dtype="<u4")
    return {"workload": "long_dna_local(seed=2, n=262144)", "mode": "local", "gap_open": -3, "gap_extend": -1,
            "match": 2, "mismatch": -3, "score": r.score, "q_begin": r.q_begin, "q_end": r.q_end,
            "s_begin": r.s_begin, "s_end": r.s_end, "cigar_len": len(r.cigar),
            "cigar_sha256": hashlib.sha256(words.tobytes()).hexdigest(),
            "cigar_head": oracle.cigar_string(r.cigar[:12]), "cigar_tail": oracle.cigar_string(r.cigar[-12:]),
            "oracle_seconds": round(time.time() - t0, 1)}


def global_1k():
    """The 1000 x 1000 global linear DNA pair with its canonical CIGAR."""
    w = synth.long_dna_global_1k(seed=1)
    a, b = w.pair(0)
    r = oracle.align(_sc(w), a, b, traceback=True)
    return {"workload": "long_dna_global_1k(seed=1)", "mode": "global", "gap_open": 0, "gap_extend": -1, "match": 2,
            "mismatch": -1, "score": r.score, "q_begin": r.q_begin, "q_end": r.q_end, "s_begin": r.s_begin,
            "s_end": r.s_end, "cigar": oracle.cigar_string(r.cigar)}


def _sample(w, traceback, count=64, seed=0):
    """The oracle's results on a seeded sample of a batch's pairs (the pairs bench.py checks)."""
    import numpy as np
    idx = np.random.default_rng(seed).choice(w.n_pairs, size=min(count, w.n_pairs), replace=False)
    sc = _sc(w)
    out = []
    for k in idx:
        a, b = w.pair(int(k))
        if traceback:
            r = oracle.align(sc, a, b, traceback=True)
            out.append({"k": int(k), "score": r.score, "q_begin": r.q_begin, "q_end": r.q_end, "s_begin": r.s_begin,
                        "s_end": r.s_end, "cigar": oracle.cigar_string(r.cigar)})
        else:
            r = oracle.align(sc, a, b, impl="linspace")
            out.append({"k": int(k), "score": r.score, "q_end": r.q_end, "s_end": r.s_end})
    return {"workload": w.name, "n_pairs": w.n_pairs, "traceback": traceback, "pairs": out}


def reads_sample():
    """64 seeded pairs of the 2^20 read/window batch (semi-global affine) with their canonical CIGARs."""
    return _sample(synth.reads_semiglobal(n_pairs=1 << 20), True)


def protein_sample():
    """64 seeded pairs of the 65536-pair protein batch (local affine), score and end cell."""
    return _sample(synth.protein_uneven(n_pairs=65536), False)


def _digests(w):
    """Chunked digests (tests/golden/digest.py) of the oracle's results on every pair of a batch."""
    sys.path.insert(0, HERE)
    import digest
    t0 = time.time()
    res, cig, coff = oracle.align_batch(_sc(w), w.q, w.q_off, w.s, w.s_off, traceback=w.traceback)
    secs = time.time() - t0
    d = digest.chunk_digests(res, w.traceback, cig, coff)
    return {"workload": w.name, "n_pairs": w.n_pairs, "traceback": bool(w.traceback), "chunk": digest.CHUNK,
            "fields": list(digest.FIELDS_TB if w.traceback else digest.FIELDS_SCORE), "digests": d,
            "oracle_seconds": round(secs, 1)}


def reads_digest():
    """Every pair of the 2^20 read/window batch (semi-global affine, canonical CIGARs), as chunk digests."""
    return _digests(synth.reads_semiglobal(n_pairs=1 << 20))


def protein_digest():
    """Every pair of the 65536-pair protein batch (local affine, score and end cell), as chunk digests."""
    return _digests(synth.protein_uneven(n_pairs=65536))


SERVE_REQUESTS, SERVE_SEED = 200000, 5
SERVE_SAMPLE = {"read": 32, "protein": 32, "long": 8}


def serve_sample():
    """The oracle's results for the first requests of each class of the serving stream (seed 5, 200,000
    requests; the sequences do not depend on the arrival rate)."""
    items, sig = synth.serve_stream(SERVE_REQUESTS, 1.0, seed=SERVE_SEED)
    out = {"workload": "serve_stream(seed=%d, n_req=%d)" % (SERVE_SEED, SERVE_REQUESTS), "classes": {}}
    for klass, count in SERVE_SAMPLE.items():
        sel = [it for it in items if it.klass == klass][:count]
        w = synth.serve_workload(sel, klass, sig)
        res, cig, coff = oracle.align_batch(_sc(w), w.q, w.q_off, w.s, w.s_off, traceback=w.traceback)
        rows = []
        for k, it in enumerate(sel):
            e = {"rid": it.rid, "score": int(res["score"][k]), "q_end": int(res["q_end"][k]),
                 "s_end": int(res["s_end"][k])}
            if w.traceback:
                L = int(res["cigar_len"][k])
                e.update(q_begin=int(res["q_begin"][k]), s_begin=int(res["s_begin"][k]),
                         cigar=oracle.cigar_string([(int(x) >> 4, int(x) & 15) for x in cig[coff[k]:coff[k] + L]]))
            rows.append(e)
        out["classes"][klass] = rows
    return out


JOBS = {"long_local_262144": long_local_262144, "long_local_393216": long_local_393216,
        "long_local_262144_cigar": long_local_262144_cigar, "global_1k": global_1k, "reads_sample": reads_sample,
        "protein_sample": protein_sample, "reads_digest": reads_digest, "protein_digest": protein_digest,
        "serve_sample": serve_sample}

if __name__ == "__main__":
    names = sys.argv[1:] or list(JOBS)
    for name in names:
        val = JOBS[name]()
        path = os.path.join(HERE, name + ".json")
        with open(path, "w") as f:
            json.dump(val, f, indent=1)
            f.write("\n")
        print("wrote", path, {k: (v if len(str(v)) < 200 else "...") for k, v in val.items() if k != "cigar"})
