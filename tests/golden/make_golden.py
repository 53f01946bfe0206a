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


JOBS = {"long_local_262144": long_local_262144, "global_1k": global_1k, "reads_sample": reads_sample,
        "protein_sample": protein_sample}

if __name__ == "__main__":
    names = sys.argv[1:] or list(JOBS)
    for name in names:
        val = JOBS[name]()
        path = os.path.join(HERE, name + ".json")
        with open(path, "w") as f:
            json.dump(val, f, indent=1)
            f.write("\n")
        print("wrote", path, {k: v for k, v in val.items() if k != "cigar"})
