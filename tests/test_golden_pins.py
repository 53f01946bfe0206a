"""The stored expected values under tests/golden/ reproduce from the oracle as it stands: the digest of
the first chunk of the read/window batch's results (with CIGARs), and the first stored requests of the
read and protein classes of the serving stream.  (The full digests take minutes of host time and are
written by tests/golden/make_golden.py.)"""
import json
import os
import sys

import numpy as np

import oracle
import synth
from helpers import oracle_scoring

HERE = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, os.path.join(HERE, "golden"))
import digest  # noqa: E402


def test_reads_digest_first_chunk_reproduces():
    g = json.load(open(os.path.join(HERE, "golden", "reads_digest.json")))
    w = synth.reads_semiglobal(n_pairs=1 << 20)
    sub = w.subset(np.arange(g["chunk"]))
    res, cig, coff = oracle.align_batch(oracle_scoring(sub), sub.q, sub.q_off, sub.s, sub.s_off, traceback=True)
    assert digest.chunk_digests(res, True, cig, coff, chunk=g["chunk"]) == g["digests"][:1]


def test_digest_detects_a_changed_cigar_word():
    w = synth.reads_semiglobal(n_pairs=64)
    res, cig, coff = oracle.align_batch(oracle_scoring(w), w.q, w.q_off, w.s, w.s_off, traceback=True)
    d0 = digest.chunk_digests(res, True, cig, coff, chunk=32)
    cig2 = cig.copy()
    cig2[coff[40]] ^= 16  # one run length of pair 40 changed
    d1 = digest.chunk_digests(res, True, cig2, coff, chunk=32)
    assert d0[0] == d1[0] and d0[1] != d1[1]


def test_serve_sample_reproduces():
    g = json.load(open(os.path.join(HERE, "golden", "serve_sample.json")))
    items, sig = synth.serve_stream(64, 1.0, seed=5)  # the sequences do not depend on the rate or the count
    by_rid = {it.rid: it for it in items}
    for klass in ("read", "protein"):
        rows = [e for e in g["classes"][klass] if e["rid"] in by_rid][:4]
        assert rows
        w = synth.serve_workload([by_rid[e["rid"]] for e in rows], klass, sig)
        res, cig, coff = oracle.align_batch(oracle_scoring(w), w.q, w.q_off, w.s, w.s_off, traceback=w.traceback)
        for k, e in enumerate(rows):
            assert (int(res["score"][k]), int(res["q_end"][k]), int(res["s_end"][k])) == (
                e["score"], e["q_end"], e["s_end"])
            if w.traceback:
                L = int(res["cigar_len"][k])
                runs = [(int(x) >> 4, int(x) & 15) for x in cig[coff[k]:coff[k] + L]]
                assert oracle.cigar_string(runs) == e["cigar"]
