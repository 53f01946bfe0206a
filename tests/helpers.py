"""Test-side helpers: run a workload through the HIP library and through the oracle, compare."""
from __future__ import annotations

import numpy as np

import oracle
import synth


def oracle_scoring(w: synth.Workload) -> oracle.Scoring:
    return oracle.Scoring.matrix(w.mode, w.sigma_table(), w.gap_open, w.gap_extend)


def run_oracle(w: synth.Workload, traceback: bool, threads=None):
    """Returns (results structured array, list of CIGAR run lists or None)."""
    res, cig, coff = oracle.align_batch(oracle_scoring(w), w.q, w.q_off, w.s, w.s_off, traceback=traceback,
                                        threads=threads)
    cigars = None
    if traceback:
        cigars = []
        for k in range(w.n_pairs):
            L = int(res["cigar_len"][k])
            cigars.append([(int(x) >> 4, int(x) & 15) for x in cig[coff[k]:coff[k] + L]])
    return res, cigars


def run_gpu(w: synth.Workload, flags: int, max_n=None, max_m=None, stream=None, config=None):
    import torch

    import paper_2002_04561_amd as aln
    n, m = w.lengths()
    max_n = int(n.max()) if max_n is None and len(n) else (max_n or 0)
    max_m = int(m.max()) if max_m is None and len(m) else (max_m or 0)
    q, qo, s, so = aln.to_device(w)
    ba = aln.BatchAligner(aln.scoring_of(w), q, qo, s, so, max_n, max_m, flags, config=config)
    ba.run(stream)
    torch.cuda.synchronize()
    res = ba.results()
    cigars = ba.cigars() if flags & aln.TRACEBACK else None
    return res, cigars


def compare(w: synth.Workload, gres, gcig, ores, ocig, label=""):
    """Bit-exact comparison; returns a list of mismatch descriptions (empty when identical)."""
    bad = []
    for k in range(w.n_pairs):
        g = (int(gres["score"][k]), int(gres["q_end"][k]), int(gres["s_end"][k]), int(gres["flags"][k]) & 4)
        o = (int(ores["score"][k]), int(ores["q_end"][k]), int(ores["s_end"][k]), int(ores["flags"][k]) & 4)
        if gcig is not None:
            g = g + (int(gres["q_begin"][k]), int(gres["s_begin"][k]), tuple(gcig[k]))
            o = o + (int(ores["q_begin"][k]), int(ores["s_begin"][k]), tuple(ocig[k]))
        else:
            g = g + (int(gres["q_begin"][k]), int(gres["s_begin"][k]))
            o = o + (-1, -1)
        if g != o:
            n, m = w.lengths()
            bad.append("%s pair %d (n=%d m=%d): gpu %s oracle %s" % (label, k, n[k], m[k], str(g)[:300],
                                                                      str(o)[:300]))
    return bad


def rescore(mode, sigma, go, ge, q, s, q_begin, s_begin, cigar):
    """Re-adds a CIGAR's columns over q[q_begin:], s[s_begin:] (each maximal gap run scores go + k*ge)."""
    i, j, total = q_begin, s_begin, 0
    for length, op in cigar:
        if op == 0:
            for _ in range(length):
                total += int(sigma[q[i]][s[j]])
                i += 1
                j += 1
        elif op == 1:
            total += go + length * ge
            i += length
        else:
            total += go + length * ge
            j += length
    return total, i, j
