"""Randomised parity sweep.  Each case draws its own scoring scheme (2 to 24 letters; a symmetric or
asymmetric substitution table, or match/mismatch; linear or affine gaps), its mode, score-only or
traceback, and an execution configuration: which pairs take the band wavefront, its orientation, grouping
and cell width, and the width of the one-pair-per-lane kernels.  Every pair of the batch (lengths 0..260,
half of the subjects mutated copies of their queries, so optima and ties are not all near zero) must equal
the oracle bit for bit: score, end cell, begin cell and CIGAR."""
import numpy as np
import pytest

import synth
from helpers import compare, run_gpu, run_oracle

pytestmark = pytest.mark.gpu

ALPHABETS = (2, 3, 4, 5, 8, 12, 13, 20, 24)


def _case(seed):
    rng = np.random.default_rng(9000 + seed)
    A = int(rng.choice(ALPHABETS))
    mode = int(rng.integers(0, 3))
    if rng.random() < 0.6:
        t = rng.integers(-6, 3, (A, A))
        if rng.random() < 0.5:
            t = np.triu(t, 1)
            t = t + t.T
        np.fill_diagonal(t, rng.integers(1, 9, A))
        subst, match, mismatch = t.astype(np.int8), None, None
    else:
        subst, match, mismatch = None, int(rng.integers(1, 6)), -int(rng.integers(1, 6))
    ge = -int(rng.integers(1, 4))
    go = 0 if rng.random() < 0.3 else -int(rng.integers(1, 12))
    tb = bool(rng.random() < 0.5)
    w = synth.random_pairs(int(rng.integers(1 << 30)), 96, 0, 260, A, mode, go, ge, match=match,
                           mismatch=mismatch, subst=subst, related=0.5)
    cfg = None
    if rng.random() < 0.7:
        cfg = dict(wf_min_cells=int(rng.choice([1, 4096, 1 << 14, 1 << 20])),
                   wf_orient=int(rng.choice([-1, 1, 2])),
                   wf_group=int(rng.choice([1, 4])),
                   wf_waves_per_cu=int(rng.choice([0, 4, 16])),
                   small_bits=int(rng.choice([16, 32])),
                   wf_bits=int(rng.choice([16, 32])))
    label = "seed %d: A=%d mode=%d go=%d ge=%d table=%s tb=%s cfg=%s" % (
        seed, A, mode, go, ge, "no" if subst is None else "yes", tb, cfg)
    return w, tb, cfg, label


@pytest.mark.parametrize("seed", range(64))
def test_random_scheme_batch(gpu, seed):
    import paper_2002_04561_amd as aln
    w, tb, cfg, label = _case(seed)
    print(label, flush=True)
    config = aln.BatchConfig(**cfg) if cfg else None
    gres, gcig = run_gpu(w, aln.TRACEBACK if tb else aln.SCORE_ONLY, config=config)
    ores, ocig = run_oracle(w, tb)
    bad = compare(w, gres, gcig, ores, ocig, label)
    assert not bad, "\n".join(bad[:10])
