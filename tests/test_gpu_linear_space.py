"""Linear-space traceback of one pair (aln_align_long with ALN_LINEAR_SPACE, every traceback above 2^24 cells
unless ALN_STORED_CODES asks for a code per cell, and every one above 64 GiB of codes): checkpoint rows and columns kept by the forward pass, tiles relaxed again segment by segment,
bottom first, and walked.  The canonical CIGAR, begin and end cells must equal the oracle's (full
matrices, Sec. III-A) on every shape; a small code budget forces segments of 1024 rows, so walks cross
many segment and tile boundaries, inside gaps too.  At full size the linear-space CIGAR of the 262144^2
pair equals the one of the stored-code walk and the oracle's canonical CIGAR (its own linear-space
traceback, stored as a digest), and a pair whose codes would take 72 GiB comes back with a CIGAR that
re-scores to the oracle's score and end cell."""
import json
import os

import numpy as np
import pytest

import oracle
import synth
from helpers import rescore

pytestmark = pytest.mark.gpu
HERE = os.path.dirname(os.path.abspath(__file__))


@pytest.fixture
def small_budget():
    import paper_2002_04561_amd as aln
    aln.aln_set_traceback_budget(64 << 10)  # one tile row (1024 rows) per segment
    yield
    aln.aln_set_traceback_budget(0)


def _run_ls(q, s, mode, A, go, ge, match=None, mismatch=None, subst=None, linear=True):
    import torch

    import paper_2002_04561_amd as aln
    sc = aln.Scoring(mode, A, go, ge, match=match or 0, mismatch=mismatch or 0, subst=subst)
    qd = torch.from_numpy(np.ascontiguousarray(q, dtype=np.uint8) if len(q) else np.zeros(1, np.uint8)).cuda()
    sd = torch.from_numpy(np.ascontiguousarray(s, dtype=np.uint8) if len(s) else np.zeros(1, np.uint8)).cuda()
    # linear=False asks for a code per cell (ALN_STORED_CODES), which the library still refuses above 64 GiB
    flags = aln.TRACEBACK | (aln.LINEAR_SPACE if linear else aln.STORED_CODES)
    la = aln.LongAligner(sc, qd[:len(q)], sd[:len(s)], flags=flags)
    la.run()
    torch.cuda.synchronize()
    r = la.result()
    return (int(r["score"]), int(r["q_begin"]), int(r["q_end"]), int(r["s_begin"]), int(r["s_end"]),
            la.cigar_runs(), int(r["flags"]))


def _expect(q, s, sc):
    r = oracle.align(sc, q, s, traceback=True)
    return (r.score, r.q_begin, r.q_end, r.s_begin, r.s_end, r.cigar, 0)


def _related(rng, q, m, sub=0.08, indel=0.02, A=4):
    s = synth.mutate_geometric(rng, q, sub, indel, 3.0, A)[:m]
    if len(s) < m:
        s = np.concatenate([s, rng.integers(0, A, m - len(s), dtype=np.uint8)])
    return s


SHAPES = [(1, 1), (5, 3), (700, 64), (64, 700), (1000, 1100), (1025, 2049), (2100, 4500), (3000, 2100),
          (4097, 300), (300, 4500)]


@pytest.mark.parametrize("mode", [0, 1, 2], ids=["global", "local", "semi"])
@pytest.mark.parametrize("gap", [(0, -1), (-3, -1)], ids=["linear", "affine"])
def test_linear_space_shapes(gpu, small_budget, mode, gap):
    rng = np.random.default_rng(80 + mode)
    go, ge = gap
    sc = oracle.Scoring.simple(mode, 4, 2, -3, go, ge)
    for (n, m) in SHAPES:
        q = rng.integers(0, 4, n, dtype=np.uint8)
        s = _related(rng, q, m) if rng.random() < 0.7 else rng.integers(0, 4, m, dtype=np.uint8)
        print("mode %d gap %s n %d m %d" % (mode, gap, n, m), flush=True)
        got = _run_ls(q, s, mode, 4, go, ge, match=2, mismatch=-3)
        assert got == _expect(q, s, sc), (n, m)


@pytest.mark.parametrize("mode", [0, 1, 2], ids=["global", "local", "semi"])
@pytest.mark.parametrize("gap", [(0, -1), (-3, -1)], ids=["linear", "affine"])
def test_linear_space_window_fallback(gpu, small_budget, mode, gap):
    """A path that leaves its segment's window on the left: the subject is the 8192-letter query with 7,000
    unrelated letters inserted after its first 4096, so the alignment deletes them (with affine gaps in one
    horizontal gap on row 4096; the two halves score 2 x 12,288, more than the gap costs, in every mode).  The segment of
    rows 3073..4096 is relaxed again first only in a window of about 5,000 columns left of the walk; the
    walk stops at the window's edge inside the gap, the tiles left of it are relaxed again and the walk
    goes on.  Equal to the oracle's canonical traceback; and with 100 inserted letters, which stay in the
    window, too."""
    rng = np.random.default_rng(95 + mode)
    go, ge = gap
    sc = oracle.Scoring.simple(mode, 4, 3, -3, go, ge)
    for ins in (7000, 100):
        q = rng.integers(0, 4, 8192, dtype=np.uint8)
        s = np.concatenate([q[:4096], rng.integers(0, 4, ins, dtype=np.uint8), q[4096:]])
        print("mode %d gap %s insertion %d" % (mode, gap, ins), flush=True)
        got = _run_ls(q, s, mode, 4, go, ge, match=3, mismatch=-3)
        r = oracle.align(sc, q, s, traceback=True, impl="checkpointed")
        exp = (r.score, r.q_begin, r.q_end, r.s_begin, r.s_end, r.cigar, 0)
        assert got == exp, (ins, got[:5], exp[:5])
        if ins == 7000 and go < 0:
            # affine gaps: one deletion run carries the walk past the window's edge (linear gaps may spread
            # the deletions over many rows)
            assert max(L for L, op in exp[5] if op == 2) >= 6000, exp[5][:8]


@pytest.mark.parametrize("mode", [0, 1, 2], ids=["global", "local", "semi"])
def test_linear_space_gaps_across_boundaries(gpu, small_budget, mode):
    """Long gaps that cross a segment boundary (row 1024) and a tile column boundary (column 2048)."""
    rng = np.random.default_rng(90 + mode)
    sc = oracle.Scoring.simple(mode, 4, 2, -3, -3, -1)
    base = rng.integers(0, 4, 3000, dtype=np.uint8)
    extra = rng.integers(0, 4, 150, dtype=np.uint8)
    for at in (950, 2000):
        longer = np.concatenate([base[:at], extra, base[at:]])
        for q, s in ((longer, base), (base, longer)):
            print("mode %d gap at %d n %d m %d" % (mode, at, len(q), len(s)), flush=True)
            got = _run_ls(q, s, mode, 4, -3, -1, match=2, mismatch=-3)
            assert got == _expect(q, s, sc), (at, len(q), len(s))


def test_linear_space_protein(gpu, small_budget):
    rng = np.random.default_rng(91)
    sig = synth.protein_sigma(rng)
    for mode in (0, 1, 2):
        sc = oracle.Scoring.matrix(mode, sig.astype(np.int32), -11, -1)
        q = rng.integers(0, 20, 2500, dtype=np.uint8)
        s = _related(rng, q, 2300, 0.3, 0.02, 20)
        print("protein mode %d" % mode, flush=True)
        got = _run_ls(q, s, mode, 20, -11, -1, subst=sig)
        assert got == _expect(q, s, sc), mode


def test_linear_space_default_budget_one_segment(gpu):
    """With the default budget a 3000 x 2600 pair is one segment: the same CIGAR as the stored-code walk."""
    rng = np.random.default_rng(92)
    q = rng.integers(0, 4, 3000, dtype=np.uint8)
    s = _related(rng, q, 2600)
    a = _run_ls(q, s, 1, 4, -3, -1, 2, -3, linear=True)
    b = _run_ls(q, s, 1, 4, -3, -1, 2, -3, linear=False)
    assert a == b and a[6] == 0


@pytest.mark.parametrize("seed", range(12))
def test_linear_space_random_scheme(gpu, small_budget, seed):
    rng = np.random.default_rng(9700 + seed)
    A = int(rng.choice([2, 4, 5, 13, 20]))
    mode = int(rng.integers(0, 3))
    sub = match = mismatch = None
    if rng.random() < 0.6:
        t = rng.integers(-6, 3, (A, A))
        if rng.random() < 0.5:
            t = np.triu(t, 1)
            t = t + t.T
        np.fill_diagonal(t, rng.integers(1, 9, A))
        sub = t.astype(np.int8)
    else:
        match, mismatch = int(rng.integers(1, 6)), -int(rng.integers(1, 6))
    ge = -int(rng.integers(1, 4))
    go = 0 if rng.random() < 0.3 else -int(rng.integers(1, 12))
    sc = (oracle.Scoring.matrix(mode, sub.astype(np.int32), go, ge) if sub is not None else
          oracle.Scoring.simple(mode, A, match, mismatch, go, ge))
    n, m = int(rng.integers(1, 4200)), int(rng.integers(1, 4200))
    q = rng.integers(0, A, n, dtype=np.uint8)
    s = _related(rng, q, m, A=A) if rng.random() < 0.7 else rng.integers(0, A, m, dtype=np.uint8)
    label = "seed %d: A=%d mode=%d go=%d ge=%d table=%s n=%d m=%d" % (seed, A, mode, go, ge, sub is not None, n, m)
    print(label, flush=True)
    got = _run_ls(q, s, mode, A, go, ge, match=match, mismatch=mismatch, subst=sub)
    assert got == _expect(q, s, sc), label


@pytest.mark.slow
def test_linear_space_full_262144_equals_stored_codes(gpu):
    """The 262144 x 262144 local affine pair: the linear-space CIGAR, begin and end cells equal the stored-code
    walk's, the score and end cell the oracle's stored value, and the CIGAR re-scores to the score."""
    g = json.load(open(os.path.join(HERE, "golden", "long_local_262144.json")))
    w = synth.long_dna_local(seed=2, n=262144)
    a, b = w.pair(0)
    ls = _run_ls(a, b, 1, 4, -3, -1, 2, -3, linear=True)
    assert ls[6] == 0 and (ls[0], ls[2], ls[4]) == (g["score"], g["q_end"], g["s_end"])
    total, i, j = rescore(1, w.sigma_table(), -3, -1, a, b, ls[1], ls[3], ls[5])
    assert (total, i, j) == (ls[0], ls[2], ls[4])
    st = _run_ls(a, b, 1, 4, -3, -1, 2, -3, linear=False)
    assert st == ls
    _check_canonical(ls)


def _check_canonical(got):
    """The full-size canonical alignment from the oracle's linear-space traceback (stored as a digest)."""
    import hashlib
    path = os.path.join(HERE, "golden", "long_local_262144_cigar.json")
    if not os.path.exists(path):
        pytest.skip("canonical CIGAR of the full pair not generated")
    g = json.load(open(path))
    words = np.array([(L << 4) | op for L, op in got[5]], dtype="<u4")
    assert (got[0], got[1], got[2], got[3], got[4], len(got[5])) == (
        g["score"], g["q_begin"], g["q_end"], g["s_begin"], g["s_end"], g["cigar_len"])
    assert hashlib.sha256(words.tobytes()).hexdigest() == g["cigar_sha256"]


@pytest.mark.slow
def test_linear_space_beyond_64gib(gpu):
    """The 393216 x 393216 local affine pair, whose codes would take 72 GiB: traced back in linear space; score and
    end cell equal the oracle's stored value and the CIGAR re-scores to them."""
    path = os.path.join(HERE, "golden", "long_local_393216.json")
    if not os.path.exists(path):
        pytest.skip("golden value not generated")
    g = json.load(open(path))
    w = synth.long_dna_local(seed=2, n=393216)
    a, b = w.pair(0)
    got = _run_ls(a, b, 1, 4, -3, -1, 2, -3, linear=False)  # chosen by size
    assert got[6] == 0 and (got[0], got[2], got[4]) == (g["score"], g["q_end"], g["s_end"])
    total, i, j = rescore(1, w.sigma_table(), -3, -1, a, b, got[1], got[3], got[5])
    assert (total, i, j) == (got[0], got[2], got[4])
    assert 0 <= got[1] < got[2] and 0 <= got[3] < got[4]
