"""GPU parity of aln_align_long (one pair, band wavefront) against the oracle."""
import json
import os

import numpy as np
import pytest

import oracle
import synth

pytestmark = pytest.mark.gpu
HERE = os.path.dirname(os.path.abspath(__file__))


def _run(q, s, mode, A, go, ge, match=None, mismatch=None, subst=None):
    import torch

    import paper_2002_04561_amd as aln
    sc = aln.Scoring(mode, A, go, ge, match=match or 0, mismatch=mismatch or 0, subst=subst)
    qd = torch.from_numpy(np.ascontiguousarray(q, dtype=np.uint8) if len(q) else np.zeros(1, np.uint8)).cuda()
    sd = torch.from_numpy(np.ascontiguousarray(s, dtype=np.uint8) if len(s) else np.zeros(1, np.uint8)).cuda()
    la = aln.LongAligner(sc, qd[:len(q)], sd[:len(s)])
    la.run()
    torch.cuda.synchronize()
    r = la.result()
    return int(r["score"]), int(r["q_end"]), int(r["s_end"]), int(r["flags"])


def _oracle(q, s, mode, A, go, ge, match=None, mismatch=None, subst=None):
    if subst is not None:
        sc = oracle.Scoring.matrix(mode, subst.astype(np.int32), go, ge)
    else:
        sc = oracle.Scoring.simple(mode, A, match, mismatch, go, ge)
    r = oracle.align(sc, q, s, impl="linspace")
    return r.score, r.q_end, r.s_end, 0


SHAPES = [(1, 1), (5, 3), (63, 64), (64, 65), (255, 70), (256, 256), (257, 1000), (700, 40), (40, 700),
          (1000, 1300), (1536, 900), (2049, 2500)]


@pytest.mark.parametrize("mode", [0, 1, 2], ids=["global", "local", "semi"])
@pytest.mark.parametrize("gap", [(0, -1), (-3, -1)], ids=["linear", "affine"])
def test_long_dna_shapes(gpu, mode, gap):
    rng = np.random.default_rng(40 + mode)
    go, ge = gap
    for (n, m) in SHAPES:
        q = rng.integers(0, 4, n, dtype=np.uint8)
        s = synth.mutate_geometric(rng, q, 0.05, 0.01, 3.0)[:m] if rng.random() < 0.6 else \
            rng.integers(0, 4, m, dtype=np.uint8)
        if len(s) < m:
            s = np.concatenate([s, rng.integers(0, 4, m - len(s), dtype=np.uint8)])
        got = _run(q, s, mode, 4, go, ge, match=2, mismatch=-3)
        exp = _oracle(q, s, mode, 4, go, ge, match=2, mismatch=-3)
        assert got == exp, (n, m, got, exp)


@pytest.mark.parametrize("mode", [0, 1, 2], ids=["global", "local", "semi"])
def test_long_protein_table(gpu, mode):
    rng = np.random.default_rng(77)
    sig = synth.protein_sigma(rng)
    for (n, m) in [(300, 500), (1025, 777), (2000, 2100)]:
        q = rng.integers(0, 20, n, dtype=np.uint8)
        s = rng.integers(0, 20, m, dtype=np.uint8)
        got = _run(q, s, mode, 20, -11, -1, subst=sig)
        exp = _oracle(q, s, mode, 20, -11, -1, subst=sig)
        assert got == exp, (n, m, got, exp)


@pytest.mark.parametrize("gap", [(0, -4), (-5, -2)], ids=["linear", "affine"])
def test_long_local_ties_mid_band(gpu, gap):
    """Local optima that end inside a band's range-free steps, with ties: one window of the query (a segment
    and 60 letters either side) planted twice in an unrelated subject gives end cells of equal score in one
    row; the one with the smaller column must be reported (the tie rule), also where a band keeps a row's
    improving groups of steps and resolves them later."""
    rng = np.random.default_rng(4242)
    go, ge = gap
    F = 60
    for (n, m, L) in [(1000, 1500, 60), (2600, 2100, 90), (777, 3000, 40), (1300, 1300, 200)]:
        q = rng.integers(0, 4, n, dtype=np.uint8)
        s = rng.integers(0, 4, m, dtype=np.uint8)
        a = int(rng.integers(100 + F, n - L - 100 - F))
        b1 = int(rng.integers(100 + F, m // 2 - L - F))
        b2 = int(rng.integers(m // 2 + F, m - L - 100 - F))
        s[b1 - F:b1 + L + F] = q[a - F:a + L + F]
        s[b2 - F:b2 + L + F] = q[a - F:a + L + F]
        got = _run(q, s, 1, 4, go, ge, match=1, mismatch=-3)
        exp = _oracle(q, s, 1, 4, go, ge, match=1, mismatch=-3)
        assert got == exp, (n, m, L, got, exp)
        assert exp[2] < b2 - F, (n, m, exp)  # the first copy's end cell


def test_long_empty_and_bad(gpu):
    assert _run(np.zeros(0, np.uint8), np.array([1, 2], np.uint8), 0, 4, -3, -1, 2, -3)[:3] == (-5, 0, 2)
    assert _run(np.array([1, 2], np.uint8), np.zeros(0, np.uint8), 1, 4, -3, -1, 2, -3)[:3] == (0, 0, 0)
    got = _run(np.array([1, 7, 2], np.uint8), np.array([1, 2], np.uint8), 1, 4, -3, -1, 2, -3)
    assert got[3] & 4


def test_long_prefix_of_full_workload(gpu):
    """The first 8192 rows of the 262144 x 262144 workload against the oracle (same seeded input)."""
    w = synth.long_dna_local(seed=2, n=262144)
    a, b = w.pair(0)
    a = a[:8192]
    b = b[:20000]
    got = _run(a, b, 1, 4, -3, -1, 2, -3)
    exp = _oracle(a, b, 1, 4, -3, -1, 2, -3)
    assert got == exp


@pytest.mark.slow
def test_long_full_262144(gpu):
    """The full 262144 x 262144 local affine pair against the stored oracle value."""
    path = os.path.join(HERE, "golden", "long_local_262144.json")
    if not os.path.exists(path):
        pytest.skip("golden value not generated")
    g = json.load(open(path))
    w = synth.long_dna_local(seed=2, n=262144)
    a, b = w.pair(0)
    got = _run(a, b, 1, 4, -3, -1, 2, -3)
    assert got[:3] == (g["score"], g["q_end"], g["s_end"])


def _run_tb(q, s, mode, A, go, ge, match=None, mismatch=None, subst=None, cap=None):
    import torch

    import paper_2002_04561_amd as aln
    sc = aln.Scoring(mode, A, go, ge, match=match or 0, mismatch=mismatch or 0, subst=subst)
    qd = torch.from_numpy(np.ascontiguousarray(q, dtype=np.uint8) if len(q) else np.zeros(1, np.uint8)).cuda()
    sd = torch.from_numpy(np.ascontiguousarray(s, dtype=np.uint8) if len(s) else np.zeros(1, np.uint8)).cuda()
    # a code per cell at every size (the linear-space traceback has tests of its own)
    la = aln.LongAligner(sc, qd[:len(q)], sd[:len(s)], flags=aln.TRACEBACK | aln.STORED_CODES, cigar_capacity=cap)
    la.run()
    torch.cuda.synchronize()
    r = la.result()
    return (int(r["score"]), int(r["q_begin"]), int(r["q_end"]), int(r["s_begin"]), int(r["s_end"]),
            la.cigar_runs(), int(r["flags"]), int(r["cigar_len"]))


@pytest.mark.parametrize("mode", [0, 1, 2], ids=["global", "local", "semi"])
@pytest.mark.parametrize("gap", [(0, -1), (-3, -1)], ids=["linear", "affine"])
def test_long_traceback_shapes(gpu, mode, gap):
    rng = np.random.default_rng(60 + mode)
    go, ge = gap
    sc = oracle.Scoring.simple(mode, 4, 2, -3, go, ge)
    for (n, m) in [(1, 1), (5, 3), (64, 70), (255, 300), (257, 257), (700, 64), (1000, 1100)]:
        q = rng.integers(0, 4, n, dtype=np.uint8)
        s = synth.mutate_geometric(rng, q, 0.08, 0.02, 3.0)[:m]
        if len(s) < m:
            s = np.concatenate([s, rng.integers(0, 4, m - len(s), dtype=np.uint8)])
        got = _run_tb(q, s, mode, 4, go, ge, match=2, mismatch=-3)
        r = oracle.align(sc, q, s, traceback=True)
        assert got[:6] == (r.score, r.q_begin, r.q_end, r.s_begin, r.s_end, r.cigar), (n, m)


@pytest.mark.parametrize("mode", [0, 1, 2], ids=["global", "local", "semi"])
@pytest.mark.parametrize("where", ["inner", "leading", "trailing"])
def test_long_traceback_long_gaps(gpu, mode, where):
    """Gap runs longer than the 64 cells the traceback walk looks ahead and crossing its 128-cell windows:
    one side carries an extra stretch of 150 (or 70) letters, in the middle or at either end, so the
    optimal path takes a long deletion and a long insertion.  At the ends the runs reach row or column 1."""
    rng = np.random.default_rng(70 + mode)
    sc = oracle.Scoring.simple(mode, 4, 2, -3, -3, -1)
    base = rng.integers(0, 4, 600, dtype=np.uint8)
    extra = rng.integers(0, 4, 150 if where == "inner" else 70, dtype=np.uint8)
    if where == "inner":
        longer = np.concatenate([base[:200], extra, base[200:]])
    elif where == "leading":
        longer = np.concatenate([extra, base])
    else:
        longer = np.concatenate([base, extra])
    for q, s in ((base, longer), (longer, base)):
        got = _run_tb(q, s, mode, 4, -3, -1, match=2, mismatch=-3)
        r = oracle.align(sc, q, s, traceback=True)
        assert got[:6] == (r.score, r.q_begin, r.q_end, r.s_begin, r.s_end, r.cigar), (len(q), len(s))


def test_long_traceback_protein(gpu):
    rng = np.random.default_rng(61)
    sig = synth.protein_sigma(rng)
    for mode in (0, 1, 2):
        sc = oracle.Scoring.matrix(mode, sig.astype(np.int32), -11, -1)
        q = rng.integers(0, 20, 600, dtype=np.uint8)
        s = rng.integers(0, 20, 520, dtype=np.uint8)
        got = _run_tb(q, s, mode, 20, -11, -1, subst=sig)
        r = oracle.align(sc, q, s, traceback=True)
        assert got[:6] == (r.score, r.q_begin, r.q_end, r.s_begin, r.s_end, r.cigar), mode


def test_long_traceback_global_1k_golden(gpu):
    """The 1000 x 1000 global linear pair (+2/-1, gap -1) against the stored oracle CIGAR."""
    g = json.load(open(os.path.join(HERE, "golden", "global_1k.json")))
    w = synth.long_dna_global_1k(seed=1)
    a, b = w.pair(0)
    got = _run_tb(a, b, 0, 4, 0, -1, match=2, mismatch=-1)
    assert got[0] == g["score"] and oracle.cigar_string(got[5]) == g["cigar"]


def test_long_traceback_truncation(gpu):
    rng = np.random.default_rng(62)
    q = rng.integers(0, 4, 300, dtype=np.uint8)
    s = rng.integers(0, 4, 300, dtype=np.uint8)
    full = _run_tb(q, s, 0, 4, -3, -1, 2, -3)
    short = _run_tb(q, s, 0, 4, -3, -1, 2, -3, cap=2)
    assert full[7] > 2 and short[6] & 2 and short[7] == full[7]


@pytest.mark.slow
def test_long_traceback_full_262144(gpu):
    """Traceback of the full 262144 x 262144 local affine pair, with the 4-bit predecessor code of every cell held
    in HBM (about 34 GB): score and end cell equal the stored oracle value, and the CIGAR re-scores to exactly that
    score over q[q_begin:q_end] x s[s_begin:s_end]."""
    from helpers import rescore
    path = os.path.join(HERE, "golden", "long_local_262144.json")
    if not os.path.exists(path):
        pytest.skip("golden value not generated")
    g = json.load(open(path))
    w = synth.long_dna_local(seed=2, n=262144)
    a, b = w.pair(0)
    score, qb, qe, sb, se, runs, flags, clen = _run_tb(a, b, 1, 4, -3, -1, 2, -3)
    assert flags == 0 and (score, qe, se) == (g["score"], g["q_end"], g["s_end"])
    assert clen == len(runs) > 0 and 0 <= qb < qe and 0 <= sb < se
    total, i, j = rescore(1, w.sigma_table(), -3, -1, a, b, qb, sb, runs)
    assert (total, i, j) == (score, qe, se)


@pytest.mark.parametrize("seed", range(32))
def test_long_random_scheme(gpu, seed):
    """One pair per call under a randomly drawn scheme: 2 to 24 letters, a symmetric or asymmetric table or
    match/mismatch, linear or affine gaps, any mode, score-only or with the CIGAR, lengths 1..2600 (often a
    mutated copy with long indels).  Score and end cell, and with a CIGAR the begin cell and every run, must
    equal the oracle."""
    rng = np.random.default_rng(9500 + seed)
    A = int(rng.choice([2, 3, 4, 5, 8, 13, 20, 24]))
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
    n, m = int(rng.integers(1, 2600)), int(rng.integers(1, 2600))
    q = rng.integers(0, A, n, dtype=np.uint8)
    if rng.random() < 0.7:
        s = synth.mutate_geometric(rng, q, 0.08, 0.02, 6.0, A)[:m]
        if len(s) < m:
            s = np.concatenate([s, rng.integers(0, A, m - len(s), dtype=np.uint8)])
    else:
        s = rng.integers(0, A, m, dtype=np.uint8)
    tb = bool(rng.random() < 0.6)
    label = "seed %d: A=%d mode=%d go=%d ge=%d table=%s n=%d m=%d tb=%s" % (
        seed, A, mode, go, ge, sub is not None, n, m, tb)
    print(label, flush=True)
    if tb:
        got = _run_tb(q, s, mode, A, go, ge, match=match, mismatch=mismatch, subst=sub)
        r = oracle.align(sc, q, s, traceback=True)
        assert got[:6] == (r.score, r.q_begin, r.q_end, r.s_begin, r.s_end, r.cigar), label
        assert got[6] == 0, label
    else:
        got = _run(q, s, mode, A, go, ge, match=match, mismatch=mismatch, subst=sub)
        r = oracle.align(sc, q, s, impl="linspace")
        assert got == (r.score, r.q_end, r.s_end, 0), label
