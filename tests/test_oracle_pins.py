"""Pins of the oracle against what the paper and the mathematics fix (CPU only).

* brute-force enumeration of every alignment (oracle/brute.py) for lengths <= 6: score, end cell,
  begin cell and canonical CIGAR, every mode x gap model, alphabets 2 / 4 / 20, symmetric and
  asymmetric substitution tables;
* closed forms, textbook reductions (LCS, Levenshtein) written as separate one-line recurrences;
* invariants: swap and reversal symmetry, local >= semi-global >= global, local >= 0, rescoring of
  every CIGAR, linear == affine with go = 0 (including the CIGAR), two-row == full-matrix results.
"""
import functools
import itertools

import numpy as np
import pytest

import oracle
from helpers import rescore
from oracle.brute import brute_align

MODES = [oracle.GLOBAL, oracle.LOCAL, oracle.SEMIGLOBAL]


def _cases(seed, count, maxlen, alphabets=(2, 4, 20)):
    rng = np.random.default_rng(seed)
    for _ in range(count):
        A = int(rng.choice(alphabets))
        mode = int(rng.integers(0, 3))
        n, m = int(rng.integers(0, maxlen + 1)), int(rng.integers(0, maxlen + 1))
        q = rng.integers(0, A, n)
        s = rng.integers(0, A, m)
        sig = rng.integers(-4, 5, (A, A)).astype(np.int32)
        if rng.random() < 0.5:
            sig = np.triu(sig) + np.triu(sig, 1).T
        go = int(rng.integers(-4, 1))
        ge = int(rng.integers(-3, 0))
        yield mode, A, sig, go, ge, q, s


@pytest.mark.parametrize("seed", range(6))
def test_oracle_equals_brute_force(seed):
    for mode, A, sig, go, ge, q, s in _cases(seed, 250, 6):
        sc = oracle.Scoring.matrix(mode, sig, go, ge)
        r = oracle.align(sc, q, s, traceback=True)
        b = brute_align(mode, sig, go, ge, q, s)
        got = (r.score, r.q_begin, r.q_end, r.s_begin, r.s_end, r.cigar)
        exp = (b.score, b.q_begin, b.q_end, b.s_begin, b.s_end, b.cigar)
        assert got == exp, (mode, go, ge, list(q), list(s), sig.tolist())
        ls = oracle.align(sc, q, s, impl="linspace")
        assert (ls.score, ls.q_end, ls.s_end) == (b.score, b.q_end, b.s_end)
        if go == 0:
            lin = oracle.align(sc, q, s, traceback=True, impl="linear")
            assert (lin.score, lin.q_begin, lin.q_end, lin.s_begin, lin.s_end, lin.cigar) == exp


def test_brute_force_plants_detected():
    """A planted mistake in the oracle's recurrence must be caught by the brute-force pin: a copy of the
    scoring with a flipped gap sign, or a dropped open cost, gives different optima."""
    q, s = [0, 1, 1, 0, 1], [0, 0, 1, 1]
    sig = np.array([[2, -1], [-1, 2]], np.int32)
    b = brute_align(oracle.GLOBAL, sig, -3, -1, q, s)
    wrong = oracle.align(oracle.Scoring.matrix(oracle.GLOBAL, sig, 0, -1), q, s)  # go dropped
    assert wrong.score != b.score
    right = oracle.align(oracle.Scoring.matrix(oracle.GLOBAL, sig, -3, -1), q, s)
    assert right.score == b.score


def test_paper_example_scheme_hand_worked():
    """The scheme of the C example in Sec. III-C (+2/-1, linear gap -1), worked by hand:
    ACGT vs AGT: A-A (+2), C-gap (-1), G-G (+2), T-T (+2) = 5, CIGAR 1M1I2M."""
    sc = oracle.Scoring.simple(oracle.GLOBAL, 4, 2, -1, 0, -1)
    r = oracle.align(sc, [0, 1, 2, 3], [0, 2, 3], traceback=True)
    assert r.score == 5 and oracle.cigar_string(r.cigar) == "1M1I2M"


def test_closed_forms():
    rng = np.random.default_rng(7)
    for go, ge in [(0, -1), (-3, -1), (-11, -1), (-5, -2)]:
        for k in range(1, 9):
            a = rng.integers(0, 4, k)
            sc = oracle.Scoring.simple(oracle.GLOBAL, 4, 2, -3, go, ge)
            # global against the empty sequence: one gap of length k
            assert oracle.align(sc, a, []).score == go + k * ge
            assert oracle.align(sc, [], a).score == go + k * ge
            r = oracle.align(sc, a, [], traceback=True)
            assert r.cigar == [(k, oracle.OP_I)]
        sc = oracle.Scoring.simple(oracle.GLOBAL, 4, 2, -3, go, ge)
        assert oracle.align(sc, [], []).score == 0
    # identical sequences: global = local = n * match
    for n in (1, 5, 40, 200):
        a = rng.integers(0, 4, n)
        for mode in (oracle.GLOBAL, oracle.LOCAL):
            sc = oracle.Scoring.simple(mode, 4, 3, -2, -4, -1)
            r = oracle.align(sc, a, a, traceback=True)
            assert r.score == 3 * n and r.cigar == [(n, oracle.OP_M)]
    # semi-global with the read an exact substring of the window
    for L, pad in [(10, 5), (50, 30), (120, 64)]:
        win = rng.integers(0, 4, L + pad)
        o = int(rng.integers(0, pad + 1))
        read = win[o:o + L]
        sc = oracle.Scoring.simple(oracle.SEMIGLOBAL, 4, 1, -4, -5, -2)
        r = oracle.align(sc, read, win, traceback=True)
        assert r.score == L and r.s_end - r.s_begin == L and r.q_begin == 0 and r.q_end == L


@functools.lru_cache(maxsize=None)
def _lcs(a, b):
    if not a or not b:
        return 0
    if a[-1] == b[-1]:
        return _lcs(a[:-1], b[:-1]) + 1
    return max(_lcs(a[:-1], b), _lcs(a, b[:-1]))


@functools.lru_cache(maxsize=None)
def _lev(a, b):
    if not a:
        return len(b)
    if not b:
        return len(a)
    return min(_lev(a[:-1], b) + 1, _lev(a, b[:-1]) + 1, _lev(a[:-1], b[:-1]) + (a[-1] != b[-1]))


def test_textbook_reductions():
    """Global, linear gap, (1, 0, 0) is the LCS length; (0, -1, -1) is minus the Levenshtein distance.
    (gap_extend = 0 is outside the library's domain but fine for the oracle's arithmetic.)"""
    rng = np.random.default_rng(3)
    for _ in range(200):
        n, m = int(rng.integers(0, 12)), int(rng.integers(0, 12))
        a = tuple(int(x) for x in rng.integers(0, 3, n))
        b = tuple(int(x) for x in rng.integers(0, 3, m))
        lcs = oracle.Scoring.simple(oracle.GLOBAL, 3, 1, 0, 0, 0)
        assert oracle.align(lcs, a, b).score == _lcs(a, b)
        assert oracle.align(lcs, a, b, impl="linear").score == _lcs(a, b)
        lev = oracle.Scoring.simple(oracle.GLOBAL, 3, 0, -1, 0, -1)
        assert oracle.align(lev, a, b).score == -_lev(a, b)


def test_invariants_random():
    rng = np.random.default_rng(12)
    for t in range(300):
        A = int(rng.choice([4, 20]))
        n, m = int(rng.integers(0, 60)), int(rng.integers(0, 60))
        q, s = rng.integers(0, A, n), rng.integers(0, A, m)
        sig = rng.integers(-5, 6, (A, A)).astype(np.int32)
        sig = np.triu(sig) + np.triu(sig, 1).T  # symmetric
        go, ge = int(rng.integers(-6, 1)), int(rng.integers(-3, 0))
        scores = {}
        for mode in MODES:
            sc = oracle.Scoring.matrix(mode, sig, go, ge)
            r = oracle.align(sc, q, s, traceback=True)
            scores[mode] = r.score
            # swap symmetry for a symmetric table
            assert oracle.align(sc, s, q).score == r.score
            # reversal symmetry
            assert oracle.align(sc, q[::-1], s[::-1]).score == r.score
            # rescoring the CIGAR reproduces the score and lands on the end cell
            tot, ie, je = rescore(mode, sig, go, ge, q, s, r.q_begin, r.s_begin, r.cigar)
            assert (tot, ie, je) == (r.score, r.q_end, r.s_end)
            if mode == oracle.GLOBAL:
                assert (r.q_begin, r.s_begin, r.q_end, r.s_end) == (0, 0, n, m)
            if mode == oracle.SEMIGLOBAL:
                assert r.q_begin == 0 or r.s_begin == 0
                assert r.q_end == n or r.s_end == m
            # two-row score-only agrees with full matrices
            ls = oracle.align(sc, q, s, impl="linspace")
            assert (ls.score, ls.q_end, ls.s_end) == (r.score, r.q_end, r.s_end)
            if go == 0:
                lin = oracle.align(sc, q, s, traceback=True, impl="linear")
                assert (lin.score, lin.q_begin, lin.q_end, lin.s_begin, lin.s_end, lin.cigar) == \
                       (r.score, r.q_begin, r.q_end, r.s_begin, r.s_end, r.cigar)
        assert scores[oracle.LOCAL] >= 0
        assert scores[oracle.LOCAL] >= scores[oracle.SEMIGLOBAL] >= scores[oracle.GLOBAL]


def test_local_zero_for_disjoint_alphabets():
    sig = -np.ones((4, 4), np.int32)
    np.fill_diagonal(sig, 3)
    sc = oracle.Scoring.matrix(oracle.LOCAL, sig, -2, -1)
    r = oracle.align(sc, [0, 1, 0, 1, 1], [2, 3, 3, 2], traceback=True)
    assert (r.score, r.q_begin, r.q_end, r.s_begin, r.s_end, r.cigar) == (0, 0, 0, 0, 0, [])


def test_linear_affine0_identity_exhaustive_small():
    """linear(g) and affine(0, g) give the same score, coordinates and CIGAR on every binary pair up to length 4."""
    seqs = [t for L in range(5) for t in itertools.product([0, 1], repeat=L)]
    for mode in MODES:
        sc = oracle.Scoring.simple(mode, 2, 1, -1, 0, -1)
        for a in seqs:
            for b in seqs:
                x = oracle.align(sc, a, b, traceback=True)
                y = oracle.align(sc, a, b, traceback=True, impl="linear")
                assert (x.score, x.q_begin, x.q_end, x.s_begin, x.s_end, x.cigar) == \
                       (y.score, y.q_begin, y.q_end, y.s_begin, y.s_end, y.cigar)


def test_batch_driver_matches_single():
    import synth
    w = synth.random_pairs(9, 60, 0, 80, 4, oracle.LOCAL, -3, -1, match=2, mismatch=-3, related=0.5)
    sc = oracle.Scoring.matrix(w.mode, w.sigma_table(), w.gap_open, w.gap_extend)
    res, cig, coff = oracle.align_batch(sc, w.q, w.q_off, w.s, w.s_off, traceback=True, threads=3)
    for k in range(w.n_pairs):
        a, b = w.pair(k)
        r = oracle.align(sc, a, b, traceback=True)
        assert (res["score"][k], res["q_begin"][k], res["q_end"][k]) == (r.score, r.q_begin, r.q_end)
        got = [(int(x) >> 4, int(x) & 15) for x in cig[coff[k]:coff[k] + res["cigar_len"][k]]]
        assert got == r.cigar


@pytest.mark.parametrize("seed", range(3))
def test_checkpointed_traceback_equals_brute_force(seed):
    """The oracle's linear-space traceback (kept rows every K rows, one block recomputed at a time) against
    the brute-force enumeration, with blocks of 1, 2 and 3 rows, so walks cross block boundaries in every
    state."""
    for mode, A, sig, go, ge, q, s in _cases(100 + seed, 200, 6):
        sc = oracle.Scoring.matrix(mode, sig, go, ge)
        b = brute_align(mode, sig, go, ge, q, s)
        for K in (1, 2, 3):
            r = oracle.align(sc, q, s, traceback=True, impl="checkpointed", block_rows=K)
            assert (r.score, r.q_begin, r.q_end, r.s_begin, r.s_end, r.cigar) == (
                b.score, b.q_begin, b.q_end, b.s_begin, b.s_end, b.cigar), (K, mode, go, ge, list(q), list(s))


def test_checkpointed_traceback_equals_full_matrices():
    """Larger related pairs (up to 400 letters, long gaps) against the full-matrix traceback, every mode and
    gap model, block heights from 1 row to more than the pair."""
    import synth
    rng = np.random.default_rng(11)
    for trial in range(60):
        mode = MODES[trial % 3]
        A = int(rng.choice([4, 20]))
        go, ge = (0, -1) if trial % 4 == 0 else (-int(rng.integers(1, 12)), -int(rng.integers(1, 3)))
        sig = rng.integers(-4, 3, (A, A)).astype(np.int32)
        np.fill_diagonal(sig, rng.integers(2, 9, A))
        sc = oracle.Scoring.matrix(mode, sig, go, ge)
        n = int(rng.integers(0, 400))
        q = rng.integers(0, A, n, dtype=np.uint8)
        s = synth.mutate_geometric(rng, q, 0.1, 0.03, 6.0, A)[:int(rng.integers(0, 400))] if n else \
            rng.integers(0, A, int(rng.integers(0, 50)), dtype=np.uint8)
        f = oracle.align(sc, q, s, traceback=True)
        for K in (1, 5, 64, 1000):
            r = oracle.align(sc, q, s, traceback=True, impl="checkpointed", block_rows=K)
            assert (r.score, r.q_begin, r.q_end, r.s_begin, r.s_end, r.cigar) == (
                f.score, f.q_begin, f.q_end, f.s_begin, f.s_end, f.cigar), (trial, K)
