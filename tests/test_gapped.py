"""aln_cigar_to_gapped (host only): the gapped-string form of an alignment (Sec. III-C of the paper
returns the alignment as two gapped strings).  Pinned without the library's own arithmetic: the strings
with their gaps removed are the aligned parts of the two sequences, and re-adding their columns (a
letter pair scores sigma, each maximal gap run in one string scores go + k*ge) gives the oracle's
score."""
import numpy as np
import pytest

import oracle
import paper_2002_04561_amd as aln
import synth

LET = "ACGTNRYKMSWBDHVEFILP"


def _column_score(qa, sa, sigma, go, ge):
    total, k = 0, 0
    while k < len(qa):
        if qa[k] == "-" or sa[k] == "-":
            which = 0 if qa[k] == "-" else 1
            run = 0
            while k < len(qa) and (qa[k] == "-" if which == 0 else sa[k] == "-"):
                run += 1
                k += 1
            total += go + run * ge
        else:
            total += int(sigma[LET.index(qa[k])][LET.index(sa[k])])
            k += 1
    return total


@pytest.mark.parametrize("mode", [synth.GLOBAL, synth.LOCAL, synth.SEMIGLOBAL])
@pytest.mark.parametrize("alpha,go,ge", [(4, 0, -1), (4, -3, -1), (20, -11, -1)])
def test_gapped_strings_rescore(mode, alpha, go, ge):
    rng = np.random.default_rng(7 + mode + alpha)
    subst = synth.protein_sigma(rng)[:alpha, :alpha] if alpha == 20 else None
    w = synth.random_pairs(11 + mode, 24, 0, 60, alpha, mode, go, ge, match=2, mismatch=-3, subst=subst, related=0.6)
    sigma = w.sigma_table()
    sc = oracle.Scoring.matrix(mode, sigma, go, ge)
    for k in range(w.n_pairs):
        a, b = w.pair(k)
        r = oracle.align(sc, a, b, traceback=True)
        rec = {"q_begin": r.q_begin, "s_begin": r.s_begin}
        qa, sa = aln.aln_cigar_to_gapped(a, b, rec, r.cigar, LET)
        assert len(qa) == len(sa) == sum(L for L, _ in r.cigar)
        assert qa.replace("-", "") == "".join(LET[c] for c in a[r.q_begin:r.q_end])
        assert sa.replace("-", "") == "".join(LET[c] for c in b[r.s_begin:r.s_end])
        assert not any(x == "-" and y == "-" for x, y in zip(qa, sa))
        assert _column_score(qa, sa, sigma, go, ge) == r.score


def test_paper_scheme_example():
    """ACGT against AGT, global, +2/-1, linear gap -1: score 5, one letter of the query against a gap."""
    a = np.array([0, 1, 2, 3], np.uint8)
    b = np.array([0, 2, 3], np.uint8)
    sc = oracle.Scoring.simple(synth.GLOBAL, 4, 2, -1, 0, -1)
    r = oracle.align(sc, a, b, traceback=True)
    qa, sa = aln.aln_cigar_to_gapped(a, b, {"q_begin": r.q_begin, "s_begin": r.s_begin}, r.cigar, "ACGT")
    assert (r.score, qa, sa) == (5, "ACGT", "A-GT")


def test_gapped_rejects_bad_input():
    a = np.array([0, 1, 2], np.uint8)
    b = np.array([0, 1], np.uint8)
    with pytest.raises(aln.AlnError):  # the CIGAR runs past the subject
        aln.aln_cigar_to_gapped(a, b, {"q_begin": 0, "s_begin": 0}, [(3, 0)], "ACGT")
    with pytest.raises(aln.AlnError):  # an op outside M/I/D
        aln.aln_cigar_to_gapped(a, b, {"q_begin": 0, "s_begin": 0}, [(1, 5)], "ACGT")
    with pytest.raises(aln.AlnError):  # a score-only result has no begin cell
        aln.aln_cigar_to_gapped(a, b, {"q_begin": -1, "s_begin": -1}, [], "ACGT")
    qa, sa = aln.aln_cigar_to_gapped(a, b, {"q_begin": 0, "s_begin": 0}, [(1, 0), (1, 1), (1, 0)], None)
    assert (qa, sa) == ("ABC", "A-B")
