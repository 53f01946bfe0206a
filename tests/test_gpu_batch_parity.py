"""GPU parity of aln_align_batch against the oracle: bit-exact scores, end cells, begin cells and CIGARs."""
import itertools

import numpy as np
import pytest

import synth
from helpers import compare, run_gpu, run_oracle

pytestmark = pytest.mark.gpu

PROT = synth.protein_sigma(np.random.default_rng(11))


def _mid_sigma(rng):
    """A symmetric 8-letter table (diagonal +3..+6, off-diagonal -4..+1): alphabets of 5..12 letters take the
    16-bit kernel's 8-row strips."""
    t = np.triu(rng.integers(-4, 2, (8, 8)), 1)
    t = t + t.T
    np.fill_diagonal(t, rng.integers(3, 7, 8))
    return t.astype(np.int8)


MID = _mid_sigma(np.random.default_rng(12))

SCHEMES = {
    # name: (alphabet, match, mismatch, subst, gap_open, gap_extend)
    "dna_linear": (4, 2, -1, None, 0, -1),
    "dna_affine": (4, 1, -4, None, -5, -2),
    "prot_affine": (20, None, None, PROT, -11, -1),
    "prot_linear": (20, None, None, PROT, 0, -4),
    "mid8_affine": (8, None, None, MID, -6, -1),
}


def _workload(seed, n_pairs, nmin, nmax, mode, scheme, related=0.5, mmin=None, mmax=None):
    A, ma, mi, sub, go, ge = SCHEMES[scheme]
    return synth.random_pairs(seed, n_pairs, nmin, nmax, A, mode, go, ge, match=ma, mismatch=mi, subst=sub,
                              related=related, mmin=mmin, mmax=mmax)


@pytest.mark.parametrize("mode", [0, 1, 2], ids=["global", "local", "semi"])
@pytest.mark.parametrize("scheme", list(SCHEMES))
@pytest.mark.parametrize("tb", [False, True], ids=["score", "traceback"])
def test_random_ragged(gpu, mode, scheme, tb):
    import paper_2002_04561_amd as aln
    w = _workload(100 + mode * 10 + len(scheme), 150, 0, 300, mode, scheme)
    flags = aln.TRACEBACK if tb else aln.SCORE_ONLY
    gres, gcig = run_gpu(w, flags)
    ores, ocig = run_oracle(w, tb)
    bad = compare(w, gres, gcig, ores, ocig, "%d/%s/%s" % (mode, scheme, tb))
    assert not bad, "\n".join(bad[:10])


@pytest.mark.parametrize("mode", [0, 1, 2], ids=["global", "local", "semi"])
@pytest.mark.parametrize("go", [0, -2])
def test_exhaustive_binary(gpu, mode, go):
    """All pairs of binary sequences of length 0..4 (31 x 31 pairs) -- ties everywhere."""
    import paper_2002_04561_amd as aln
    seqs = [np.array(t, dtype=np.uint8) for L in range(5) for t in itertools.product([0, 1], repeat=L)]
    qs = [a for a in seqs for _ in seqs]
    ss = [b for _ in seqs for b in seqs]
    q, qo = synth.pack(qs)
    s, so = synth.pack(ss)
    w = synth.Workload("binary", mode, 2, go, -1, q, qo, s, so, match=1, mismatch=-1)
    gres, gcig = run_gpu(w, aln.TRACEBACK)
    ores, ocig = run_oracle(w, True)
    bad = compare(w, gres, gcig, ores, ocig, "binary")
    assert not bad, "\n".join(bad[:10])


@pytest.mark.parametrize("mode", [0, 1, 2], ids=["global", "local", "semi"])
def test_edge_shapes(gpu, mode):
    import paper_2002_04561_amd as aln
    rng = np.random.default_rng(5)
    shapes = [(0, 0), (0, 5), (5, 0), (1, 1), (1, 2000), (2000, 1), (7, 900), (900, 7), (64, 64), (65, 63),
              (8, 8), (9, 8), (16, 1), (1, 16)]
    qs = [rng.integers(0, 4, a, dtype=np.uint8) for a, _ in shapes]
    ss = [rng.integers(0, 4, b, dtype=np.uint8) for _, b in shapes]
    q, qo = synth.pack(qs)
    s, so = synth.pack(ss)
    w = synth.Workload("edges", mode, 4, -3, -1, q, qo, s, so, match=2, mismatch=-3)
    for flags in (aln.SCORE_ONLY, aln.TRACEBACK):
        gres, gcig = run_gpu(w, flags)
        ores, ocig = run_oracle(w, bool(flags))
        bad = compare(w, gres, gcig, ores, ocig, "edges")
        assert not bad, "\n".join(bad[:10])


def test_bad_codes_flagged(gpu):
    import paper_2002_04561_amd as aln
    qs = [np.array([0, 1, 2, 3], np.uint8), np.array([0, 1, 9, 3], np.uint8), np.array([1, 1], np.uint8)]
    ss = [np.array([0, 1, 2], np.uint8), np.array([0, 1], np.uint8), np.array([1, 200], np.uint8)]
    q, qo = synth.pack(qs)
    s, so = synth.pack(ss)
    w = synth.Workload("bad", 1, 4, -3, -1, q, qo, s, so, match=2, mismatch=-3)
    gres, gcig = run_gpu(w, aln.TRACEBACK)
    assert int(gres["flags"][0]) & aln.RES_BAD_CODE == 0
    assert int(gres["flags"][1]) & aln.RES_BAD_CODE
    assert int(gres["flags"][2]) & aln.RES_BAD_CODE
    ores, ocig = run_oracle(w, True)
    bad = compare(w, gres, gcig, ores, ocig, "bad")
    assert not bad, "\n".join(bad)


@pytest.mark.parametrize("mode", [0, 1, 2], ids=["global", "local", "semi"])
@pytest.mark.parametrize("scheme", ["prot_affine", "dna_affine", "dna_linear"])
def test_uneven_split_score_only(gpu, mode, scheme):
    """Log-uniform lengths 64..3000: pairs with n*m >= 2^20 take the band wavefront, the rest one lane each."""
    import paper_2002_04561_amd as aln
    A, ma, mi, sub, go, ge = SCHEMES[scheme]
    rng = np.random.default_rng(300 + mode)
    lens = np.rint(np.exp(rng.uniform(np.log(64), np.log(3000), (120, 2)))).astype(int)
    qs = [rng.integers(0, A, a, dtype=np.uint8) for a, _ in lens]
    ss = [synth.mutate_geometric(rng, qs[k], 0.1, 0.02, 2.0, A)[:b] if k % 3 == 0 else
          rng.integers(0, A, b, dtype=np.uint8) for k, (_, b) in enumerate(lens)]
    q, qo = synth.pack(qs)
    s, so = synth.pack(ss)
    w = synth.Workload("uneven", mode, A, go, ge, q, qo, s, so, match=ma, mismatch=mi, subst=sub)
    n, m = w.lengths()
    assert np.any(n * m >= (1 << 20)) and np.any(n * m < (1 << 20))
    gres, _ = run_gpu(w, aln.SCORE_ONLY, config=aln.BatchConfig(wf_min_cells=1 << 20))
    ores, _ = run_oracle(w, False)
    bad = compare(w, gres, None, ores, None, "uneven")
    assert not bad, "\n".join(bad[:10])


@pytest.mark.parametrize("mode", [0, 1, 2], ids=["global", "local", "semi"])
@pytest.mark.parametrize("tb", [False, True], ids=["score", "traceback"])
def test_overflow_redo(gpu, mode, tb):
    """Pairs whose scores leave the 16-bit range: identical 300-letter pairs at match +120 (36000 > 32767), mixed
    with ordinary pairs.  Local pairs run in 16 bits under ALN_FORCE_INT16, saturate and are redone; every pair
    must come back bit-exact, and exactly the big-score pairs carry ALN_RES_INT32_REDO."""
    import paper_2002_04561_amd as aln
    rng = np.random.default_rng(9 + mode)
    qs, ss, hot = [], [], []
    for k in range(200):
        if k % 7 == 0:
            a = rng.integers(0, 4, 300, dtype=np.uint8)
            qs.append(a)
            ss.append(a.copy())
            hot.append(True)
        else:
            qs.append(rng.integers(0, 4, int(rng.integers(0, 280)), dtype=np.uint8))
            ss.append(rng.integers(0, 4, int(rng.integers(0, 280)), dtype=np.uint8))
            hot.append(False)
    q, qo = synth.pack(qs)
    s, so = synth.pack(ss)
    w = synth.Workload("overflow", mode, 4, -30, -20, q, qo, s, so, match=120, mismatch=-40)
    ores, ocig = run_oracle(w, tb)
    lanes_only = aln.BatchConfig(wf_min_cells=-1)  # every pair on the one-pair-per-lane kernels
    for extra in (0, aln.FORCE_INT16):
        flags = (aln.TRACEBACK if tb else aln.SCORE_ONLY) | extra
        gres, gcig = run_gpu(w, flags, config=lanes_only)
        bad = compare(w, gres, gcig, ores, ocig, "overflow")
        assert not bad, "\n".join(bad[:10])
        redo = (gres["flags"] & aln.RES_INT32_REDO) != 0
        assert np.all(redo[np.array(hot)]), "big-score pairs must be recomputed in 32 bits"
        assert int(np.sum(ores["score"][np.array(hot)] > 32767)) == int(np.sum(hot))


@pytest.mark.parametrize("mode", [0, 1, 2], ids=["global", "local", "semi"])
@pytest.mark.parametrize("scheme", ["dna_affine", "prot_affine", "dna_linear"])
def test_int16_equals_int32(gpu, mode, scheme):
    """The packed 16-bit path and ALN_FORCE_INT32 give identical results (scores, ends, CIGARs)."""
    import paper_2002_04561_amd as aln
    w = _workload(500 + mode, 300, 0, 260, mode, scheme)
    a, ac = run_gpu(w, aln.TRACEBACK)
    b, bc = run_gpu(w, aln.TRACEBACK | aln.FORCE_INT32)
    for k in range(w.n_pairs):
        assert tuple(a[k])[:6] == tuple(b[k])[:6] and ac[k] == bc[k], k
    assert not np.any(a["flags"] & aln.RES_INT32_REDO)


ASYM3 = np.array([[2, -1, -3], [0, 1, -2], [-2, 3, 1]], dtype=np.int8)  # sigma(q, s) != sigma(s, q)
WF_SCHEMES = {
    # register profile (alphabet <= 4), asymmetric table, ties likely
    "asym3_affine": (3, None, None, ASYM3, -2, -1),
    # per-lane LDS profile (alphabet 20)
    "prot_affine": SCHEMES["prot_affine"],
    "prot_linear": SCHEMES["prot_linear"],
    # sigma - ge beyond a signed byte: the 32-bit LDS table
    "dna_bigscore": (4, 100, -60, None, -50, -30),
}


@pytest.mark.parametrize("mode", [0, 1, 2], ids=["global", "local", "semi"])
@pytest.mark.parametrize("scheme", list(WF_SCHEMES))
@pytest.mark.parametrize("orient", [1, -1, 2], ids=["oriented", "as_given", "cheaper"])
@pytest.mark.parametrize("group", [1, 4, 416], ids=["alone", "grouped", "grouped_packed16"])
def test_wavefront_every_pair(gpu, mode, scheme, orient, group):
    """Every non-empty pair on the band wavefront (wf_min_cells = 1), lengths log-uniform 1..1500 in both
    directions, so that pairs run transposed (orient = 1, the longer sequence along the rows) or as given;
    results must not depend on it, ties included."""
    import paper_2002_04561_amd as aln
    A, ma, mi, sub, go, ge = WF_SCHEMES[scheme]
    rng = np.random.default_rng(700 + 10 * mode + len(scheme) + (orient > 0))
    lens = np.rint(np.exp(rng.uniform(0, np.log(1500), (90, 2)))).astype(int)
    lens[:6] = [(1, 1), (1, 700), (700, 1), (0, 40), (40, 0), (257, 1300)]
    qs = [rng.integers(0, A, a, dtype=np.uint8) for a, _ in lens]
    ss = [synth.mutate_geometric(rng, qs[k], 0.1, 0.02, 2.0, A)[:b] if k % 2 == 0 and b <= len(qs[k]) else
          rng.integers(0, A, b, dtype=np.uint8) for k, (_, b) in enumerate(lens)]
    q, qo = synth.pack(qs)
    s, so = synth.pack(ss)
    w = synth.Workload("wf_" + scheme, mode, A, go, ge, q, qo, s, so, match=ma, mismatch=mi, subst=sub)
    if group == 416 and mode != 1:
        pytest.skip("packed 16-bit bands are local-only")
    cfg = aln.BatchConfig(wf_min_cells=1, wf_orient=orient, wf_group=4 if group == 416 else group,
                          wf_bits=16 if group == 416 else 32)
    gres, _ = run_gpu(w, aln.SCORE_ONLY, config=cfg)
    ores, _ = run_oracle(w, False)
    bad = compare(w, gres, None, ores, None, "wf/%s/%d" % (scheme, orient))
    assert not bad, "\n".join(bad[:10])


@pytest.mark.parametrize("go", [0, -3], ids=["linear", "affine"])
@pytest.mark.parametrize("orient", [1, -1], ids=["oriented", "as_given"])
@pytest.mark.parametrize("group", [1, 4, 416], ids=["alone", "grouped", "grouped_packed16"])
@pytest.mark.parametrize("tb", [False, True], ids=["score", "traceback"])
def test_wavefront_local_ties_across_bands(gpu, go, orient, group, tb):
    """Local optima that tie across band boundaries (bands of 256 rows).  Runs of one letter score
    H(i, j) = 2 min(i, j), so a whole column or row of cells reaches the optimum; periodic sequences tie
    on every third diagonal; a shared prefix puts the optimum on or just below a band's last row.  A band
    only records cells that reach the largest score the band above hands down, so these pin that the
    first optimum in (score, i, j) order still comes back, transposed or not."""
    import paper_2002_04561_amd as aln
    rng = np.random.default_rng(4100 + 10 * group + (orient > 0) + (go != 0) * 2 + tb * 4)
    run = lambda k: np.zeros(k, dtype=np.uint8)
    per = lambda k: np.resize(np.array([0, 1, 2], dtype=np.uint8), k)
    rnd = lambda k: rng.integers(0, 4, k, dtype=np.uint8)
    pairs = [(run(700), run(300)), (run(300), run(700)), (run(600), run(600)), (run(257), run(1000)),
             (run(1000), run(257)), (run(256), run(256)), (run(513), run(200)), (run(200), run(513)),
             (per(750), per(390)), (per(390), per(750)), (per(1024), per(1024))]
    for cut in (255, 256, 257, 512):
        x = rnd(cut)
        pairs.append((np.concatenate([x, rnd(300)]), x.copy()))
        pairs.append((x.copy(), np.concatenate([x, rnd(300)])))
        pairs.append((np.concatenate([rnd(40), x, rnd(200)]), np.concatenate([x, x])))
    q, qo = synth.pack([a for a, _ in pairs])
    s, so = synth.pack([b for _, b in pairs])
    w = synth.Workload("ties_bands", 1, 4, go, -1, q, qo, s, so, match=2, mismatch=-3)
    flags = aln.TRACEBACK if tb else aln.SCORE_ONLY
    if group == 416 and tb:
        pytest.skip("packed 16-bit bands are score-only")
    cfg = aln.BatchConfig(wf_min_cells=1, wf_orient=orient, wf_group=4 if group == 416 else group,
                          wf_bits=16 if group == 416 else 32)
    gres, gcig = run_gpu(w, flags, config=cfg)
    ores, ocig = run_oracle(w, tb)
    bad = compare(w, gres, gcig if tb else None, ores, ocig if tb else None, "ties/%d/%d" % (orient, group))
    assert not bad, "\n".join(bad[:10])


PACKED_SCHEMES = {
    # (alphabet, match, mismatch, gap_open, gap_extend): the step bound max|sigma| + |go| + 2|ge| is
    # 7, 32 (the largest the packed bands take), 5 (linear gaps) and 40 (beyond the bound: wf_bits =
    # 16 must fall back to 32-bit bands)
    "dna": (4, 2, -3, -3, -1),
    "at_bound": (4, 10, -10, -12, -5),
    "linear": (4, 3, -2, 0, -1),
    "beyond_bound": (4, 20, -20, -10, -5),
}


@pytest.mark.parametrize("scheme", list(PACKED_SCHEMES))
@pytest.mark.parametrize("orient", [1, -1], ids=["oriented", "as_given"])
def test_wavefront_packed16(gpu, scheme, orient):
    """Grouped score-only local bands in packed 16-bit cells (wf_bits = 16) against the oracle and
    against the 32-bit bands: related pairs long enough that scores pass 32,767 (only the per-block
    offsets keep the cells in 16 bits), pairs shorter than a half band (128 rows), between a half and
    a band, of several bands, and unrelated pairs whose optima stay small."""
    import paper_2002_04561_amd as aln
    A, ma, mi, go, ge = PACKED_SCHEMES[scheme]
    rng = np.random.default_rng(5200 + len(scheme) * 3 + (orient > 0))
    lens = [(20000, 19000), (19000, 20000), (100, 900), (129, 700), (200, 300), (256, 256), (257, 600),
            (3000, 2500), (1, 500), (500, 1), (127, 128), (640, 5000)]
    lens += [tuple(int(x) for x in rng.integers(1, 3000, 2)) for _ in range(20)]
    qs, ss = [], []
    for k, (a, b) in enumerate(lens):
        x = rng.integers(0, A, a, dtype=np.uint8)
        if k % 3 != 2:
            y = synth.mutate_geometric(rng, x, 0.04, 0.01, 2.0, A)[:b]
            if len(y) < b:
                y = np.concatenate([y, rng.integers(0, A, b - len(y), dtype=np.uint8)])
        else:
            y = rng.integers(0, A, b, dtype=np.uint8)
        qs.append(x)
        ss.append(y)
    q, qo = synth.pack(qs)
    s, so = synth.pack(ss)
    w = synth.Workload("packed16_" + scheme, 1, A, go, ge, q, qo, s, so, match=ma, mismatch=mi)
    cfg = dict(wf_min_cells=1, wf_orient=orient, wf_group=4)
    gres, _ = run_gpu(w, aln.SCORE_ONLY, config=aln.BatchConfig(wf_bits=16, **cfg))
    ores, _ = run_oracle(w, False)
    bad = compare(w, gres, None, ores, None, "p16/%s/%d" % (scheme, orient))
    assert not bad, "\n".join(bad[:10])
    assert int(ores["score"][0]) > 32767  # the first pair's optimum does not fit 16 bits
    g32, _ = run_gpu(w, aln.SCORE_ONLY, config=aln.BatchConfig(wf_bits=32, **cfg))
    for f in ("score", "q_end", "s_end", "flags"):
        assert np.array_equal(gres[f], g32[f]), f


@pytest.mark.parametrize("diag", [None, 19, 21], ids=["protein", "at_bound", "beyond_bound"])
@pytest.mark.parametrize("orient", [1, -1], ids=["oriented", "as_given"])
def test_wavefront_packed16_protein(gpu, diag, orient):
    """Packed 16-bit bands with per-lane 20-letter profiles (local affine -11/-1): the protein table (+4..+11 on
    the diagonal), one with +19 (step bound max|sigma| + |go| + 2|ge| = 32, the largest the packed bands
    take) and one with +21 (beyond it: wf_bits = 16 falls back to 32-bit bands), against the oracle and the
    32-bit bands; related pairs long enough that the optimum passes 32,767, short, multi-band and unrelated
    pairs."""
    import paper_2002_04561_amd as aln
    rng = np.random.default_rng(7300 + (diag or 0) + (orient > 0))
    sig = synth.protein_sigma(rng)
    if diag is not None:
        sig = sig.copy()
        np.fill_diagonal(sig, diag)
    lens = [(6000, 5800), (5800, 6000), (100, 900), (129, 700), (256, 256), (257, 600), (1, 500), (500, 1),
            (127, 128), (640, 3000)]
    lens += [tuple(int(x) for x in rng.integers(1, 2500, 2)) for _ in range(16)]
    qs, ss = [], []
    for k, (a, b) in enumerate(lens):
        x = rng.integers(0, 20, a, dtype=np.uint8)
        if k % 3 != 2:
            y = synth.mutate_geometric(rng, x, 0.04, 0.01, 2.0, 20)[:b]
            if len(y) < b:
                y = np.concatenate([y, rng.integers(0, 20, b - len(y), dtype=np.uint8)])
        else:
            y = rng.integers(0, 20, b, dtype=np.uint8)
        qs.append(x)
        ss.append(y)
    q, qo = synth.pack(qs)
    s, so = synth.pack(ss)
    w = synth.Workload("packed16_protein", synth.LOCAL, 20, -11, -1, q, qo, s, so, subst=sig)
    cfg = dict(wf_min_cells=1, wf_orient=orient, wf_group=4)
    gres, _ = run_gpu(w, aln.SCORE_ONLY, config=aln.BatchConfig(wf_bits=16, **cfg))
    ores, _ = run_oracle(w, False)
    bad = compare(w, gres, None, ores, None, "p16 protein/%s/%d" % (diag, orient))
    assert not bad, "\n".join(bad[:10])
    assert int(ores["score"][0]) > 32767  # the first pair's optimum does not fit 16 bits
    g32, _ = run_gpu(w, aln.SCORE_ONLY, config=aln.BatchConfig(wf_bits=32, **cfg))
    for f in ("score", "q_end", "s_end", "flags"):
        assert np.array_equal(gres[f], g32[f]), f


@pytest.mark.parametrize("waves", [1, 4, 16, 32])
@pytest.mark.parametrize("group", [1, 4], ids=["alone", "grouped"])
def test_wavefront_waves_per_cu(gpu, waves, group):
    """The persistent grid size changes nothing: few waves per CU (long queues) and many."""
    import paper_2002_04561_amd as aln
    w = _workload(880 + waves, 120, 100, 2500, 1, "prot_affine")
    cfg = aln.BatchConfig(wf_min_cells=1 << 14, wf_waves_per_cu=waves, wf_group=group)
    gres, _ = run_gpu(w, aln.SCORE_ONLY, config=cfg)
    ores, _ = run_oracle(w, False)
    bad = compare(w, gres, None, ores, None, "waves %d" % waves)
    assert not bad, "\n".join(bad[:10])


def test_understated_totals_flag_wavefront_pairs(gpu):
    """total_q / total_s below the real sums leave the workspace too small for the wavefront pairs' bands
    and row slots; the planner's capacity check drops those pairs with ALN_RES_DEVICE_ERROR instead of
    overrunning the workspace, and the one-pair-per-lane pairs still come back exact."""
    import torch

    import paper_2002_04561_amd as aln
    rng = np.random.default_rng(41)
    qs = [rng.integers(0, 4, 1500 if k % 4 == 0 else 60, dtype=np.uint8) for k in range(24)]
    ss = [rng.integers(0, 4, 1400 if k % 4 == 0 else 70, dtype=np.uint8) for k in range(24)]
    q, qo = synth.pack(qs)
    s, so = synth.pack(ss)
    w = synth.Workload("understated", 1, 4, -3, -1, q, qo, s, so, match=2, mismatch=-3)
    dq, dqo, ds, dso = aln.to_device(w)
    # the 60 x 70 pairs (4200 cells) stay one per lane: a threshold of 2^16 cells, given explicitly
    ba = aln.BatchAligner(aln.scoring_of(w), dq, dqo, ds, dso, 1500, 1400, aln.SCORE_ONLY, total_q=64, total_s=64,
                          config=aln.BatchConfig(wf_min_cells=1 << 16))
    ba.run()
    torch.cuda.synchronize()
    res = ba.results()
    ores, _ = run_oracle(w, False)
    for k in range(w.n_pairs):
        if k % 4 == 0:
            assert res["flags"][k] & aln.RES_DEVICE_ERROR, k
        else:
            assert (res["score"][k], res["q_end"][k], res["s_end"][k]) == (ores["score"][k], ores["q_end"][k],
                                                                          ores["s_end"][k]), k


@pytest.mark.parametrize("tb", [False, True], ids=["score", "traceback"])
def test_local_int16_beyond_the_bound(gpu, tb):
    """Unrelated protein pairs whose min(n, m) x max sigma exceeds the 16-bit a-priori bound, but whose local
    optima stay far below 32767, keep their 16-bit results (no ALN_RES_INT32_REDO) and equal the oracle's bit
    for bit; two identical pairs reach 32767 and are redone in 32 bits.  Score-only: 3300..4000 letters under
    the +4..+11 table, identical pairs of 5200.  Traceback (whose lanes take pairs under 2^18 cells): 400..500
    letters under the same table with a diagonal of +100, identical pairs of 500."""
    import paper_2002_04561_amd as aln
    rng = np.random.default_rng(41)
    sig = synth.protein_sigma(rng)
    lo, hi, hot = (3300, 4000, 5200) if not tb else (400, 500, 500)
    if tb:
        sig = sig.copy()
        np.fill_diagonal(sig, 100)
    qs, ss = [], []
    for k in range(48):
        n, m = int(rng.integers(lo, hi)), int(rng.integers(lo, hi))
        qs.append(rng.integers(0, 20, n, dtype=np.uint8))
        ss.append(rng.integers(0, 20, m, dtype=np.uint8))
    for _ in range(2):
        a = rng.integers(0, 20, hot, dtype=np.uint8)
        qs.append(a)
        ss.append(a.copy())
    q, qo = synth.pack(qs)
    s, so = synth.pack(ss)
    w = synth.Workload("local16", synth.LOCAL, 20, -11, -1, q, qo, s, so, subst=sig, traceback=tb)
    n, m = w.lengths()
    assert (np.minimum(n, m) * int(sig.max()) > 32000).all()  # the a-priori bound fails for every pair
    assert tb is False or (n * m < (1 << 18)).all()
    ores, ocig = run_oracle(w, tb)
    assert (ores["score"][-2:] > 32767).all() and (ores["score"][:-2] < 32767).all()
    lanes_only = aln.BatchConfig(wf_min_cells=-1)
    flags = aln.TRACEBACK if tb else aln.SCORE_ONLY
    gres, gcig = run_gpu(w, flags, config=lanes_only)
    bad = compare(w, gres, gcig, ores, ocig, "local16")
    assert not bad, "\n".join(bad[:10])
    redo = (gres["flags"] & aln.RES_INT32_REDO) != 0
    assert not redo[:-2].any() and redo[-2:].all()


@pytest.mark.parametrize("tb", [False, True], ids=["score", "cigar"])
def test_per_band_level_order(gpu, tb):
    """The per-band engine hands its bands out level by level (band 0 of every pair, then band 1, ...): a
    batch of pairs with 1 to 12 bands in shuffled order, some with an empty side, every pair on the band
    wavefront and the engine forced to one wave per band, is exact against the oracle, score and end cell
    (and CIGAR).  Pairs of one band, pairs whose bands outnumber the others' and empty pairs share the
    levels."""
    import paper_2002_04561_amd as aln
    rng = np.random.default_rng(4711 + tb)
    qs, ss = [], []
    for k in range(160):
        nb = int(rng.integers(1, 13))
        n = int(rng.integers((nb - 1) * 256 + 1, nb * 256 + 1))
        m = int(rng.integers(1, 900)) if k % 9 else 0
        a = rng.integers(0, 4, n, dtype=np.uint8)
        if m and rng.random() < 0.6:
            b = synth.mutate_geometric(rng, a, 0.06, 0.01, 3.0)[:m]
            if len(b) < m:
                b = np.concatenate([b, rng.integers(0, 4, m - len(b), dtype=np.uint8)])
        else:
            b = rng.integers(0, 4, m, dtype=np.uint8)
        qs.append(a)
        ss.append(b)
    q, qo = synth.pack(qs)
    s, so = synth.pack(ss)
    w = synth.Workload("level_order", synth.LOCAL, 4, -3, -1, q, qo, s, so, match=2, mismatch=-3)
    cfg = aln.BatchConfig(wf_min_cells=1, wf_group=1, wf_orient=0)
    flags = aln.TRACEBACK if tb else aln.SCORE_ONLY
    gres, gcig = run_gpu(w, flags, config=cfg)
    ores, ocig = run_oracle(w, tb)
    bad = compare(w, gres, gcig, ores, ocig, "level order/%s" % ("cigar" if tb else "score"))
    assert not bad, "\n".join(bad[:10])
