"""aln_align_batch_noalloc: the batch call with its workspace in the library's device scratch instead of a
caller buffer.  Its results must be bit-identical to aln_align_batch's on the same pairs (which the parity
tests hold to the oracle), on two calls in a row, the second with a smaller batch (the scratch keeps the
first call's contents), score-only and with CIGARs; a batch that needs more than the scratch is refused
before any device work."""
import ctypes

import numpy as np
import pytest

import synth

pytestmark = pytest.mark.gpu


def _buffers(w, flags):
    import torch

    import paper_2002_04561_amd as aln
    n, m = w.lengths()
    q, qo, s, so = aln.to_device(w)
    out = torch.full((w.n_pairs * 8,), -7, dtype=torch.int32, device="cuda")
    cig = coff = None
    if flags & aln.TRACEBACK:
        cap = np.maximum(n + m, 1)
        c = np.zeros(w.n_pairs + 1, np.int64)
        np.cumsum(cap, out=c[1:])
        coff = torch.from_numpy(c).cuda()
        cig = torch.full((int(c[-1]),), -1, dtype=torch.int32, device="cuda")
    return dict(q=q, qo=qo, s=s, so=so, out=out, cig=cig, coff=coff, max_n=max(int(n.max()), 1),
                max_m=max(int(m.max()), 1))


def _results(b, w, flags):
    import paper_2002_04561_amd as aln
    res = b["out"].to("cpu").numpy().view(aln.RESULT_DTYPE).copy()
    cig = None
    if flags & aln.TRACEBACK:
        words = b["cig"].to("cpu").numpy().view(np.uint32)
        coff = b["coff"].to("cpu").numpy()
        cig = [words[coff[k]:coff[k] + res["cigar_len"][k]].tolist() for k in range(w.n_pairs)]
    return res, cig


def _with_workspace(w, flags):
    import torch

    import paper_2002_04561_amd as aln
    b = _buffers(w, flags)
    sc = aln.scoring_of(w)
    nbytes = aln.aln_batch_workspace_size(sc, w.n_pairs, b["max_n"], b["max_m"], int(b["q"].numel()),
                                          int(b["s"].numel()), flags)
    ws = torch.empty(nbytes, dtype=torch.uint8, device="cuda")
    st = aln.aln_align_batch(sc, w.n_pairs, b["q"], b["qo"], b["s"], b["so"], b["max_n"], b["max_m"],
                             int(b["q"].numel()), int(b["s"].numel()), flags, b["out"], b["cig"], b["coff"], ws,
                             nbytes)
    assert st == 0
    torch.cuda.synchronize()
    return _results(b, w, flags)


def _noalloc(w, flags):
    import torch

    import paper_2002_04561_amd as aln
    b = _buffers(w, flags)
    sc = aln.scoring_of(w).c()
    ptr = lambda t: None if t is None else int(t.data_ptr())  # noqa: E731
    stream = int(torch.cuda.current_stream().cuda_stream)
    st = aln.lib().aln_align_batch_noalloc(ctypes.byref(sc), w.n_pairs, ptr(b["q"]), ptr(b["qo"]), ptr(b["s"]),
                                           ptr(b["so"]), b["max_n"], b["max_m"], int(b["q"].numel()),
                                           int(b["s"].numel()), flags, None, ptr(b["out"]), ptr(b["cig"]),
                                           ptr(b["coff"]), stream)
    assert st == 0, st
    torch.cuda.synchronize()
    return _results(b, w, flags)


@pytest.mark.parametrize("tb", [False, True], ids=["score", "cigar"])
def test_noalloc_equals_batch_twice(gpu, tb):
    import paper_2002_04561_amd as aln
    flags = aln.TRACEBACK if tb else aln.SCORE_ONLY
    big = synth.random_pairs(301, 400, 20, 300, 4, synth.SEMIGLOBAL, -5, -2, match=1, mismatch=-4, related=0.7)
    small = synth.random_pairs(302, 60, 5, 120, 4, synth.SEMIGLOBAL, -5, -2, match=1, mismatch=-4, related=0.7)
    for w in (big, small):
        got = _noalloc(w, flags)
        exp = _with_workspace(w, flags)
        assert np.array_equal(got[0], exp[0])
        assert got[1] == exp[1]


def test_noalloc_local_with_wavefront_pairs(gpu):
    """Pairs large enough for the band wavefront share the scratch with the one-pair-per-lane kernels."""
    import paper_2002_04561_amd as aln
    w1 = synth.random_pairs(303, 24, 200, 1500, 4, synth.LOCAL, -3, -1, match=2, mismatch=-3, related=0.8)
    w2 = synth.random_pairs(304, 10, 100, 900, 4, synth.LOCAL, -3, -1, match=2, mismatch=-3, related=0.8)
    for w in (w1, w2):
        got = _noalloc(w, aln.SCORE_ONLY)
        exp = _with_workspace(w, aln.SCORE_ONLY)
        assert np.array_equal(got[0], exp[0])


def test_noalloc_refuses_oversize(gpu):
    import torch

    import paper_2002_04561_amd as aln
    cap = int(aln.lib().aln_noalloc_scratch_bytes())
    assert cap == 64 << 20
    sc = aln.Scoring(synth.GLOBAL, 4, -3, -1, match=2, mismatch=-3).c()
    # a traceback batch of 2^20 pairs up to 4000 x 4000 needs far more than the scratch
    # no buffer is passed: the size check refuses the call before anything would read them
    st = aln.lib().aln_align_batch_noalloc(ctypes.byref(sc), 1 << 20, None, None, None, None, 4000, 4000, 1 << 31,
                                           1 << 31, aln.TRACEBACK, None, None, None, None,
                                           int(torch.cuda.current_stream().cuda_stream))
    assert st == -4
