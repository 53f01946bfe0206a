"""aln_traceback: CIGARs re-emitted from the end cells a forward call found.  Every pair is compared
bit-exactly with the oracle's canonical traceback (Sec. III-A definitions, the readings of the oracle):
after a score-only batch, after a batch whose CIGAR buffers were too small (only the truncated pairs are
traced back, into resized buffers), in place (out = fwd), and with end cells that are not valid."""
import numpy as np
import pytest

import synth
from helpers import compare, run_oracle

pytestmark = pytest.mark.gpu


def _schemes():
    rng = np.random.default_rng(5)
    sig20 = synth.protein_sigma(rng)
    return [
        ("global_linear", synth.random_pairs(51, 120, 0, 300, 4, synth.GLOBAL, 0, -1, match=2, mismatch=-1, related=0.5)),
        ("local_affine", synth.random_pairs(52, 120, 0, 300, 4, synth.LOCAL, -3, -1, match=2, mismatch=-3, related=0.7)),
        ("semi_affine", synth.random_pairs(53, 120, 0, 300, 4, synth.SEMIGLOBAL, -5, -2, match=1, mismatch=-4,
                                           related=0.7)),
        ("local_protein", synth.random_pairs(54, 80, 0, 400, 20, synth.LOCAL, -11, -1, subst=sig20, related=0.4)),
        ("global_affine_table", synth.random_pairs(55, 80, 0, 200, 20, synth.GLOBAL, -11, -1, subst=sig20,
                                                   related=0.4)),
    ]


def _forward(w, flags, cap=None):
    import torch

    import paper_2002_04561_amd as aln
    n, m = w.lengths()
    q, qo, s, so = aln.to_device(w)
    ba = aln.BatchAligner(aln.scoring_of(w), q, qo, s, so, max(int(n.max()), 1), max(int(m.max()), 1), flags,
                          cigar_capacity=cap)
    ba.run()
    torch.cuda.synchronize()
    return ba, (q, qo, s, so)


@pytest.mark.parametrize("k", range(5))
def test_traceback_after_score_only(gpu, k):
    import paper_2002_04561_amd as aln
    name, w = _schemes()[k]
    ores, ocig = run_oracle(w, True)
    ba, (q, qo, s, so) = _forward(w, aln.SCORE_ONLY)
    n, m = w.lengths()
    res, runs = aln.traceback_pairs(aln.scoring_of(w), q, qo, s, so, max(int(n.max()), 1), max(int(m.max()), 1),
                                    ba.out)
    bad = compare(w, res, runs, ores, ocig, name)
    assert not bad, bad[:3]


def test_truncated_cigars_recovered(gpu):
    """A traceback batch with one CIGAR word of room per pair: pairs of several runs come back truncated with
    the count they need; aln_traceback on just those pairs, with that much room, gives the oracle's CIGARs."""
    import torch

    import paper_2002_04561_amd as aln
    name, w = _schemes()[2]
    ores, ocig = run_oracle(w, True)
    ba, _ = _forward(w, aln.TRACEBACK, cap=np.ones(w.n_pairs, np.int64))
    res = ba.results()
    trunc = np.nonzero(res["flags"] & aln.RES_CIGAR_TRUNC)[0]
    assert len(trunc) > 10
    need = res["cigar_len"][trunc].astype(np.int64)
    assert np.array_equal(need, ores["cigar_len"][trunc])
    sub = w.subset(trunc)
    q, qo, s, so = aln.to_device(sub)
    fwd = ba.out.view(-1, 8)[torch.from_numpy(trunc).cuda()].reshape(-1).contiguous()
    sn, sm = sub.lengths()
    tres, truns = aln.traceback_pairs(aln.scoring_of(sub), q, qo, s, so, int(sn.max()), int(sm.max()), fwd,
                                      cigar_capacity=need)
    for j, k in enumerate(trunc):
        assert int(tres["flags"][j]) == 0
        assert truns[j] == ocig[k], (k, truns[j], ocig[k])
        assert (int(tres["q_begin"][j]), int(tres["s_begin"][j])) == (int(ores["q_begin"][k]), int(ores["s_begin"][k]))


def test_in_place_and_bad_end_cells(gpu):
    import torch

    import paper_2002_04561_amd as aln
    name, w = _schemes()[1]
    ores, ocig = run_oracle(w, True)
    ba, (q, qo, s, so) = _forward(w, aln.SCORE_ONLY)
    n, m = w.lengths()
    fwd = ba.out.clone()
    rec = fwd.view(-1, 8)
    rec[3, 0] += 1                   # a score that is not H at the end cell
    rec[5, 2] = int(n[5]) + 1        # an end row outside the matrix
    sc = aln.scoring_of(w)
    nbytes = aln.aln_traceback_workspace_size(sc, w.n_pairs, int(n.max()), int(m.max()))
    ws = torch.empty(nbytes, dtype=torch.uint8, device="cuda")
    cap = np.maximum((n + m), 1)
    coff = np.zeros(w.n_pairs + 1, np.int64)
    np.cumsum(cap, out=coff[1:])
    cig = torch.empty(int(coff[-1]), dtype=torch.int32, device="cuda")
    st = aln.aln_traceback(sc, w.n_pairs, q, qo, s, so, int(n.max()), int(m.max()), fwd, fwd, cig,
                           torch.from_numpy(coff).cuda(), ws, nbytes)
    assert st == 0
    torch.cuda.synchronize()
    res = fwd.to("cpu").numpy().view(aln.RESULT_DTYPE)
    words = cig.to("cpu").numpy().view(np.uint32)
    for k in range(w.n_pairs):
        if k in (3, 5):
            assert int(res["flags"][k]) & aln.RES_BAD_END, k
            continue
        runs = [(int(x) >> 4, int(x) & 15) for x in words[coff[k]:coff[k] + int(res["cigar_len"][k])]]
        got = (int(res["score"][k]), int(res["q_begin"][k]), int(res["q_end"][k]), int(res["s_begin"][k]),
               int(res["s_end"][k]), int(res["flags"][k]), runs)
        exp = (int(ores["score"][k]), int(ores["q_begin"][k]), int(ores["q_end"][k]), int(ores["s_begin"][k]),
               int(ores["s_end"][k]), 0, ocig[k])
        assert got == exp, k


def test_mixed_length_traceback_batch(gpu):
    """A traceback batch whose lengths spread log-uniformly over 64..4096 (local affine protein table): every
    pair's CIGAR equals the oracle's, through aln_align_batch with ALN_TRACEBACK and through a score-only
    call followed by aln_traceback.  The traceback slabs of the one-pair-per-lane kernels run fewer waves
    when the largest pair would make them exceed their budget, so the workspace stays bounded."""
    import torch

    import paper_2002_04561_amd as aln
    rng = np.random.default_rng(17)
    sig = synth.protein_sigma(rng)
    lens = np.rint(np.exp(rng.uniform(np.log(64), np.log(4096), (96, 2)))).astype(int)
    qs = [rng.integers(0, 20, n, dtype=np.uint8) for n, _ in lens]
    ss = [rng.integers(0, 20, m, dtype=np.uint8) for _, m in lens]
    q, qo = synth.pack(qs)
    s, so = synth.pack(ss)
    w = synth.Workload("mixed_tb", synth.LOCAL, 20, -11, -1, q, qo, s, so, subst=sig, traceback=True)
    ores, ocig = run_oracle(w, True)
    ba, (dq, dqo, ds, dso) = _forward(w, aln.TRACEBACK)
    assert ba.ws_bytes < (9 << 30)
    res = ba.results()
    bad = compare(w, res, ba.cigars(), ores, ocig, "batch")
    assert not bad, bad[:3]
    fw, _ = _forward(w, aln.SCORE_ONLY)
    n, m = w.lengths()
    tres, truns = aln.traceback_pairs(aln.scoring_of(w), dq, dqo, ds, dso, int(n.max()), int(m.max()), fw.out)
    bad = compare(w, tres, truns, ores, ocig, "traceback")
    assert not bad, bad[:3]
    torch.cuda.synchronize()
