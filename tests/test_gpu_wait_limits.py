"""Bounded device-side waits.  With a poll limit of one, the band wavefront's hand-off waits (device memory
between bands on their own waves, LDS between the bands of a workgroup, and the couriers' device-memory
waits) give up almost at once: every kernel must still exit, the pairs of the affected launch come back
flagged ALN_RES_DEVICE_ERROR, and pairs that did not go through a failed wait are exact.  With the limits
restored the same calls match the oracle."""
import numpy as np
import pytest

import synth
from helpers import compare, run_gpu, run_oracle

pytestmark = pytest.mark.gpu


def _workload():
    # pairs of 6..10 bands of 256 rows, plus small pairs that run one pair per lane
    big = synth.random_pairs(31, 6, 1500, 2500, 4, synth.LOCAL, -3, -1, match=2, mismatch=-3, related=0.8)
    small = synth.random_pairs(32, 40, 10, 60, 4, synth.LOCAL, -3, -1, match=2, mismatch=-3, related=0.5)
    qs = [big.pair(k)[0] for k in range(big.n_pairs)] + [small.pair(k)[0] for k in range(small.n_pairs)]
    ss = [big.pair(k)[1] for k in range(big.n_pairs)] + [small.pair(k)[1] for k in range(small.n_pairs)]
    q, qo = synth.pack(qs)
    s, so = synth.pack(ss)
    return synth.Workload("wait_limits", synth.LOCAL, 4, -3, -1, q, qo, s, so, match=2, mismatch=-3)


def test_tiny_wait_limit_gives_up_and_exits(gpu):
    import torch

    import paper_2002_04561_amd as aln
    w = _workload()
    ores, _ = run_oracle(w, False)
    n, m = w.lengths()
    big = n * m >= 1 << 16
    configs = [aln.BatchConfig(wf_min_cells=1 << 16, wf_group=1), aln.BatchConfig(wf_min_cells=1 << 16, wf_group=4)]
    flagged = 0
    try:
        aln.aln_set_wait_limits(1, 1)
        for cfg in configs:
            res, _ = run_gpu(w, aln.SCORE_ONLY, config=cfg)
            err = (res["flags"] & aln.RES_DEVICE_ERROR) != 0
            flagged += int(err.sum())
            assert not err[~big].any(), "one-pair-per-lane pairs have no waits"
            ok = ~err
            assert np.array_equal(res["score"][ok], ores["score"][ok].astype(np.int32)), cfg
            assert np.array_equal(res["q_end"][ok], ores["q_end"][ok].astype(np.int32)), cfg
        # one long pair through aln_align_long (grouped bands and couriers)
        a, b = w.pair(0)
        la = aln.LongAligner(aln.scoring_of(w), torch.from_numpy(a.copy()).cuda(), torch.from_numpy(b.copy()).cuda())
        la.run()
        torch.cuda.synchronize()
        r = la.result()
        if int(r["flags"]) & aln.RES_DEVICE_ERROR:
            flagged += 1
        else:
            assert (int(r["score"]), int(r["q_end"]), int(r["s_end"])) == (
                int(ores["score"][0]), int(ores["q_end"][0]), int(ores["s_end"][0]))
    finally:
        aln.aln_set_wait_limits(0, 0)
    assert flagged > 0, "a poll limit of one should make some hand-off wait give up"
    for cfg in configs:
        res, _ = run_gpu(w, aln.SCORE_ONLY, config=cfg)
        assert not compare(w, res, None, ores, None, "restored")
