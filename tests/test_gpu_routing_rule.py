"""The planner's routing rule (aln_batch_route) and the device following it.  Score-only batches send pairs
of 2^12 cells or more to the band wavefront while they are too few to fill the one-pair-per-lane kernels
(128 pairs x 8 waves per compute unit), and pairs of 2^16 cells or more once they fill them; traceback
batches send pairs of 2^18 cells or more, or with a side above 1024.  On the device the routing shows
through the documented capacity check: with total_q = total_s = 0 the wavefront's row slots are sized for
nothing, so every multi-band pair routed there comes back flagged ALN_RES_DEVICE_ERROR, while pairs run
one per lane come back exact."""
import numpy as np
import pytest

import synth
from helpers import compare, run_oracle

pytestmark = pytest.mark.gpu

INT64_MAX = (1 << 63) - 1


def _cus():
    import torch
    return torch.cuda.get_device_properties(0).multi_processor_count


def test_route_rule_values(gpu):
    import paper_2002_04561_amd as aln
    fill = 128 * 8 * _cus()
    assert aln.aln_batch_route(1) == (1 << 12, INT64_MAX)
    assert aln.aln_batch_route(fill - 1) == (1 << 12, INT64_MAX)
    assert aln.aln_batch_route(fill) == (1 << 16, INT64_MAX)
    assert aln.aln_batch_route(10, config=aln.BatchConfig(wf_min_cells=777)) == (777, INT64_MAX)
    assert aln.aln_batch_route(10, config=aln.BatchConfig(wf_min_cells=-1)) == (INT64_MAX, INT64_MAX)
    # traceback: fixed, whatever the config
    assert aln.aln_batch_route(10, aln.TRACEBACK) == (1 << 18, 1024)
    assert aln.aln_batch_route(fill, aln.TRACEBACK, aln.BatchConfig(wf_min_cells=5)) == (1 << 18, 1024)
    with pytest.raises(aln.AlnError):
        aln.aln_batch_route(-1)
    with pytest.raises(aln.AlnError):
        aln.aln_batch_route(1, 1 << 9)


def _two_shapes(n_pairs, n, m_lo, m_hi, seed):
    """Alternating pairs of n x m_lo (just under the threshold) and n x m_hi (at or above it)."""
    rng = np.random.default_rng(seed)
    qs, ss = [], []
    for k in range(n_pairs):
        m = m_lo if k % 2 == 0 else m_hi
        a = rng.integers(0, 4, n, dtype=np.uint8)
        b = a[:m].copy()
        flip = rng.random(m) < 0.1
        b[flip] = rng.integers(0, 4, int(flip.sum()), dtype=np.uint8)
        qs.append(a)
        ss.append(b)
    q, qo = synth.pack(qs)
    s, so = synth.pack(ss)
    return synth.Workload("route", synth.LOCAL, 4, -3, -1, q, qo, s, so, match=2, mismatch=-3)


def _run_understated(w):
    """aln_align_batch with total_q = total_s = 0 (an understatement the planner's capacity check catches)."""
    import torch

    import paper_2002_04561_amd as aln
    n, m = w.lengths()
    q, qo, s, so = aln.to_device(w)
    sc = aln.scoring_of(w)
    max_n, max_m = int(n.max()), int(m.max())
    ws_bytes = aln.aln_batch_workspace_size(sc, w.n_pairs, max_n, max_m, 0, 0, aln.SCORE_ONLY)
    ws = torch.empty(max(ws_bytes, 256), dtype=torch.uint8, device="cuda")
    out = torch.empty(w.n_pairs * 8, dtype=torch.int32, device="cuda")
    st = aln.aln_align_batch(sc, w.n_pairs, q, qo, s, so, max_n, max_m, 0, 0, aln.SCORE_ONLY, out, None, None, ws,
                             ws_bytes)
    assert st == 0
    torch.cuda.synchronize()
    return out.to("cpu").numpy().view(aln.RESULT_DTYPE)


@pytest.mark.parametrize("big_batch", [False, True])
def test_device_follows_the_rule(gpu, big_batch):
    """257-row pairs (two bands) with 2^12 - 1 / 2^12 + 16 cells in a small batch, 2^16 - 1 / 2^16 + 256 cells
    in a batch that fills the per-lane kernels: the pairs at or above the threshold are the flagged ones."""
    import paper_2002_04561_amd as aln
    if big_batch:
        n_pairs = 128 * 8 * _cus()
        w = _two_shapes(n_pairs, 257, 255, 256, seed=81)  # 65535 and 65792 cells
        assert aln.aln_batch_route(n_pairs)[0] == 1 << 16
    else:
        w = _two_shapes(64, 257, 15, 16, seed=82)  # 3855 and 4112 cells
        assert aln.aln_batch_route(64)[0] == 1 << 12
    res = _run_understated(w)
    flagged = (res["flags"] & aln.RES_DEVICE_ERROR) != 0
    assert flagged[1::2].all() and not flagged[0::2].any()
    # the pairs run one per lane are exact; check a sample against the oracle
    keep = np.arange(0, w.n_pairs, 2)[:512]
    sub = w.subset(keep)
    ores, _ = run_oracle(sub, False)
    bad = compare(sub, res[keep], None, ores, None, "per-lane")
    assert not bad, bad[:3]
