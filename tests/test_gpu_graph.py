"""aln_align_batch captured in a HIP graph: every replay equals the eager result and the oracle."""
import numpy as np
import pytest

import synth
from helpers import compare, run_oracle

pytestmark = pytest.mark.gpu


def _mixed_workload():
    rng = np.random.default_rng(77)
    lens = np.rint(np.exp(rng.uniform(np.log(40), np.log(2500), (160, 2)))).astype(int)
    qs = [rng.integers(0, 20, a, dtype=np.uint8) for a, _ in lens]
    ss = [rng.integers(0, 20, b, dtype=np.uint8) for _, b in lens]
    q, qo = synth.pack(qs)
    s, so = synth.pack(ss)
    sig = synth.protein_sigma(rng)
    return synth.Workload("mixed", synth.LOCAL, 20, -11, -1, q, qo, s, so, subst=sig)


@pytest.mark.parametrize("kind", ["uneven_score", "reads_traceback"])
def test_graph_replays(gpu, kind):
    import torch

    import paper_2002_04561_amd as aln
    if kind == "uneven_score":
        w = _mixed_workload()
        flags = aln.SCORE_ONLY
    else:
        w = synth.reads_semiglobal(seed=5, n_pairs=3000)
        flags = aln.TRACEBACK
    n, m = w.lengths()
    q, qo, s, so = aln.to_device(w)
    ba = aln.BatchAligner(aln.scoring_of(w), q, qo, s, so, int(n.max()), int(m.max()), flags)
    ba.run()
    torch.cuda.synchronize()
    eager = ba.results().copy()
    eager_cig = ba.cigars() if flags & aln.TRACEBACK else None
    ores, ocig = run_oracle(w, bool(flags & aln.TRACEBACK))
    assert not compare(w, eager, eager_cig, ores, ocig, "eager")

    g = torch.cuda.CUDAGraph()
    side = torch.cuda.Stream()
    side.wait_stream(torch.cuda.current_stream())
    with torch.cuda.stream(side):
        with torch.cuda.graph(g):
            ba.run()
    torch.cuda.current_stream().wait_stream(side)
    torch.cuda.synchronize()
    for rep in range(3):
        ba.out.zero_()
        if ba.cigar is not None:
            ba.cigar.zero_()
        junk = torch.randn(1 << 20, device="cuda").sum()  # unrelated eager work between replays
        torch.cuda.synchronize()
        g.replay()
        torch.cuda.synchronize()
        got = ba.results()
        got_cig = ba.cigars() if flags & aln.TRACEBACK else None
        bad = compare(w, got, got_cig, ores, ocig, "replay %d" % rep)
        assert not bad, "\n".join(bad[:5])
        assert float(junk) == float(junk)
