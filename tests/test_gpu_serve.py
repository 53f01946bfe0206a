"""Serving loop: every served result equals the oracle's and the same request's result alone;
memory stays within budget."""
import numpy as np
import pytest

import synth
from helpers import run_oracle

pytestmark = pytest.mark.gpu


def _stream(seed, n_req, rate_hz):
    """The serving mix (synth.serve_stream) at test sizes: proteins up to 2048 letters, long pairs of
    4096 x 4096 run alone through aln_align_long."""
    from paper_2002_04561_amd.serve import Request
    items, sig = synth.serve_stream(n_req, rate_hz, seed=seed, long_len=4096, protein_max=2048)
    reqs = [Request(it.rid, it.klass, it.q, it.s, it.arrival, traceback=synth.SERVE_CLASSES[it.klass]["traceback"],
                    long=it.klass == "long") for it in items]
    return reqs, items, sig


def _oracle_results(items, sig):
    """rid -> (score, q_begin, q_end, s_begin, s_end, flags) and CIGAR runs (None when score-only), from
    the oracle, per class."""
    out = {}
    for klass in synth.SERVE_CLASSES:
        sel = [it for it in items if it.klass == klass]
        if not sel:
            continue
        w = synth.serve_workload(sel, klass, sig)
        res, cig = run_oracle(w, w.traceback)
        for k, it in enumerate(sel):
            qb = int(res["q_begin"][k]) if w.traceback else -1
            sb = int(res["s_begin"][k]) if w.traceback else -1
            tup = (int(res["score"][k]), qb, int(res["q_end"][k]), sb, int(res["s_end"][k]), int(res["flags"][k]))
            out[it.rid] = (tup, cig[k] if w.traceback else None)
    return out


def _scorings(sig):
    import paper_2002_04561_amd as aln
    return {"read": aln.Scoring(synth.SEMIGLOBAL, 4, -5, -2, match=1, mismatch=-4),
            "protein": aln.Scoring(synth.LOCAL, 20, -11, -1, subst=sig),
            "long": aln.Scoring(synth.LOCAL, 4, -3, -1, match=2, mismatch=-3)}


def _alone(reqs, scorings):
    from paper_2002_04561_amd.serve import AlignServer
    out = {}
    for r in reqs:
        srv = AlignServer(scorings, budget_bytes=1 << 34, streams=1)
        r2 = type(r)(r.rid, r.klass, r.q, r.s, 0.0, r.traceback, r.long)
        srv.run([r2], realtime=False)
        c = srv.completed[0]
        out[r.rid] = (c.result, c.cigar)
    return out


def test_mix_equals_oracle_and_alone_and_budget(gpu):
    """Every served result equals the oracle's and its result alone; the device memory the server's batches
    held at once (torch's allocator peak over the run) stays within the budget."""
    import torch

    from paper_2002_04561_amd.serve import AlignServer
    reqs, items, sig = _stream(21, 400, 20000.0)
    sc = _scorings(sig)
    budget = 256 << 20
    srv = AlignServer(sc, budget_bytes=budget, streams=3, max_pairs=64)
    torch.cuda.synchronize()
    base = torch.cuda.memory_allocated()
    torch.cuda.reset_peak_memory_stats()
    stats = srv.run(reqs, realtime=True)
    torch.cuda.synchronize()
    live_peak = torch.cuda.max_memory_allocated() - base
    assert stats["requests"] == len(reqs)
    assert stats["peak_bytes"] <= budget
    assert live_peak <= budget, (live_peak, budget)
    got = {c.rid: (c.result, c.cigar) for c in srv.completed}
    assert sorted(got) == sorted(r.rid for r in reqs)
    expect = _oracle_results(items, sig)
    bad = [(rid, got[rid], expect[rid]) for rid in got if got[rid] != expect[rid]]
    assert not bad, [str(b)[:300] for b in bad[:5]]
    alone = _alone(reqs, sc)
    bad = [rid for rid in got if got[rid] != alone[rid]]
    assert not bad, bad[:10]
    assert set(stats["classes"]) == {"read", "protein", "long"}


def test_tiny_budget_completes(gpu):
    """A budget that holds only the largest single request's batch: requests go one or a few at a time,
    all complete, and the allocator's peak stays within the budget."""
    import torch

    from paper_2002_04561_amd.serve import Admission, AlignServer
    reqs, items, sig = _stream(22, 60, 50000.0)
    reqs = [r for r in reqs if not r.long]
    srv = AlignServer(_scorings(sig), budget_bytes=1 << 40, streams=2, max_pairs=64)
    budget = max(srv.batch_bytes(Admission.shapes([r])(1)) for r in reqs) + 1
    srv = AlignServer(_scorings(sig), budget_bytes=budget, streams=2, max_pairs=64)
    torch.cuda.synchronize()
    base = torch.cuda.memory_allocated()
    torch.cuda.reset_peak_memory_stats()
    stats = srv.run(reqs, realtime=False)
    torch.cuda.synchronize()
    assert stats["requests"] == len(reqs) and stats["peak_bytes"] <= budget
    assert torch.cuda.max_memory_allocated() - base <= budget
    expect = _oracle_results([it for it in items if it.klass != "long"], sig)
    bad = [c.rid for c in srv.completed if (c.result, c.cigar) != expect[c.rid]]
    assert not bad, bad[:10]
