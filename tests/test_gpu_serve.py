"""Serving loop: each request's result is the same alone and in the mix; memory stays within budget."""
import numpy as np
import pytest

import synth

pytestmark = pytest.mark.gpu


def _stream(seed, n_req, rate_hz):
    from paper_2002_04561_amd.serve import Request
    rng = np.random.default_rng(seed)
    reads = synth.reads_semiglobal(seed=seed, n_pairs=n_req)
    sig = synth.protein_sigma(rng)
    reqs = []
    t = 0.0
    for k in range(n_req):
        t += rng.exponential(1.0 / rate_hz)
        u = rng.random()
        if u < 0.8:
            a, b = reads.pair(k)
            reqs.append(Request(k, "read", a.copy(), b.copy(), t, traceback=True))
        elif u < 0.99:
            n, m = np.rint(np.exp(rng.uniform(np.log(64), np.log(2048), 2))).astype(int)
            reqs.append(Request(k, "protein", rng.integers(0, 20, n, dtype=np.uint8),
                                rng.integers(0, 20, m, dtype=np.uint8), t))
        else:
            a = rng.integers(0, 4, 4096, dtype=np.uint8)
            b = synth.mutate_geometric(rng, a, 0.05, 0.01, 3.0)[:4096]
            reqs.append(Request(k, "long", a, b, t, long=True))
    return reqs, sig


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


def test_mix_equals_alone_and_budget(gpu):
    from paper_2002_04561_amd.serve import AlignServer, request_bytes
    reqs, sig = _stream(21, 400, 20000.0)
    sc = _scorings(sig)
    budget = 64 << 20
    srv = AlignServer(sc, budget_bytes=budget, streams=3, max_pairs=64)
    stats = srv.run(reqs, realtime=True)
    assert stats["requests"] == len(reqs)
    assert stats["peak_bytes"] <= budget
    got = {c.rid: (c.result, c.cigar) for c in srv.completed}
    alone = _alone(reqs, sc)
    bad = [rid for rid in got if got[rid] != alone[rid]]
    assert not bad, bad[:10]
    assert set(stats["classes"]) == {"read", "protein", "long"} or len(stats["classes"]) >= 2


def test_tiny_budget_completes(gpu):
    from paper_2002_04561_amd.serve import AlignServer, request_bytes
    reqs, sig = _stream(22, 60, 50000.0)
    reqs = [r for r in reqs if not r.long]
    budget = max(request_bytes(r) for r in reqs) + 1
    srv = AlignServer(_scorings(sig), budget_bytes=budget, streams=2, max_pairs=64)
    stats = srv.run(reqs, realtime=False)
    assert stats["requests"] == len(reqs) and stats["peak_bytes"] <= budget
