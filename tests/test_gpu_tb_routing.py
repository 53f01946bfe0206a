"""Traceback batches whose pairs spread from 64 to 16384 letters.  Pairs of 2^18 cells or more, or longer
than 1024 on a side, run on the band wavefront with their predecessor codes in an arena of the workspace;
the rest run one pair per lane, whose code slabs then hold pairs up to 1024 x 1024 only.  Every pair's
score, end and begin cells and CIGAR equal the oracle's canonical traceback (Sec. III-A), with an arena
that holds every wavefront pair and with one too small for most of them (those that find no room run
per lane, with the same results)."""
from concurrent.futures import ThreadPoolExecutor

import numpy as np
import pytest

import oracle
import synth
from helpers import compare, oracle_scoring

pytestmark = pytest.mark.gpu

# pairs placed at the routing boundaries: 512 x 511 stays per lane (just under 2^18 cells), 512 x 512
# and 1024 x 1024 go to the wavefront, and so does every pair longer than 1024 on one side however few
# its cells, even with the other side empty (then it has no bands)
EDGES = [(512, 511), (512, 512), (1024, 1024), (1025, 1), (1, 1025), (64, 16384), (16384, 64), (0, 3000),
         (3000, 0), (16384, 16384)]


def _mixed(seed, n_random, lmax, mode, alphabet, go, ge, edges, **kw):
    rng = np.random.default_rng(seed)
    lens = np.rint(np.exp(rng.uniform(np.log(64), np.log(lmax), (n_random, 2)))).astype(int).tolist()
    lens = [tuple(x) for x in lens] + [e for e in edges if max(e) <= lmax]
    order = rng.permutation(len(lens))
    qs, ss = [], []
    for k in order:
        n, m = lens[k]
        a = rng.integers(0, alphabet, max(n, m), dtype=np.uint8)
        b = a.copy()
        mut = rng.random(len(b)) < 0.15  # related pairs, so local and semi-global CIGARs are long
        b[mut] = rng.integers(0, alphabet, int(mut.sum()), dtype=np.uint8)
        qs.append(a[:n])
        ss.append(b[:m])
    q, qo = synth.pack(qs)
    s, so = synth.pack(ss)
    return synth.Workload("tb_routing", mode, alphabet, go, ge, q, qo, s, so, traceback=True, **kw)


def _oracle(w):
    """The oracle's canonical results, pair by pair: the full-matrix traceback for pairs up to 2^22 cells,
    the checkpointed one (same results, pinned against it) above, on host threads."""
    sc = oracle_scoring(w)
    n, m = w.lengths()

    def one(k):
        q = w.q[w.q_off[k]:w.q_off[k + 1]]
        s = w.s[w.s_off[k]:w.s_off[k + 1]]
        impl = "affine" if int(n[k]) * int(m[k]) <= (1 << 22) else "checkpointed"
        return oracle.align(sc, q, s, traceback=True, impl=impl)

    with ThreadPoolExecutor(8) as ex:
        al = list(ex.map(one, range(w.n_pairs)))
    res = {key: np.array([getattr(a, key) for a in al]) for key in
           ("score", "q_begin", "q_end", "s_begin", "s_end", "flags")}
    return res, [a.cigar for a in al]


def _gpu(w):
    import torch

    import paper_2002_04561_amd as aln
    n, m = w.lengths()
    q, qo, s, so = aln.to_device(w)
    ba = aln.BatchAligner(aln.scoring_of(w), q, qo, s, so, int(n.max()), int(m.max()), aln.TRACEBACK)
    ba.run()
    torch.cuda.synchronize()
    return ba


SCHEMES = [
    ("local_protein", dict(mode=synth.LOCAL, alphabet=20, go=-11, ge=-1, subst=True)),
    ("global_dna", dict(mode=synth.GLOBAL, alphabet=4, go=-3, ge=-1, match=2, mismatch=-3)),
    ("semi_dna", dict(mode=synth.SEMIGLOBAL, alphabet=4, go=-5, ge=-2, match=1, mismatch=-4)),
]


def _workload(k, n_random, lmax, edges):
    name, p = SCHEMES[k]
    p = dict(p)
    kw = {}
    if p.pop("subst", False):
        kw["subst"] = synth.protein_sigma(np.random.default_rng(40 + k))
    else:
        kw["match"], kw["mismatch"] = p.pop("match"), p.pop("mismatch")
    return _mixed(60 + k, n_random, lmax, p["mode"], p["alphabet"], p["go"], p["ge"], edges, **kw)


@pytest.mark.parametrize("k", range(len(SCHEMES)))
def test_mixed_64_to_16384_equals_oracle(gpu, k):
    """48 pairs of log-uniform lengths 64..16384 plus the boundary shapes: bit-exact against the oracle.
    The workspace holds the arena and per-lane slabs for 1024 x 1024 pairs: far below one slab of
    16384 x 16384 codes (8.6 GB per wave), which a per-lane-only traceback would need."""
    import paper_2002_04561_amd as aln
    w = _workload(k, 48, 16384, EDGES)
    ba = _gpu(w)
    assert ba.ws_bytes < (4 << 30), ba.ws_bytes
    ores, ocig = _oracle(w)
    bad = compare(w, ba.results(), ba.cigars(), ores, ocig, SCHEMES[k][0])
    assert not bad, bad[:3]
    assert not (ba.results()["flags"].astype(np.int64) & ~aln.RES_INT32_REDO).any()


def test_small_arena_falls_back_per_lane(gpu):
    """An arena of 32 MiB holds only a few of the wavefront pairs' codes (a 4096 x 4096 pair takes 8 MiB);
    the rest run one pair per lane, whose slabs are then sized for the largest pair.  Results equal the
    oracle's and those of the default arena."""
    import paper_2002_04561_amd as aln
    w = _workload(0, 40, 4096, [(512, 512), (1025, 3), (4096, 4096), (4096, 64), (0, 100)])
    full = _gpu(w)
    aln.aln_set_batch_code_arena(32 << 20)
    try:
        small = _gpu(w)
    finally:
        aln.aln_set_batch_code_arena(0)
    ores, ocig = _oracle(w)
    bad = compare(w, small.results(), small.cigars(), ores, ocig, "small arena")
    assert not bad, bad[:3]
    bad = compare(w, full.results(), full.cigars(), ores, ocig, "default arena")
    assert not bad, bad[:3]


def test_bad_codes_and_empty_sides_on_the_wavefront(gpu):
    """Letters >= alphabet_size give ALN_RES_BAD_CODE and no CIGAR wherever the pair runs: a pair longer
    than 1024 whose other side is empty (no bands: its letters are checked when its result is made), a
    banded wavefront pair and a per-lane pair; the same shapes with valid letters give the oracle's
    results."""
    rng = np.random.default_rng(71)
    shapes = [(3000, 0), (0, 2500), (2000, 1500), (100, 90), (3000, 0), (2000, 1500), (1, 1025)]
    qs = [rng.integers(0, 4, n, dtype=np.uint8) for n, _ in shapes]
    ss = [rng.integers(0, 4, m, dtype=np.uint8) for _, m in shapes]
    qs[0][1234] = 4
    ss[1][2499] = 9
    ss[2][7] = 4
    qs[3][0] = 200
    q, qo = synth.pack(qs)
    s, so = synth.pack(ss)
    import paper_2002_04561_amd as aln
    for mode in (synth.GLOBAL, synth.LOCAL, synth.SEMIGLOBAL):
        w = synth.Workload("tb_bad_codes", mode, 4, -3, -1, q, qo, s, so, match=2, mismatch=-3, traceback=True)
        ba = _gpu(w)
        ores, ocig = _oracle(w)
        res = ba.results()
        bad = compare(w, res, ba.cigars(), ores, ocig, "mode %d" % mode)
        assert not bad, bad[:3]
        assert [bool(f & aln.RES_BAD_CODE) for f in res["flags"]] == [True, True, True, True, False, False, False]
