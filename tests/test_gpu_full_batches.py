"""The two benchmark batches at full size, in the launch configurations the benchmark measures:
2^20 read/window pairs with CIGARs (semi-global affine) and 65,536 protein pairs of uneven lengths
(local affine, score-only).  Every pair is checked bit-exactly against the oracle: the results of all
pairs, CIGARs included, are hashed in chunks of consecutive pairs (tests/golden/digest.py) and compared
with the digests of the oracle's results stored in tests/golden/ (written by
tests/golden/make_golden.py, which calls only the oracle).  A seeded sample of 64 pairs of each is also
compared field by field, which names the pair when something differs."""
import json
import os
import sys

import numpy as np
import pytest

import synth

sys.path.insert(0, os.path.join(os.path.dirname(os.path.abspath(__file__)), "golden"))
import digest  # noqa: E402

pytestmark = pytest.mark.gpu
HERE = os.path.dirname(os.path.abspath(__file__))

# the library's defaults, and the fixed configurations the committed profiles were taken with
READS_CONFIGS = {"default": None,
                 "profiled": dict(wf_min_cells=1 << 20, wf_waves_per_cu=8, wf_orient=-1)}
PROTEIN_CONFIGS = {"default": None,
                   "profiled": dict(wf_min_cells=1, wf_waves_per_cu=24, wf_orient=2, wf_group=1),
                   "grouped": dict(wf_min_cells=1 << 12, wf_waves_per_cu=16, wf_orient=2, wf_group=4)}


def _cigar_string(runs):
    return "".join("%d%s" % (n, "MID"[op]) for n, op in runs)


def _run(w, flags, config):
    import torch

    import paper_2002_04561_amd as aln
    n, m = w.lengths()
    q, qo, s, so = aln.to_device(w)
    cfg = aln.BatchConfig(**config) if config else None
    ba = aln.BatchAligner(aln.scoring_of(w), q, qo, s, so, int(n.max()), int(m.max()), flags, config=cfg)
    ba.run()
    torch.cuda.synchronize()
    return ba


def _check_digests(w, ba, res, name):
    """Chunk digests of every pair's results against the oracle's stored digests."""
    g = json.load(open(os.path.join(HERE, "golden", name)))
    assert g["n_pairs"] == w.n_pairs and g["workload"] == w.name and g["chunk"] == digest.CHUNK
    if w.traceback:
        cig = ba.cigar.to("cpu").numpy().view(np.uint32)
        d = digest.chunk_digests(res, True, cig, ba.cigar_off.to("cpu").numpy())
    else:
        d = digest.chunk_digests(res, False)
    bad = [c for c, (x, y) in enumerate(zip(d, g["digests"])) if x != y]
    assert len(d) == len(g["digests"]) and not bad, "chunks of %d pairs differing from the oracle: %s" % (
        digest.CHUNK, bad[:20])


def _check_all(w, res):
    n, m = w.lengths()
    import paper_2002_04561_amd as aln
    assert not np.any(res["flags"] & ~np.uint32(aln.RES_INT32_REDO)), "error flags set"  # a redo is not an error
    assert np.all((res["q_end"] >= 0) & (res["q_end"] <= n) & (res["s_end"] >= 0) & (res["s_end"] <= m))


@pytest.fixture(scope="module")
def reads():
    return synth.reads_semiglobal(n_pairs=1 << 20)


@pytest.fixture(scope="module")
def protein():
    return synth.protein_uneven(n_pairs=65536)


@pytest.mark.parametrize("cfg", list(READS_CONFIGS))
def test_reads_full_batch(gpu, reads, cfg):
    import paper_2002_04561_amd as aln
    golden = json.load(open(os.path.join(HERE, "golden", "reads_sample.json")))
    assert golden["n_pairs"] == reads.n_pairs and golden["workload"] == reads.name
    ba = _run(reads, aln.TRACEBACK, READS_CONFIGS[cfg])
    res = ba.results()
    _check_all(reads, res)
    idx = [int(e["k"]) for e in golden["pairs"]]
    cig = ba.cigars(idx)
    sample_bad = []
    for e in golden["pairs"]:
        k = int(e["k"])
        g = (int(res["score"][k]), int(res["q_begin"][k]), int(res["q_end"][k]), int(res["s_begin"][k]),
             int(res["s_end"][k]), _cigar_string(cig[k]))
        o = (e["score"], e["q_begin"], e["q_end"], e["s_begin"], e["s_end"], e["cigar"])
        if g != o:
            sample_bad.append((cfg, k, g, o))
    assert not sample_bad, sample_bad[:4]
    _check_digests(reads, ba, res, "reads_digest.json")


@pytest.mark.parametrize("cfg", list(PROTEIN_CONFIGS))
def test_protein_full_batch(gpu, protein, cfg):
    import paper_2002_04561_amd as aln
    golden = json.load(open(os.path.join(HERE, "golden", "protein_sample.json")))
    assert golden["n_pairs"] == protein.n_pairs and golden["workload"] == protein.name
    ba = _run(protein, aln.SCORE_ONLY, PROTEIN_CONFIGS[cfg])
    res = ba.results()
    _check_all(protein, res)
    for e in golden["pairs"]:
        k = int(e["k"])
        g = (int(res["score"][k]), int(res["q_end"][k]), int(res["s_end"][k]))
        assert g == (e["score"], e["q_end"], e["s_end"]), (cfg, k, g)
    _check_digests(protein, ba, res, "protein_digest.json")
