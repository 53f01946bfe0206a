"""The autotuner's search, with no device: a fake batch and a timer that is a known function of the
configuration.  It searches one coordinate at a time from the library's defaults in the order of
tune.SEARCH, keeps a candidate only when it is faster, never tries thresholds that would leave a pair
above LANE_CELLS_MAX cells on one lane, and caches the winner under the workload's signature."""
import numpy as np
import pytest
import torch

from paper_2002_04561_amd import BatchConfig, tune


class _FakeBatch:
    def __init__(self, n, m, flags=0, mode=1, go=-11, alphabet=20):
        qo = np.zeros(len(n) + 1, np.int64)
        so = np.zeros(len(m) + 1, np.int64)
        np.cumsum(n, out=qo[1:])
        np.cumsum(m, out=so[1:])
        self.q_off, self.s_off = torch.from_numpy(qo), torch.from_numpy(so)
        self.flags = flags
        self.scoring = type("S", (), {"mode": mode, "gap_open": go, "alphabet_size": alphabet})()
        self.config = None
        self.runs = 0

    def run(self, stream=None):
        self.runs += 1


@pytest.fixture(autouse=True)
def _clean_cache():
    tune._CACHE.clear()
    yield
    tune._CACHE.clear()


def _timer(costs, seen):
    """A stand-in for tune._time: milliseconds as a sum of per-field costs."""
    fields = {f for f, _ in costs}

    def fake(ba, cfg, stream, repeats, cutoff):
        seen.append(cfg)
        ba.config = cfg
        return 100.0 + sum(costs.get((f, getattr(cfg, f)), 0.0) for f in fields)
    return fake


def test_coordinate_search_keeps_only_improvements(monkeypatch):
    costs = {("wf_min_cells", 1 << 12): -30.0, ("wf_waves_per_cu", 24): -5.0, ("wf_waves_per_cu", 8): +50.0,
             ("wf_orient", 2): -7.0, ("wf_group", 4): +3.0, ("small_bits", 32): +1.0, ("wf_bits", 16): +2.0}
    seen = []
    monkeypatch.setattr(tune, "_time", _timer(costs, seen))
    n = np.full(256, 300)
    ba = _FakeBatch(n, n)
    cfg, table = tune.tune(ba, stream=object())
    # wf_group 1 ties the default 0 and small_bits/wf_bits only lose: only strict improvements are kept
    assert cfg == BatchConfig(wf_min_cells=1 << 12, wf_waves_per_cu=24, wf_orient=2, small_bits=16, wf_group=0,
                              wf_bits=32)
    assert ba.config == cfg
    # every candidate differs from the best so far in one field, and the fields come in tune.SEARCH order
    fields = [f for f, _ in tune.SEARCH]
    timer = _timer(costs, [])
    best, best_ms, last = seen[0], timer(ba, seen[0], None, 0, 0), -1
    for c in seen[1:]:
        diff = [f for f in fields if getattr(c, f) != getattr(best, f)]
        assert len(diff) == 1, (best, c)
        assert fields.index(diff[0]) >= last
        last = fields.index(diff[0])
        ms = timer(ba, c, None, 0, 0)
        if ms < best_ms:
            best, best_ms = c, ms
    assert best == cfg
    assert len(table) == len(seen)


def test_lane_cell_limit_skips_thresholds(monkeypatch):
    seen = []
    monkeypatch.setattr(tune, "_time", _timer({}, seen))
    n = np.array([100, 5000])  # the second pair has 2.5e7 cells, above LANE_CELLS_MAX
    ba = _FakeBatch(n, n)
    tune.tune(ba, stream=object())
    tried = {c.wf_min_cells for c in seen}
    assert all(0 < v <= tune.LANE_CELLS_MAX for v in tried)
    assert -1 not in tried and (1 << 20) in tried


def test_cache_by_signature(monkeypatch):
    seen = []
    monkeypatch.setattr(tune, "_time", _timer({("wf_orient", 1): -1.0}, seen))
    n = np.full(64, 200)
    tune.tune(_FakeBatch(n, n), stream=object())
    first = len(seen)
    cfg2, _ = tune.tune(_FakeBatch(n, n), stream=object())  # same signature: no timing
    assert len(seen) == first and cfg2.wf_orient == 1
    tune.tune(_FakeBatch(n * 40, n * 40), stream=object())  # other cell histogram: searched again
    assert len(seen) > first


def test_signature_depends_on_workload_not_on_order():
    sc = type("S", (), {"mode": 1, "gap_open": -11, "alphabet_size": 20})()
    n = np.array([10, 2000, 300])
    m = np.array([50, 100, 4000])
    a = tune.signature(sc, 0, n, m)
    assert a == tune.signature(sc, 0, n[::-1], m[::-1])
    assert a != tune.signature(sc, 1, n, m)
    assert a != tune.signature(sc, 0, n * 3, m)
