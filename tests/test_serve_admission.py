"""Admission logic of the serving loop, with no device: budget accounting, FIFO order, queuing."""
import numpy as np
import pytest

from paper_2002_04561_amd.serve import Admission, Request, request_bytes


def _req(rid, klass, n, m, t, tb=False, long=False):
    return Request(rid, klass, np.zeros(n, np.uint8), np.zeros(m, np.uint8), t, tb, long)


def test_budget_never_exceeded_and_fifo():
    rng = np.random.default_rng(1)
    reqs = [_req(k, "a" if k % 3 else "b", int(rng.integers(1, 300)), int(rng.integers(1, 300)), k * 1e-3,
                 tb=bool(k % 2)) for k in range(400)]
    budget = 4 * max(request_bytes(r) for r in reqs)
    adm = Admission(budget)
    for r in reqs:
        adm.arrive(r)
    seen = {"a": [], "b": []}
    inflight = []
    while adm.pending() or inflight:
        k = adm.oldest_class()
        batch = adm.take_batch(k, 16) if k else []
        assert adm.in_use <= budget
        if batch:
            seen[k] += [r.rid for r in batch]
            inflight.append(batch)
        if not batch or len(inflight) > 2:
            adm.release(inflight.pop(0))
    assert adm.in_use == 0 and adm.peak <= budget
    for k in seen:  # every request once, in arrival order within its class
        ids = [r.rid for r in reqs if r.klass == k]
        assert seen[k] == ids


def test_tiny_budget_queues_without_loss():
    reqs = [_req(k, "a", 200, 200, 0.0, tb=True) for k in range(20)]
    adm = Admission(request_bytes(reqs[0]) + 10)  # one request at a time
    for r in reqs:
        adm.arrive(r)
    done = 0
    while adm.pending():
        b = adm.take_batch("a", 8)
        assert len(b) == 1
        adm.release(b)
        done += 1
    assert done == 20


def test_long_requests_run_alone_and_oversize_refused():
    adm = Admission(10 ** 9)
    adm.arrive(_req(0, "x", 100, 100, 0.0, long=True))
    adm.arrive(_req(1, "x", 100, 100, 0.1, long=True))
    assert len(adm.take_batch("x", 8)) == 1
    with pytest.raises(ValueError):
        Admission(100).arrive(_req(2, "x", 1000, 1000, 0.0, tb=True))


def test_oldest_class_skips_excluded_classes():
    """A class at its in-flight cap is passed over: the oldest waiting request of the other classes goes next,
    and nothing is chosen when only excluded classes wait."""
    adm = Admission(1 << 30)
    adm.arrive(_req(0, "long", 64, 64, 0.0))
    adm.arrive(_req(1, "read", 10, 12, 0.5))
    adm.arrive(_req(2, "protein", 30, 20, 0.7))
    assert adm.oldest_class() == "long"
    assert adm.oldest_class(exclude={"long"}) == "read"
    assert adm.oldest_class(exclude={"long", "read"}) == "protein"
    assert adm.oldest_class(exclude={"long", "read", "protein"}) is None


def test_longest_prefix_under_a_given_cost():
    """With a cost passed in, a batch is the longest FIFO prefix whose cost fits what is left, found by
    bisection; the charge is the cost of the batch taken, and release returns exactly that."""
    from paper_2002_04561_amd.serve import BatchShape
    calls = []

    def cost(b: BatchShape) -> int:
        calls.append(b.n_pairs)
        return 1000 + 10 * b.total_q + b.max_m  # grows with every added request
    reqs = [_req(k, "a", 10 + k, 20, k * 1e-3) for k in range(100)]
    adm = Admission(5000, cost)
    for r in reqs:
        adm.arrive(r)
    calls.clear()
    first = adm.take_batch("a", 64)
    assert len(calls) < 10  # bisection, not one call per request
    k = len(first)
    tq = sum(10 + j for j in range(k))
    assert cost(BatchShape("a", k, tq, 20 * k, 9 + k, 20, 0, False, False)) <= 5000
    tq2 = tq + 10 + k
    assert 1000 + 10 * tq2 + 20 > 5000  # one more would not fit
    assert adm.in_use == 1000 + 10 * tq + 20
    adm.release(first)
    assert adm.in_use == 0
