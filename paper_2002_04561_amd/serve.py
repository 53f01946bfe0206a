"""Continuous-batching alignment server over the mialign C ABI.

Requests (one pair each, of a named class with its own scoring scheme) arrive over time.  The
server keeps up to `streams` batches in flight on separate HIP streams, so batches launched while
others run overlap on the device.  Whenever a stream is free it forms the next batch from the
requests that have arrived, oldest class first, and admits requests in arrival order while the
device memory they need stays within the budget; a request that does not fit waits for memory to
be released by finishing batches.  Sequences are copied once into device memory at admission and
stay there until their batch completes.

Memory a batch holds while in flight is what its calls allocate on the device: the workspace the
library's size query asks for (aln_batch_workspace_size, or aln_long_workspace_size for a request that
runs alone), plus the sequences, offsets, results and CIGAR buffers, each rounded up to the caching
allocator's 512-byte blocks (`AlignServer.batch_bytes`).  Admission takes the longest FIFO prefix of
a class whose batch fits what the budget has left.

The admission logic (`Admission`) is plain Python with the cost of a batch passed in, so it can be
exercised without a device; `request_bytes` is the stand-alone estimate it uses when no cost is given.
"""
from __future__ import annotations

import collections
import time
from dataclasses import dataclass, field
from typing import Callable, Dict, List, Optional

import numpy as np


@dataclass
class Request:
    rid: int
    klass: str
    q: np.ndarray
    s: np.ndarray
    arrival: float  # seconds from the start of the run
    traceback: bool = False
    long: bool = False  # run alone on the wavefront engine (aln_align_long)


def request_bytes(r: Request) -> int:
    """A device-free estimate of one request's memory: sequences, offsets and result, CIGAR room, two DP
    rows, and the 4-bit codes of every cell when traced back."""
    n, m = len(r.q), len(r.s)
    b = n + m + 48
    if r.traceback:
        b += 4 * (n + m) + (n * m + 1) // 2
    b += 16 * (m + 1) if r.long else 8 * (m + 1)
    return b


@dataclass
class BatchShape:
    """What the memory of a batch of one class depends on."""
    klass: str
    n_pairs: int
    total_q: int
    total_s: int
    max_n: int
    max_m: int
    cells: int  # sum of n * m
    traceback: bool
    long: bool


def estimate_bytes(b: BatchShape) -> int:
    """The sum of request_bytes over the batch's requests."""
    x = b.total_q + b.total_s + 48 * b.n_pairs + (16 if b.long else 8) * (b.total_s + b.n_pairs)
    if b.traceback:
        x += 4 * (b.total_q + b.total_s) + (b.cells + b.n_pairs) // 2
    return x


class Admission:
    """FIFO-per-class admission against a byte budget.  Pure bookkeeping, no device.

    cost(shape) gives the bytes a batch of that shape (all of one class) holds on the device; it must not
    shrink when a request is added.  The default, estimate_bytes, sums request_bytes."""

    def __init__(self, budget_bytes: int, cost: Optional[Callable[[BatchShape], int]] = None):
        self.budget = int(budget_bytes)
        self.cost = cost or estimate_bytes
        self.in_use = 0
        self.peak = 0
        self.waiting: Dict[str, collections.deque] = collections.defaultdict(collections.deque)
        self.charged: Dict[int, int] = {}  # id(batch) -> bytes charged

    @staticmethod
    def shapes(reqs: List[Request]):
        """shape(k): the BatchShape of the first k requests (prefix sums and maxima computed once)."""
        n = np.fromiter((len(r.q) for r in reqs), np.int64, len(reqs))
        m = np.fromiter((len(r.s) for r in reqs), np.int64, len(reqs))
        cq, cs, cc = np.cumsum(n), np.cumsum(m), np.cumsum(n * m)
        mn, mm = np.maximum.accumulate(n), np.maximum.accumulate(m)
        r0 = reqs[0]

        def shape(k: int) -> BatchShape:
            return BatchShape(r0.klass, k, int(cq[k - 1]), int(cs[k - 1]), int(mn[k - 1]), int(mm[k - 1]),
                              int(cc[k - 1]), r0.traceback, r0.long)
        return shape

    def arrive(self, r: Request):
        need = self.cost(self.shapes([r])(1))
        if need > self.budget:
            raise ValueError("request %d needs %d bytes, more than the whole budget" % (r.rid, need))
        self.waiting[r.klass].append(r)

    def oldest_class(self, exclude=()) -> Optional[str]:
        best, t = None, None
        for k, dq in self.waiting.items():
            if k in exclude:
                continue
            if dq and (t is None or dq[0].arrival < t):
                best, t = k, dq[0].arrival
        return best

    def take_batch(self, klass: str, max_pairs: int) -> List[Request]:
        """Admits the longest FIFO prefix of `klass` whose batch fits what the budget has left (a long
        request goes alone).  The prefix length is found by bisection, the cost being monotone in it."""
        dq = self.waiting[klass]
        if not dq:
            return []
        room = self.budget - self.in_use
        if dq[0].long:
            cand = [dq[0]]
        else:
            cand = []
            for r in dq:
                if r.long or len(cand) >= max_pairs:
                    break
                cand.append(r)
        shape = self.shapes(cand)
        lo, hi = 0, len(cand)  # the largest k whose batch fits the room left
        while lo < hi:
            mid = (lo + hi + 1) // 2
            if self.cost(shape(mid)) <= room:
                lo = mid
            else:
                hi = mid - 1
        if lo == 0:
            return []
        out = [dq.popleft() for _ in range(lo)]
        need = self.cost(shape(lo))
        self.in_use += need
        self.peak = max(self.peak, self.in_use)
        self.charged[id(out)] = need
        return out

    def release(self, batch: List[Request]):
        self.in_use -= self.charged.pop(id(batch))
        assert self.in_use >= 0

    def pending(self) -> int:
        return sum(len(d) for d in self.waiting.values())


@dataclass
class Completed:
    rid: int
    klass: str
    latency: float
    result: tuple
    cigar: Optional[list] = None


@dataclass
class _Flight:
    batch: List[Request]
    stream: object
    event: object
    tensors: list = field(default_factory=list)
    out: object = None
    cigar: object = None
    cigar_off: Optional[np.ndarray] = None


class AlignServer:
    """Runs a request stream through aln_align_batch / aln_align_long with continuous batching."""

    def __init__(self, scorings: Dict[str, object], budget_bytes: int, streams: int = 3, max_pairs: int = 8192,
                 device: str = "cuda", class_max_pairs: Optional[Dict[str, int]] = None,
                 class_configs: Optional[Dict[str, object]] = None, class_max_streams: Optional[Dict[str, int]] = None):
        import torch

        import paper_2002_04561_amd as aln
        self.torch, self.aln = torch, aln
        self.scorings = scorings
        self.adm = Admission(budget_bytes, self.batch_bytes)
        self.streams = [torch.cuda.Stream(device=device) for _ in range(streams)]
        self.max_pairs = max_pairs
        self.class_max_pairs = dict(class_max_pairs or {})
        self.class_configs = dict(class_configs or {})  # per class: a BatchConfig (execution choices only)
        self.class_max_streams = dict(class_max_streams or {})  # per class: most batches in flight at once
        self.device = device
        self.completed: List[Completed] = []
        self.cells = 0
        self.redo = 0  # requests whose 16-bit pass was redone in 32 bits

    def batch_bytes(self, b: BatchShape) -> int:
        """Device bytes a batch allocates while in flight: the library's workspace for it (its size query)
        and the buffers _launch creates, each rounded up to the allocator's 512-byte blocks."""
        aln = self.aln
        blk = lambda x: (max(int(x), 1) + 511) // 512 * 512  # noqa: E731
        sc = self.scorings[b.klass]
        flags = aln.TRACEBACK if b.traceback else aln.SCORE_ONLY
        if b.long:
            ws = aln.aln_long_workspace_size(sc, b.total_q, b.total_s, flags)
            x = blk(max(ws, 256)) + blk(b.total_q) + blk(b.total_s) + blk(32)
            return x + (blk(4 * (b.total_q + b.total_s + 1)) if b.traceback else 0)
        ws = aln.aln_batch_workspace_size(sc, b.n_pairs, b.max_n, b.max_m, b.total_q, b.total_s, flags)
        x = blk(max(ws, 256)) + blk(b.total_q) + blk(b.total_s) + 2 * blk(8 * (b.n_pairs + 1)) + blk(32 * b.n_pairs)
        if b.traceback:
            x += blk(4 * (b.total_q + b.total_s + b.n_pairs)) + blk(8 * (b.n_pairs + 1))
        return x

    def _launch(self, batch: List[Request], stream) -> _Flight:
        torch, aln = self.torch, self.aln
        sc = self.scorings[batch[0].klass]
        qs = [r.q for r in batch]
        ss = [r.s for r in batch]
        qo = np.zeros(len(batch) + 1, np.int64)
        so = np.zeros(len(batch) + 1, np.int64)
        np.cumsum([len(x) for x in qs], out=qo[1:])
        np.cumsum([len(x) for x in ss], out=so[1:])
        qcat = np.concatenate(qs) if qo[-1] else np.zeros(1, np.uint8)
        scat = np.concatenate(ss) if so[-1] else np.zeros(1, np.uint8)
        tb = batch[0].traceback
        flags = aln.TRACEBACK if tb else aln.SCORE_ONLY
        f = _Flight(batch, stream, torch.cuda.Event())
        with torch.cuda.stream(stream):
            # admission-time copies: pinned staging, asynchronous on this batch's stream
            hq = torch.from_numpy(qcat).pin_memory()
            hs = torch.from_numpy(scat).pin_memory()
            q = hq.to(self.device, non_blocking=True)
            s = hs.to(self.device, non_blocking=True)
            if batch[0].long:
                r = batch[0]
                la = aln.LongAligner(sc, q[:len(r.q)], s[:len(r.s)], flags, device=self.device)
                la.run(stream)
                f.out, f.cigar = la.out, la.cigar
                f.tensors = [hq, hs, q, s, la]
            else:
                dqo = torch.from_numpy(qo).pin_memory().to(self.device, non_blocking=True)
                dso = torch.from_numpy(so).pin_memory().to(self.device, non_blocking=True)
                cap = None
                if tb:
                    cap = np.maximum((qo[1:] - qo[:-1]) + (so[1:] - so[:-1]), 1)
                    f.cigar_off = np.zeros(len(batch) + 1, np.int64)
                    np.cumsum(cap, out=f.cigar_off[1:])
                ba = aln.BatchAligner(sc, q, dqo, s, dso, int(max(len(x) for x in qs)),
                                      int(max(len(x) for x in ss)), flags, cigar_capacity=cap, device=self.device,
                                      total_q=int(qo[-1]), total_s=int(so[-1]),
                                      config=self.class_configs.get(batch[0].klass))
                ba.run(stream)
                f.out, f.cigar = ba.out, ba.cigar
                f.tensors = [hq, hs, q, s, dqo, dso, ba]
            f.event.record(stream)
        self.cells += sum(len(r.q) * len(r.s) for r in batch)
        return f

    def _finish(self, f: _Flight, t0: float):
        now = time.perf_counter() - t0
        res = f.out.to("cpu").numpy().view(self.aln.RESULT_DTYPE)
        cig = f.cigar.to("cpu").numpy().view(np.uint32) if f.cigar is not None else None
        # whole columns at once: indexing structured rows field by field costs microseconds per request
        redo_bit = self.aln.RES_INT32_REDO
        flags = res["flags"].astype(np.int64)
        self.redo += int(np.count_nonzero(flags & redo_bit))
        cols = zip(res["score"].tolist(), res["q_begin"].tolist(), res["q_end"].tolist(), res["s_begin"].tolist(),
                   res["s_end"].tolist(), (flags & ~redo_bit).tolist())
        lens = res["cigar_len"].tolist()
        bases = f.cigar_off.tolist() if f.cigar_off is not None else [0] * len(f.batch)
        for k, (r, tup) in enumerate(zip(f.batch, cols)):
            runs = None
            if cig is not None:
                runs = [(w >> 4, w & 15) for w in cig[bases[k]:bases[k] + lens[k]].tolist()]
            self.completed.append(Completed(r.rid, r.klass, now - r.arrival, tup, runs))
        self.adm.release(f.batch)

    def run(self, requests: List[Request], realtime: bool = True) -> dict:
        """Serves the stream; arrival times are honoured against the wall clock when realtime."""
        torch = self.torch
        order = sorted(requests, key=lambda r: r.arrival)
        t0 = time.perf_counter()
        nxt = 0
        flights: List[Optional[_Flight]] = [None] * len(self.streams)
        while nxt < len(order) or self.adm.pending() or any(flights):
            now = time.perf_counter() - t0
            while nxt < len(order) and (not realtime or order[nxt].arrival <= now):
                self.adm.arrive(order[nxt])
                nxt += 1
            for i, f in enumerate(flights):
                if f is not None and f.event.query():
                    self._finish(f, t0)
                    flights[i] = None
            launched = False
            for i in range(len(flights)):
                if flights[i] is None:
                    busy = collections.Counter(f.batch[0].klass for f in flights if f is not None)
                    full = {c for c, cap in self.class_max_streams.items() if busy[c] >= cap}
                    k = self.adm.oldest_class(exclude=full)
                    if k is None:
                        break
                    batch = self.adm.take_batch(k, self.class_max_pairs.get(k, self.max_pairs))
                    if not batch:
                        break
                    flights[i] = self._launch(batch, self.streams[i])
                    launched = True
            if not launched:
                time.sleep(0.0002)
        torch.cuda.synchronize()
        wall = time.perf_counter() - t0
        stats = {"requests": len(self.completed), "wall_s": wall, "cells": self.cells,
                 "gcups": self.cells / wall / 1e9, "peak_bytes": self.adm.peak, "budget_bytes": self.adm.budget,
                 "int32_redo": self.redo, "classes": {}}
        by = collections.defaultdict(list)
        for c in self.completed:
            by[c.klass].append(c.latency)
        for k, v in by.items():
            a = np.array(v) * 1e3
            stats["classes"][k] = {"n": len(v), "p50_ms": float(np.percentile(a, 50)),
                                   "p99_ms": float(np.percentile(a, 99))}
        return stats
