"""Continuous-batching alignment server over the mialign C ABI.

Requests (one pair each, of a named class with its own scoring scheme) arrive over time.  The
server keeps up to `streams` batches in flight on separate HIP streams, so batches launched while
others run overlap on the device.  Whenever a stream is free it forms the next batch from the
requests that have arrived, oldest class first, and admits requests in arrival order while the
device memory they need stays within the budget; a request that does not fit waits for memory to
be released by finishing batches.  Sequences are copied once into device memory at admission and
stay there until their batch completes.

Memory a request holds while admitted (bytes):
    sequences n + m, offsets and result 48, CIGAR 4 (n + m) when traced back, plus the DP/traceback
    state of its path: a wavefront pair keeps two rows of (m + 1) x 8 bytes (and n*m/2 bytes of
    predecessor codes when traced back); a pair of a batch shares the batch kernel's per-wave row
    buffers, counted as 8 (m + 1) bytes per pair, and with traceback its predecessor codes n*m/2.

The admission logic (`Admission`) is plain Python so it can be exercised without a device.
"""
from __future__ import annotations

import collections
import time
from dataclasses import dataclass, field
from typing import Dict, List, Optional

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
    n, m = len(r.q), len(r.s)
    b = n + m + 48
    if r.traceback:
        b += 4 * (n + m) + (n * m + 1) // 2
    b += 16 * (m + 1) if r.long else 8 * (m + 1)
    return b


class Admission:
    """FIFO-per-class admission against a byte budget.  Pure bookkeeping, no device."""

    def __init__(self, budget_bytes: int):
        self.budget = int(budget_bytes)
        self.in_use = 0
        self.peak = 0
        self.waiting: Dict[str, collections.deque] = collections.defaultdict(collections.deque)

    def arrive(self, r: Request):
        if request_bytes(r) > self.budget:
            raise ValueError("request %d needs %d bytes, more than the whole budget" % (r.rid, request_bytes(r)))
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
        """Admits the longest FIFO prefix of `klass` that fits the budget (a long request goes alone)."""
        dq = self.waiting[klass]
        out: List[Request] = []
        while dq and len(out) < max_pairs:
            r = dq[0]
            need = request_bytes(r)
            if self.in_use + need > self.budget:
                break
            if r.long and out:
                break
            dq.popleft()
            self.in_use += need
            self.peak = max(self.peak, self.in_use)
            out.append(r)
            if r.long:
                break
        return out

    def release(self, batch: List[Request]):
        for r in batch:
            self.in_use -= request_bytes(r)
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
        self.adm = Admission(budget_bytes)
        self.streams = [torch.cuda.Stream(device=device) for _ in range(streams)]
        self.max_pairs = max_pairs
        self.class_max_pairs = dict(class_max_pairs or {})
        self.class_configs = dict(class_configs or {})  # per class: a BatchConfig (execution choices only)
        self.class_max_streams = dict(class_max_streams or {})  # per class: most batches in flight at once
        self.device = device
        self.completed: List[Completed] = []
        self.cells = 0
        self.redo = 0  # requests whose 16-bit pass was redone in 32 bits

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
