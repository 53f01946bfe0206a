"""Seeded synthetic workloads for pairwise alignment.

This module only draws sequences (and the protein substitution table) from a
seeded numpy PCG64 generator and packs them into concatenated code arrays with
int64 offsets.  It contains no alignment arithmetic; both the HIP library's
tests/benchmark and the CPU oracle read the same arrays.

Codes: DNA A,C,G,T = 0..3; protein = 0..19.

Workloads (stand-ins for the paper's data, which is not available here):
  long_dna_global_1k   1 pair, n = m = 1000, uniform ACGT; global, +2/-1, linear gap -1
                       (the scheme of the C example in Sec. III-C).
  long_dna_local_256k  1 pair, n = m = 262144; the second sequence is the first mutated with
                       5% substitutions and 1% indels of geometric length (mean 3), then cut or
                       padded to 262144; local affine, open -3 / extend -1, +2/-3.  Stands in for
                       the long genome pairs of Table I.
  reads_semiglobal     read/window pairs: read length L ~ U{100..250}, window uniform ACGT of
                       length L+64, read = window[o:o+L] (o ~ U{0..64}) mutated with 2%
                       substitutions and 0.5% single-base indels; semi-global affine -5/-2,
                       +1/-4.  Stands in for the simulated 150 bp Illumina reads of Sec. V.
  protein_uneven       pairs with n, m independent, round(exp(U(ln 64, ln 16384))), uniform over
                       20 letters, unrelated; symmetric 20x20 table with diagonal U{4..11} and
                       off-diagonal U{-4..3}; local affine -11/-1.
"""
from __future__ import annotations

from dataclasses import dataclass
from typing import Optional

import numpy as np

GLOBAL, LOCAL, SEMIGLOBAL = 0, 1, 2


@dataclass
class Workload:
    name: str
    mode: int
    alphabet_size: int
    gap_open: int
    gap_extend: int
    q: np.ndarray       # uint8 concatenated query codes
    q_off: np.ndarray   # int64, n_pairs + 1
    s: np.ndarray       # uint8 concatenated subject codes
    s_off: np.ndarray   # int64, n_pairs + 1
    match: Optional[int] = None
    mismatch: Optional[int] = None
    subst: Optional[np.ndarray] = None  # (A, A) int8 when a table is used
    traceback: bool = False

    @property
    def n_pairs(self) -> int:
        return len(self.q_off) - 1

    def lengths(self):
        return (self.q_off[1:] - self.q_off[:-1]), (self.s_off[1:] - self.s_off[:-1])

    def cells(self) -> int:
        n, m = self.lengths()
        return int(np.sum(n.astype(np.int64) * m.astype(np.int64)))

    def pair(self, k: int):
        return (self.q[self.q_off[k]:self.q_off[k + 1]], self.s[self.s_off[k]:self.s_off[k + 1]])

    def subset(self, idx) -> "Workload":
        idx = np.asarray(idx, dtype=np.int64)
        q, qo = _gather(self.q, self.q_off, idx)
        s, so = _gather(self.s, self.s_off, idx)
        return Workload(self.name, self.mode, self.alphabet_size, self.gap_open, self.gap_extend, q, qo, s, so,
                        self.match, self.mismatch, self.subst, self.traceback)

    def sigma_table(self) -> np.ndarray:
        """Full (A, A) table of the scheme (a workload description, used by the oracle side)."""
        if self.subst is not None:
            return self.subst.astype(np.int32)
        t = np.full((self.alphabet_size, self.alphabet_size), self.mismatch, dtype=np.int32)
        np.fill_diagonal(t, self.match)
        return t


def _gather(codes, off, idx):
    lens = off[idx + 1] - off[idx]
    new_off = np.zeros(len(idx) + 1, dtype=np.int64)
    np.cumsum(lens, out=new_off[1:])
    out = np.empty(int(new_off[-1]), dtype=np.uint8)
    for k, p in enumerate(idx):
        out[new_off[k]:new_off[k + 1]] = codes[off[p]:off[p + 1]]
    return out, new_off


def pack(seqs) -> tuple:
    """Concatenates a list of code arrays into (codes uint8, offsets int64)."""
    lens = np.array([len(x) for x in seqs], dtype=np.int64)
    off = np.zeros(len(seqs) + 1, dtype=np.int64)
    np.cumsum(lens, out=off[1:])
    codes = np.concatenate([np.asarray(x, dtype=np.uint8) for x in seqs]) if len(seqs) else np.zeros(0, np.uint8)
    return codes.astype(np.uint8, copy=False), off


def mutate_geometric(rng: np.random.Generator, src: np.ndarray, p_sub: float, p_indel: float, mean_len: float,
                     alphabet: int = 4) -> np.ndarray:
    """Walks src: substitution with p_sub (uniform over the other letters), an indel with p_indel
    (insertion of random letters or deletion of source letters, 1/2 each, length Geometric(1/mean_len)
    on {1,2,...}), else copy."""
    n = len(src)
    u = rng.random(n)
    ev = np.nonzero(u < p_indel)[0]
    sub = (u >= p_indel) & (u < p_indel + p_sub)
    out_src = src.copy()
    shift = rng.integers(1, alphabet, n, dtype=np.uint8)
    out_src[sub] = ((out_src[sub].astype(np.int64) + shift[sub]) % alphabet).astype(np.uint8)
    pieces = []
    pos = 0
    is_ins = rng.random(len(ev)) < 0.5
    lens = rng.geometric(1.0 / mean_len, len(ev))
    for k, e in enumerate(ev):
        if e < pos:
            continue  # inside a previous deletion
        pieces.append(out_src[pos:e])
        if is_ins[k]:
            pieces.append(rng.integers(0, alphabet, int(lens[k]), dtype=np.uint8))
            pos = e
        else:
            pos = e + int(lens[k])
    pieces.append(out_src[pos:])
    return np.concatenate(pieces).astype(np.uint8)


def long_dna_global_1k(seed: int = 1) -> Workload:
    rng = np.random.default_rng(seed)
    a = rng.integers(0, 4, 1000, dtype=np.uint8)
    b = rng.integers(0, 4, 1000, dtype=np.uint8)
    q, qo = pack([a])
    s, so = pack([b])
    return Workload("long_dna_global_1k", GLOBAL, 4, 0, -1, q, qo, s, so, match=2, mismatch=-1, traceback=True)


def long_dna_local(seed: int = 2, n: int = 262144) -> Workload:
    rng = np.random.default_rng(seed)
    a = rng.integers(0, 4, n, dtype=np.uint8)
    b = mutate_geometric(rng, a, 0.05, 0.01, 3.0)
    if len(b) >= n:
        b = b[:n]
    else:
        b = np.concatenate([b, rng.integers(0, 4, n - len(b), dtype=np.uint8)])
    q, qo = pack([a])
    s, so = pack([b])
    return Workload("long_dna_local_%d" % n, LOCAL, 4, -3, -1, q, qo, s, so, match=2, mismatch=-3)


def _reads_chunk(rng: np.random.Generator, n_pairs: int, lmin: int, lmax: int, pad: int, p_sub: float,
                 p_indel: float):
    L = rng.integers(lmin, lmax + 1, n_pairs).astype(np.int64)
    wlen = L + pad
    s_off = np.zeros(n_pairs + 1, dtype=np.int64)
    np.cumsum(wlen, out=s_off[1:])
    s = rng.integers(0, 4, int(s_off[-1]), dtype=np.uint8)
    o = rng.integers(0, pad + 1, n_pairs).astype(np.int64)
    src_off = np.zeros(n_pairs + 1, dtype=np.int64)
    np.cumsum(L, out=src_off[1:])
    tot = int(src_off[-1])
    pair_of = np.repeat(np.arange(n_pairs, dtype=np.int64), L)
    t = np.arange(tot, dtype=np.int64) - src_off[pair_of]
    src = s[s_off[pair_of] + o[pair_of] + t]          # read source = window[o : o + L]
    u = rng.random(tot)
    indel = u < p_indel
    sub = (u >= p_indel) & (u < p_indel + p_sub)
    ins = indel & (rng.random(tot) < 0.5)
    dele = indel & ~ins
    shift = rng.integers(1, 4, tot, dtype=np.uint8)
    src[sub] = ((src[sub] + shift[sub]) % 4).astype(np.uint8)
    # each source letter emits 0 (deleted), 1 (copied or substituted) or 2 (a random letter, then itself)
    cnt = np.ones(tot, dtype=np.int64)
    cnt[dele] = 0
    cnt[ins] = 2
    q_lens = np.add.reduceat(cnt, src_off[:-1])
    q_off = np.zeros(n_pairs + 1, dtype=np.int64)
    np.cumsum(q_lens, out=q_off[1:])
    ends = np.cumsum(cnt)
    keep = cnt > 0
    q = np.empty(int(q_off[-1]), dtype=np.uint8)
    q[ends[keep] - 1] = src[keep]
    ins_pos = ends[ins] - 2
    q[ins_pos] = rng.integers(0, 4, len(ins_pos), dtype=np.uint8)
    return q, q_off, s, s_off


READS_CHUNK = 16384


def reads_semiglobal(seed: int = 3, n_pairs: int = 1 << 20, lmin: int = 100, lmax: int = 250, pad: int = 64,
                     p_sub: float = 0.02, p_indel: float = 0.005) -> Workload:
    """Read/window pairs (single-letter indels), drawn in independent chunks of READS_CHUNK pairs,
    chunk c from PCG64 seeded with [seed, c]; so the first k pairs do not depend on n_pairs."""
    qs, qos, ss, sos = [], [], [], []
    for c in range((n_pairs + READS_CHUNK - 1) // READS_CHUNK):
        rng = np.random.default_rng([seed, c])
        q, qo, s, so = _reads_chunk(rng, READS_CHUNK, lmin, lmax, pad, p_sub, p_indel)
        take = min(READS_CHUNK, n_pairs - c * READS_CHUNK)
        qs.append(q[:qo[take]])
        ss.append(s[:so[take]])
        qos.append(qo[1:take + 1])
        sos.append(so[1:take + 1])
    q_off = np.zeros(n_pairs + 1, dtype=np.int64)
    s_off = np.zeros(n_pairs + 1, dtype=np.int64)
    if n_pairs:
        qb = np.cumsum([0] + [len(x) for x in qs[:-1]])
        sb = np.cumsum([0] + [len(x) for x in ss[:-1]])
        q_off[1:] = np.concatenate([o + b for o, b in zip(qos, qb)])
        s_off[1:] = np.concatenate([o + b for o, b in zip(sos, sb)])
    q = np.concatenate(qs) if qs else np.zeros(0, np.uint8)
    s = np.concatenate(ss) if ss else np.zeros(0, np.uint8)
    return Workload("reads_semiglobal", SEMIGLOBAL, 4, -5, -2, q, q_off, s, s_off, match=1, mismatch=-4,
                    traceback=True)


def protein_sigma(rng: np.random.Generator) -> np.ndarray:
    t = rng.integers(-4, 4, (20, 20))
    t = np.triu(t, 1)
    t = t + t.T
    np.fill_diagonal(t, rng.integers(4, 12, 20))
    return t.astype(np.int8)


def protein_uneven(seed: int = 4, n_pairs: int = 65536, lmin: int = 64, lmax: int = 16384) -> Workload:
    rng = np.random.default_rng(seed)
    sig = protein_sigma(rng)
    lo, hi = np.log(lmin), np.log(lmax)
    n = np.rint(np.exp(rng.uniform(lo, hi, n_pairs))).astype(np.int64)
    m = np.rint(np.exp(rng.uniform(lo, hi, n_pairs))).astype(np.int64)
    q_off = np.zeros(n_pairs + 1, dtype=np.int64)
    s_off = np.zeros(n_pairs + 1, dtype=np.int64)
    np.cumsum(n, out=q_off[1:])
    np.cumsum(m, out=s_off[1:])
    q = rng.integers(0, 20, int(q_off[-1]), dtype=np.uint8)
    s = rng.integers(0, 20, int(s_off[-1]), dtype=np.uint8)
    return Workload("protein_uneven", LOCAL, 20, -11, -1, q, q_off, s, s_off, subst=sig)


def random_pairs(seed: int, n_pairs: int, nmin: int, nmax: int, alphabet: int, mode: int, gap_open: int,
                 gap_extend: int, match: Optional[int] = None, mismatch: Optional[int] = None,
                 subst: Optional[np.ndarray] = None, related: float = 0.0, mmin: Optional[int] = None,
                 mmax: Optional[int] = None) -> Workload:
    """Generic test pairs: lengths uniform in [nmin, nmax] (and [mmin, mmax] for subjects); with
    probability `related` the subject is a mutated copy of the query (10% substitutions, 2% indels)."""
    rng = np.random.default_rng(seed)
    mmin = nmin if mmin is None else mmin
    mmax = nmax if mmax is None else mmax
    qs, ss = [], []
    for _ in range(n_pairs):
        n = int(rng.integers(nmin, nmax + 1))
        a = rng.integers(0, alphabet, n, dtype=np.uint8)
        if related > 0 and rng.random() < related and n > 0:
            b = mutate_geometric(rng, a, 0.10, 0.02, 2.0, alphabet)
        else:
            b = rng.integers(0, alphabet, int(rng.integers(mmin, mmax + 1)), dtype=np.uint8)
        qs.append(a)
        ss.append(b)
    q, qo = pack(qs)
    s, so = pack(ss)
    return Workload("random_pairs", mode, alphabet, gap_open, gap_extend, q, qo, s, so, match, mismatch, subst)


# Scoring schemes of the serving stream's request classes (plain data: mode, alphabet, gaps, scores).
SERVE_CLASSES = {
    "read": dict(mode=SEMIGLOBAL, alphabet_size=4, gap_open=-5, gap_extend=-2, match=1, mismatch=-4, traceback=True),
    "protein": dict(mode=LOCAL, alphabet_size=20, gap_open=-11, gap_extend=-1, traceback=False),
    "long": dict(mode=LOCAL, alphabet_size=4, gap_open=-3, gap_extend=-1, match=2, mismatch=-3, traceback=False),
}


@dataclass
class ServeItem:
    rid: int
    klass: str
    q: np.ndarray
    s: np.ndarray
    arrival: float  # seconds from the start of the stream


def serve_stream(n_req: int, rate_hz: float, seed: int = 5, long_len: int = 65536, protein_max: int = 16384):
    """A Poisson request stream mixing three classes: 80% read/window pairs (as reads_semiglobal, CIGAR
    wanted), 19% protein pairs (lengths log-uniform 64..protein_max, unrelated, 20 letters) and 1% long
    local DNA pairs of long_len x long_len (the second a mutated copy of the first, as long_dna_local).
    Returns (items, protein substitution table).  The sequences do not depend on rate_hz."""
    rng = np.random.default_rng(seed)
    reads = reads_semiglobal(seed=seed, n_pairs=n_req)
    sig = protein_sigma(rng)
    items, t = [], 0.0
    for k in range(n_req):
        t += rng.exponential(1.0 / rate_hz)
        u = rng.random()
        if u < 0.8:
            a, b = reads.pair(k)
            items.append(ServeItem(k, "read", a.copy(), b.copy(), t))
        elif u < 0.99:
            n, m = np.rint(np.exp(rng.uniform(np.log(64), np.log(protein_max), 2))).astype(int)
            items.append(ServeItem(k, "protein", rng.integers(0, 20, n, dtype=np.uint8),
                                   rng.integers(0, 20, m, dtype=np.uint8), t))
        else:
            a = rng.integers(0, 4, long_len, dtype=np.uint8)
            b = mutate_geometric(rng, a, 0.05, 0.01, 3.0)[:long_len]
            if len(b) < long_len:
                b = np.concatenate([b, rng.integers(0, 4, long_len - len(b), dtype=np.uint8)])
            items.append(ServeItem(k, "long", a, b, t))
    return items, sig


def serve_workload(items, klass: str, sig: np.ndarray) -> Workload:
    """The requests of one class of a serving stream as a batch Workload (for checking results)."""
    cls = SERVE_CLASSES[klass]
    sel = [it for it in items if it.klass == klass]
    q, qo = pack([it.q for it in sel])
    s, so = pack([it.s for it in sel])
    return Workload("serve_" + klass, cls["mode"], cls["alphabet_size"], cls["gap_open"], cls["gap_extend"], q, qo,
                    s, so, match=cls.get("match"), mismatch=cls.get("mismatch"),
                    subst=sig if klass == "protein" else None, traceback=cls["traceback"])
