"""Chunked digests of a batch's results, so that every pair of a large batch can be compared with the
oracle's results without storing them all.

A pair's record is its result fields as little-endian int64 (score, q_begin, q_end, s_begin, s_end and
cigar_len when traced back; score, q_end, s_end when score-only), and, when traced back, its CIGAR words
as little-endian uint32.  The digest of a chunk of consecutive pairs is the first 16 hex digits of the
SHA-256 of the chunk's field records followed by the concatenated CIGAR words of its pairs in order.
This is serialisation only: no alignment arithmetic happens here.
"""
import hashlib

import numpy as np

CHUNK = 4096
FIELDS_TB = ("score", "q_begin", "q_end", "s_begin", "s_end", "cigar_len")
FIELDS_SCORE = ("score", "q_end", "s_end")


def fields_of(res, traceback: bool) -> np.ndarray:
    names = FIELDS_TB if traceback else FIELDS_SCORE
    return np.stack([np.asarray(res[f]).astype(np.int64) for f in names], axis=1)


def chunk_digests(res, traceback: bool, cigar=None, cigar_off=None, chunk: int = CHUNK):
    """res: a structured array with the named fields (any integer widths); cigar: flat uint32 words with
    pair k's CIGAR at cigar[cigar_off[k] : cigar_off[k] + cigar_len[k]]."""
    f = fields_of(res, traceback)
    n = f.shape[0]
    out = []
    if traceback:
        lens = np.asarray(res["cigar_len"]).astype(np.int64)
        offs = np.asarray(cigar_off).astype(np.int64)
        words = np.asarray(cigar).view(np.uint32) if np.asarray(cigar).dtype != np.uint32 else np.asarray(cigar)
    for c0 in range(0, n, chunk):
        c1 = min(n, c0 + chunk)
        h = hashlib.sha256(np.ascontiguousarray(f[c0:c1], dtype="<i8").tobytes())
        if traceback:
            L = lens[c0:c1]
            tot = int(L.sum())
            if tot:
                starts = offs[c0:c1]
                first = np.concatenate([[0], np.cumsum(L)[:-1]])
                idx = np.repeat(starts - first, L) + np.arange(tot, dtype=np.int64)
                h.update(np.ascontiguousarray(words[idx], dtype="<u4").tobytes())
        out.append(h.hexdigest()[:16])
    return out
