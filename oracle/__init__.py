"""Reference oracle for pairwise alignment -- TEST INFRASTRUCTURE ONLY.

Only ``tests/``, ``__graft_entry__.smoke()`` and the CPU-baseline leg of
``bench.py`` may import this package.  The product library never does, and it
shares no code with the HIP path.

The arithmetic lives in ``oracle.c`` (plain scalar C, int64, full H/E/F
matrices or two rows) and follows AnySeq Sec. III-A, Eqs. (1)-(5); this module
only builds that file with gcc, marshals arguments through ctypes and turns a
match/mismatch scheme into the full substitution table the C code reads.
"""
from __future__ import annotations

import ctypes
import os
import subprocess
import threading
from dataclasses import dataclass, field
from typing import List, Optional, Sequence, Tuple

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
_LIB_PATH = os.path.join(_HERE, "liboracle.so")
_SRC = os.path.join(_HERE, "oracle.c")
_lock = threading.Lock()
_lib = None

GLOBAL, LOCAL, SEMIGLOBAL = 0, 1, 2
MODE_NAMES = {GLOBAL: "global", LOCAL: "local", SEMIGLOBAL: "semiglobal"}
OP_M, OP_I, OP_D = 0, 1, 2
FLAG_CIGAR_TRUNC = 2
FLAG_BAD_CODE = 4


def build(force: bool = False) -> str:
    """Compiles oracle.c into liboracle.so (plain -O2, no SIMD intrinsics, no OpenMP)."""
    if force or not os.path.exists(_LIB_PATH) or os.path.getmtime(_LIB_PATH) < os.path.getmtime(_SRC):
        tmp = _LIB_PATH + ".tmp%d" % os.getpid()
        subprocess.check_call(["gcc", "-O2", "-std=c11", "-shared", "-fPIC", "-o", tmp, _SRC, "-lpthread"])
        os.replace(tmp, _LIB_PATH)
    return _LIB_PATH


class _Scoring(ctypes.Structure):
    _fields_ = [
        ("mode", ctypes.c_int32),
        ("alphabet_size", ctypes.c_int32),
        ("sigma", ctypes.POINTER(ctypes.c_int32)),
        ("gap_open", ctypes.c_int64),
        ("gap_extend", ctypes.c_int64),
    ]


class _Result(ctypes.Structure):
    _fields_ = [
        ("score", ctypes.c_int64),
        ("q_begin", ctypes.c_int64),
        ("q_end", ctypes.c_int64),
        ("s_begin", ctypes.c_int64),
        ("s_end", ctypes.c_int64),
        ("cigar_len", ctypes.c_int64),
        ("flags", ctypes.c_int64),
    ]


RESULT_DTYPE = np.dtype(
    [("score", "<i8"), ("q_begin", "<i8"), ("q_end", "<i8"), ("s_begin", "<i8"), ("s_end", "<i8"),
     ("cigar_len", "<i8"), ("flags", "<i8")]
)
assert RESULT_DTYPE.itemsize == ctypes.sizeof(_Result)


def _load():
    global _lib
    with _lock:
        if _lib is None:
            build()
            lib = ctypes.CDLL(_LIB_PATH)
            u8p = ctypes.POINTER(ctypes.c_uint8)
            i64p = ctypes.POINTER(ctypes.c_int64)
            u32p = ctypes.POINTER(ctypes.c_uint32)
            for name in ("orc_align_affine_full", "orc_align_linear_full"):
                f = getattr(lib, name)
                f.argtypes = [ctypes.POINTER(_Scoring), u8p, ctypes.c_int64, u8p, ctypes.c_int64, ctypes.c_int,
                              ctypes.POINTER(_Result), u32p, ctypes.c_int64]
                f.restype = ctypes.c_int
            f = lib.orc_align_affine_checkpointed
            f.argtypes = [ctypes.POINTER(_Scoring), u8p, ctypes.c_int64, u8p, ctypes.c_int64, ctypes.c_int64,
                          ctypes.POINTER(_Result), u32p, ctypes.c_int64]
            f.restype = ctypes.c_int
            f = lib.orc_score_affine_linear_space
            f.argtypes = [ctypes.POINTER(_Scoring), u8p, ctypes.c_int64, u8p, ctypes.c_int64, ctypes.POINTER(_Result)]
            f.restype = ctypes.c_int
            f = lib.orc_align_batch
            f.argtypes = [ctypes.POINTER(_Scoring), ctypes.c_int64, u8p, i64p, u8p, i64p, ctypes.c_int,
                          ctypes.c_void_p, u32p, i64p, ctypes.c_int]
            f.restype = ctypes.c_int
            _lib = lib
    return _lib


@dataclass
class Scoring:
    """Scoring scheme: mode, alphabet, substitution table, signed gap open/extend."""

    mode: int
    alphabet_size: int
    sigma: np.ndarray  # (A, A) int32, sigma[q, s]
    gap_open: int
    gap_extend: int
    _c: Optional[_Scoring] = field(default=None, repr=False, compare=False)

    @staticmethod
    def simple(mode: int, alphabet_size: int, match: int, mismatch: int, gap_open: int, gap_extend: int) -> "Scoring":
        """The simple_subst_scoring(match, mismatch) scheme of Sec. III-C as a full table."""
        sig = np.full((alphabet_size, alphabet_size), mismatch, dtype=np.int32)
        np.fill_diagonal(sig, match)
        return Scoring(mode, alphabet_size, sig, gap_open, gap_extend)

    @staticmethod
    def matrix(mode: int, sigma: np.ndarray, gap_open: int, gap_extend: int) -> "Scoring":
        sig = np.ascontiguousarray(sigma, dtype=np.int32)
        return Scoring(mode, sig.shape[0], sig, gap_open, gap_extend)

    def c(self) -> _Scoring:
        if self._c is None:
            self.sigma = np.ascontiguousarray(self.sigma, dtype=np.int32)
            self._c = _Scoring(self.mode, self.alphabet_size,
                               self.sigma.ctypes.data_as(ctypes.POINTER(ctypes.c_int32)),
                               self.gap_open, self.gap_extend)
        return self._c


@dataclass
class Alignment:
    score: int
    q_begin: int
    q_end: int
    s_begin: int
    s_end: int
    cigar: List[Tuple[int, int]]  # (run length, op)
    flags: int = 0


def _u8(x) -> np.ndarray:
    a = np.ascontiguousarray(np.asarray(x, dtype=np.uint8))
    return a


def _ptr(a: np.ndarray, ct):
    return a.ctypes.data_as(ctypes.POINTER(ct))


def align(sc: Scoring, q: Sequence[int], s: Sequence[int], traceback: bool = False, impl: str = "affine",
          block_rows: int = 512) -> Alignment:
    """One pair.  impl: 'affine' (full H/E/F), 'linear' (one-matrix Eqs. (2)-(3), needs gap_open == 0),
    'linspace' (score-only, two rows) or 'checkpointed' (the affine results with the traceback in linear
    space: every block_rows-th row kept, one block recomputed at a time)."""
    lib = _load()
    qa, sa = _u8(q), _u8(s)
    n, m = len(qa), len(sa)
    res = _Result()
    cap = n + m + 1
    cig = np.zeros(cap, dtype=np.uint32)
    qp = _ptr(qa, ctypes.c_uint8) if n else ctypes.cast(ctypes.c_char_p(b"\0"), ctypes.POINTER(ctypes.c_uint8))
    sp = _ptr(sa, ctypes.c_uint8) if m else ctypes.cast(ctypes.c_char_p(b"\0"), ctypes.POINTER(ctypes.c_uint8))
    if impl == "affine":
        rc = lib.orc_align_affine_full(ctypes.byref(sc.c()), qp, n, sp, m, int(traceback), ctypes.byref(res),
                                       _ptr(cig, ctypes.c_uint32), cap)
    elif impl == "linear":
        rc = lib.orc_align_linear_full(ctypes.byref(sc.c()), qp, n, sp, m, int(traceback), ctypes.byref(res),
                                       _ptr(cig, ctypes.c_uint32), cap)
    elif impl == "checkpointed":
        if not traceback:
            raise ValueError("checkpointed is the traceback")
        rc = lib.orc_align_affine_checkpointed(ctypes.byref(sc.c()), qp, n, sp, m, int(block_rows), ctypes.byref(res),
                                               _ptr(cig, ctypes.c_uint32), cap)
    elif impl == "linspace":
        if traceback:
            raise ValueError("linspace is score-only")
        rc = lib.orc_score_affine_linear_space(ctypes.byref(sc.c()), qp, n, sp, m, ctypes.byref(res))
    else:
        raise ValueError(impl)
    if rc != 0:
        raise RuntimeError("oracle failed with code %d" % rc)
    cigar = [(int(w) >> 4, int(w) & 15) for w in cig[: res.cigar_len]] if traceback else []
    return Alignment(int(res.score), int(res.q_begin), int(res.q_end), int(res.s_begin), int(res.s_end), cigar,
                     int(res.flags))


def align_batch(sc: Scoring, q: np.ndarray, q_off: np.ndarray, s: np.ndarray, s_off: np.ndarray,
                traceback: bool = False, threads: Optional[int] = None):
    """Independent pairs on a pool of host threads.  Returns (results structured array, cigar, cigar_off);
    the CIGAR buffer gives each pair n+m words of room."""
    lib = _load()
    qa, sa = _u8(q), _u8(s)
    qo = np.ascontiguousarray(q_off, dtype=np.int64)
    so = np.ascontiguousarray(s_off, dtype=np.int64)
    n_pairs = len(qo) - 1
    res = np.zeros(n_pairs, dtype=RESULT_DTYPE)
    if traceback:
        lens = (qo[1:] - qo[:-1]) + (so[1:] - so[:-1]) + 1
        coff = np.zeros(n_pairs + 1, dtype=np.int64)
        np.cumsum(lens, out=coff[1:])
    else:
        coff = np.zeros(n_pairs + 1, dtype=np.int64)
    cig = np.zeros(max(int(coff[-1]), 1), dtype=np.uint32)
    if threads is None:
        threads = len(os.sched_getaffinity(0))
    if len(qa) == 0:
        qa = np.zeros(1, np.uint8)
    if len(sa) == 0:
        sa = np.zeros(1, np.uint8)
    rc = lib.orc_align_batch(ctypes.byref(sc.c()), n_pairs, _ptr(qa, ctypes.c_uint8), _ptr(qo, ctypes.c_int64),
                             _ptr(sa, ctypes.c_uint8), _ptr(so, ctypes.c_int64), int(traceback),
                             res.ctypes.data_as(ctypes.c_void_p), _ptr(cig, ctypes.c_uint32),
                             _ptr(coff, ctypes.c_int64), int(threads))
    if rc != 0:
        raise RuntimeError("oracle batch failed with code %d" % rc)
    return res, cig, coff


def cigar_string(cigar: Sequence[Tuple[int, int]]) -> str:
    return "".join("%d%s" % (n, "MID"[op]) for n, op in cigar)
