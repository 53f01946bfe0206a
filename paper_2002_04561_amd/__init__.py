"""mialign: pairwise sequence alignment on AMD MI355X (gfx950).

Thin Python binding over the C ABI declared in ``include/mialign.h``.  It only
marshals arguments: every step of the alignment runs in the HIP kernels of
``libmialign.so``.  PyTorch supplies device memory and the HIP stream.  There
is no CPU fallback: if the library is missing, importing the binding's entry
points raises.
"""
from __future__ import annotations

import ctypes
import os
from dataclasses import dataclass
from typing import Optional

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(_HERE, "libmialign.so")

GLOBAL, LOCAL, SEMIGLOBAL = 0, 1, 2
SCORE_ONLY, TRACEBACK, FORCE_INT32, FORCE_INT16, LINEAR_SPACE, STORED_CODES = 0, 1, 2, 4, 8, 16
RES_INT32_REDO, RES_CIGAR_TRUNC, RES_BAD_CODE, RES_TOO_LONG, RES_DEVICE_ERROR, RES_BAD_END = 1, 2, 4, 8, 16, 32
CIGAR_M, CIGAR_I, CIGAR_D = 0, 1, 2

STATUS = {0: "ALN_OK", -1: "ALN_E_INVALID", -2: "ALN_E_ALPHABET", -3: "ALN_E_SCORING", -4: "ALN_E_WORKSPACE",
          -5: "ALN_E_DEVICE", -6: "ALN_E_UNSUPPORTED"}

RESULT_DTYPE = np.dtype([("score", "<i4"), ("q_begin", "<i4"), ("q_end", "<i4"), ("s_begin", "<i4"),
                         ("s_end", "<i4"), ("cigar_len", "<i4"), ("flags", "<u4"), ("reserved", "<i4")])


class AlnError(RuntimeError):
    def __init__(self, status: int, what: str = ""):
        self.status = status
        super().__init__("%s%s (%d)" % (what + ": " if what else "", STATUS.get(status, "?"), status))


class aln_scoring_t(ctypes.Structure):
    _fields_ = [("mode", ctypes.c_int32), ("alphabet_size", ctypes.c_int32), ("subst", ctypes.POINTER(ctypes.c_int8)),
                ("match", ctypes.c_int32), ("mismatch", ctypes.c_int32), ("gap_open", ctypes.c_int32),
                ("gap_extend", ctypes.c_int32)]


class aln_batch_config_t(ctypes.Structure):
    _fields_ = [("wf_min_cells", ctypes.c_int64), ("wf_waves_per_cu", ctypes.c_int32), ("wf_orient", ctypes.c_int32),
                ("small_bits", ctypes.c_int32), ("wf_group", ctypes.c_int32), ("wf_bits", ctypes.c_int32),
                ("reserved", ctypes.c_int32)]


@dataclass(frozen=True)
class BatchConfig:
    """aln_batch_config_t: execution choices of a batch call (0 = the library's default)."""

    wf_min_cells: int = 0
    wf_waves_per_cu: int = 0
    wf_orient: int = 0
    small_bits: int = 0
    wf_group: int = 0
    wf_bits: int = 0

    def c(self) -> aln_batch_config_t:
        return aln_batch_config_t(self.wf_min_cells, self.wf_waves_per_cu, self.wf_orient, self.small_bits,
                                  self.wf_group, self.wf_bits, 0)


_lib = None

_SIGNATURES = {
    "aln_batch_workspace_size": (ctypes.c_int32, [ctypes.POINTER(aln_scoring_t), ctypes.c_int64, ctypes.c_int64,
                                                  ctypes.c_int64, ctypes.c_int64, ctypes.c_int64, ctypes.c_uint32,
                                                  ctypes.POINTER(ctypes.c_size_t)]),
    "aln_align_batch": (ctypes.c_int32, [ctypes.POINTER(aln_scoring_t), ctypes.c_int64, ctypes.c_void_p,
                                         ctypes.c_void_p, ctypes.c_void_p, ctypes.c_void_p, ctypes.c_int64,
                                         ctypes.c_int64, ctypes.c_int64, ctypes.c_int64, ctypes.c_uint32,
                                         ctypes.c_void_p, ctypes.c_void_p, ctypes.c_void_p, ctypes.c_void_p,
                                         ctypes.c_size_t, ctypes.c_void_p]),
    "aln_align_batch_ex": (ctypes.c_int32, [ctypes.POINTER(aln_scoring_t), ctypes.c_int64, ctypes.c_void_p,
                                            ctypes.c_void_p, ctypes.c_void_p, ctypes.c_void_p, ctypes.c_int64,
                                            ctypes.c_int64, ctypes.c_int64, ctypes.c_int64, ctypes.c_uint32,
                                            ctypes.POINTER(aln_batch_config_t), ctypes.c_void_p, ctypes.c_void_p,
                                            ctypes.c_void_p, ctypes.c_void_p, ctypes.c_size_t, ctypes.c_void_p]),
    "aln_long_workspace_size": (ctypes.c_int32, [ctypes.POINTER(aln_scoring_t), ctypes.c_int64, ctypes.c_int64,
                                                 ctypes.c_uint32, ctypes.POINTER(ctypes.c_size_t)]),
    "aln_align_long": (ctypes.c_int32, [ctypes.POINTER(aln_scoring_t), ctypes.c_void_p, ctypes.c_int64,
                                        ctypes.c_void_p, ctypes.c_int64, ctypes.c_uint32, ctypes.c_void_p,
                                        ctypes.c_void_p, ctypes.c_int64, ctypes.c_void_p, ctypes.c_size_t,
                                        ctypes.c_void_p]),
    "aln_profile_enable": (ctypes.c_int32, [ctypes.c_int]),
    "aln_profile_reset": (ctypes.c_int32, []),
    "aln_profile_read": (ctypes.c_int32, [ctypes.c_void_p, ctypes.c_int32, ctypes.POINTER(ctypes.c_int32)]),
    "aln_set_wait_limits": (ctypes.c_int32, [ctypes.c_int64, ctypes.c_int64]),
    "aln_align_batch_noalloc": (ctypes.c_int32, [ctypes.POINTER(aln_scoring_t), ctypes.c_int64, ctypes.c_void_p,
                                                 ctypes.c_void_p, ctypes.c_void_p, ctypes.c_void_p, ctypes.c_int64,
                                                 ctypes.c_int64, ctypes.c_int64, ctypes.c_int64, ctypes.c_uint32,
                                                 ctypes.POINTER(aln_batch_config_t), ctypes.c_void_p,
                                                 ctypes.c_void_p, ctypes.c_void_p, ctypes.c_void_p]),
    "aln_noalloc_scratch_bytes": (ctypes.c_size_t, []),
    "aln_set_traceback_budget": (ctypes.c_int32, [ctypes.c_int64]),
    "aln_set_batch_code_arena": (ctypes.c_int32, [ctypes.c_int64]),
    "aln_batch_route": (ctypes.c_int32, [ctypes.c_int64, ctypes.c_uint32, ctypes.c_void_p,
                                         ctypes.POINTER(ctypes.c_int64), ctypes.POINTER(ctypes.c_int64)]),
    "aln_traceback_workspace_size": (ctypes.c_int32, [ctypes.POINTER(aln_scoring_t), ctypes.c_int64, ctypes.c_int64,
                                                      ctypes.c_int64, ctypes.POINTER(ctypes.c_size_t)]),
    "aln_traceback": (ctypes.c_int32, [ctypes.POINTER(aln_scoring_t), ctypes.c_int64, ctypes.c_void_p, ctypes.c_void_p,
                                       ctypes.c_void_p, ctypes.c_void_p, ctypes.c_int64, ctypes.c_int64,
                                       ctypes.c_void_p, ctypes.c_void_p, ctypes.c_void_p, ctypes.c_void_p,
                                       ctypes.c_void_p, ctypes.c_size_t, ctypes.c_void_p]),
    "aln_cigar_to_gapped": (ctypes.c_int32, [ctypes.c_void_p, ctypes.c_int64, ctypes.c_void_p, ctypes.c_int64,
                                             ctypes.c_void_p, ctypes.c_void_p, ctypes.c_char_p, ctypes.c_void_p,
                                             ctypes.c_void_p, ctypes.c_int64]),
    "aln_status_string": (ctypes.c_char_p, [ctypes.c_int32]),
    "aln_version": (ctypes.c_char_p, []),
}


def lib():
    """Loads libmialign.so (built by paper_2002_04561_amd.build); raises if it is missing."""
    global _lib
    if _lib is None:
        if not os.path.exists(LIB_PATH):
            raise RuntimeError("libmialign.so is not built (run __graft_entry__.build() or "
                               "python paper_2002_04561_amd/build.py); there is no CPU fallback")
        L = ctypes.CDLL(LIB_PATH)
        for name, (res, args) in _SIGNATURES.items():
            f = getattr(L, name)
            f.restype = res
            f.argtypes = args
        _lib = L
    return _lib


def exported_symbols():
    return list(_SIGNATURES)


@dataclass
class Scoring:
    """aln_scoring_t: mode, alphabet, substitution table (or match/mismatch), signed gap open/extend."""

    mode: int
    alphabet_size: int
    gap_open: int
    gap_extend: int
    match: int = 0
    mismatch: int = 0
    subst: Optional[np.ndarray] = None

    def c(self) -> aln_scoring_t:
        if self.subst is not None:
            self._subst_buf = np.ascontiguousarray(self.subst, dtype=np.int8)
            ptr = self._subst_buf.ctypes.data_as(ctypes.POINTER(ctypes.c_int8))
        else:
            ptr = ctypes.POINTER(ctypes.c_int8)()
        return aln_scoring_t(self.mode, self.alphabet_size, ptr, self.match, self.mismatch, self.gap_open,
                             self.gap_extend)


def _ptr(t) -> Optional[int]:
    if t is None:
        return None
    return int(t.data_ptr())


def _stream_handle(stream) -> Optional[int]:
    if stream is None:
        import torch
        stream = torch.cuda.current_stream()
    return int(stream.cuda_stream)


def aln_batch_workspace_size(scoring: Scoring, n_pairs: int, max_n: int, max_m: int, total_q: int, total_s: int,
                             flags: int) -> int:
    out = ctypes.c_size_t(0)
    sc = scoring.c()
    st = lib().aln_batch_workspace_size(ctypes.byref(sc), n_pairs, max_n, max_m, total_q, total_s, flags,
                                        ctypes.byref(out))
    if st != 0:
        raise AlnError(st, "aln_batch_workspace_size")
    return int(out.value)


def aln_align_batch(scoring: Scoring, n_pairs: int, q, q_off, s, s_off, max_n: int, max_m: int, total_q: int,
                    total_s: int, flags: int, out, cigar, cigar_off, workspace, workspace_bytes: int,
                    stream=None) -> int:
    """Same arguments as the C function; tensors are torch device tensors.  Returns the status code."""
    sc = scoring.c()
    return int(lib().aln_align_batch(ctypes.byref(sc), n_pairs, _ptr(q), _ptr(q_off), _ptr(s), _ptr(s_off), max_n,
                                     max_m, total_q, total_s, flags, _ptr(out), _ptr(cigar), _ptr(cigar_off),
                                     _ptr(workspace), workspace_bytes, _stream_handle(stream)))


def aln_long_workspace_size(scoring: Scoring, n: int, m: int, flags: int = SCORE_ONLY) -> int:
    out = ctypes.c_size_t(0)
    sc = scoring.c()
    st = lib().aln_long_workspace_size(ctypes.byref(sc), n, m, flags, ctypes.byref(out))
    if st != 0:
        raise AlnError(st, "aln_long_workspace_size")
    return int(out.value)


def aln_align_long(scoring: Scoring, q, n: int, s, m: int, flags: int, out, cigar, cigar_capacity: int, workspace,
                   workspace_bytes: int, stream=None) -> int:
    sc = scoring.c()
    return int(lib().aln_align_long(ctypes.byref(sc), _ptr(q), n, _ptr(s), m, flags, _ptr(out), _ptr(cigar),
                                    cigar_capacity, _ptr(workspace), workspace_bytes, _stream_handle(stream)))


class LongAligner:
    """Owns the result and workspace buffers for aln_align_long on one device-resident pair."""

    def __init__(self, scoring: Scoring, q, s, flags: int = SCORE_ONLY, device="cuda", cigar_capacity=None):
        import torch
        self.scoring, self.q, self.s, self.flags = scoring, q, s, flags
        self.n, self.m = int(q.numel()), int(s.numel())
        self.out = torch.empty(8, dtype=torch.int32, device=device)
        self.cigar, self.cap = None, 0
        if flags & TRACEBACK:
            self.cap = self.n + self.m + 1 if cigar_capacity is None else int(cigar_capacity)
            self.cigar = torch.empty(max(self.cap, 1), dtype=torch.int32, device=device)
        self.ws_bytes = aln_long_workspace_size(scoring, self.n, self.m, flags)
        self.workspace = torch.empty(max(self.ws_bytes, 256), dtype=torch.uint8, device=device)

    def run(self, stream=None):
        st = aln_align_long(self.scoring, self.q, self.n, self.s, self.m, self.flags, self.out, self.cigar, self.cap,
                            self.workspace, self.ws_bytes, stream)
        if st != 0:
            raise AlnError(st, "aln_align_long")

    def result(self):
        return self.out.to("cpu").numpy().view(RESULT_DTYPE)[0]

    def cigar_runs(self):
        r = self.result()
        L = min(int(r["cigar_len"]), self.cap)
        w = self.cigar[:L].to("cpu").numpy().view(np.uint32)
        return [(int(x) >> 4, int(x) & 15) for x in w]


class aln_profile_entry_t(ctypes.Structure):
    _fields_ = [("name", ctypes.c_char * 48), ("launches", ctypes.c_int64), ("total_ms", ctypes.c_double)]


def aln_profile_enable(on: bool) -> None:
    lib().aln_profile_enable(1 if on else 0)


def aln_profile_reset() -> None:
    lib().aln_profile_reset()


def aln_profile_read() -> dict:
    """{kernel family: (launches, total_ms)} accumulated since the last reset (waits for the events)."""
    arr = (aln_profile_entry_t * 64)()
    n = ctypes.c_int32(0)
    st = lib().aln_profile_read(ctypes.cast(arr, ctypes.c_void_p), 64, ctypes.byref(n))
    if st != 0:
        raise AlnError(st, "aln_profile_read")
    return {arr[k].name.decode(): (int(arr[k].launches), float(arr[k].total_ms)) for k in range(min(n.value, 64))}


def aln_traceback_workspace_size(scoring: Scoring, n_pairs: int, max_n: int, max_m: int) -> int:
    out = ctypes.c_size_t(0)
    sc = scoring.c()
    st = lib().aln_traceback_workspace_size(ctypes.byref(sc), n_pairs, max_n, max_m, ctypes.byref(out))
    if st != 0:
        raise AlnError(st, "aln_traceback_workspace_size")
    return int(out.value)


def aln_traceback(scoring: Scoring, n_pairs: int, q, q_off, s, s_off, max_n: int, max_m: int, fwd, out, cigar,
                  cigar_off, workspace, workspace_bytes: int, stream=None) -> int:
    """Same arguments as the C function; tensors are torch device tensors.  Returns the status code."""
    sc = scoring.c()
    return int(lib().aln_traceback(ctypes.byref(sc), n_pairs, _ptr(q), _ptr(q_off), _ptr(s), _ptr(s_off), max_n, max_m,
                                   _ptr(fwd), _ptr(out), _ptr(cigar), _ptr(cigar_off), _ptr(workspace),
                                   workspace_bytes, _stream_handle(stream)))


def traceback_pairs(scoring: Scoring, q, q_off, s, s_off, max_n: int, max_m: int, fwd, cigar_capacity=None,
                    device="cuda", stream=None):
    """aln_traceback over device-resident pairs and their forward results (an int32 tensor holding
    aln_result_t records).  Returns (results structured array, CIGAR run lists), after synchronising."""
    import torch
    n_pairs = int(q_off.numel()) - 1
    if cigar_capacity is None:
        qo = q_off.to("cpu").numpy()
        so = s_off.to("cpu").numpy()
        cap = np.maximum((qo[1:] - qo[:-1]) + (so[1:] - so[:-1]), 1)
    else:
        cap = np.asarray(cigar_capacity, dtype=np.int64)
    coff = np.zeros(n_pairs + 1, dtype=np.int64)
    np.cumsum(cap, out=coff[1:])
    cig = torch.empty(max(int(coff[-1]), 1), dtype=torch.int32, device=device)
    dcoff = torch.from_numpy(coff).to(device)
    out = torch.empty(n_pairs * 8, dtype=torch.int32, device=device)
    nbytes = aln_traceback_workspace_size(scoring, n_pairs, max_n, max_m)
    ws = torch.empty(max(nbytes, 256), dtype=torch.uint8, device=device)
    st = aln_traceback(scoring, n_pairs, q, q_off, s, s_off, max_n, max_m, fwd, out, cig, dcoff, ws, nbytes, stream)
    if st != 0:
        raise AlnError(st, "aln_traceback")
    torch.cuda.synchronize()
    res = out.to("cpu").numpy().view(RESULT_DTYPE)
    words = cig.to("cpu").numpy().view(np.uint32)
    runs = []
    for k in range(n_pairs):
        L = min(int(res["cigar_len"][k]), int(coff[k + 1] - coff[k]))
        runs.append([(int(x) >> 4, int(x) & 15) for x in words[coff[k]:coff[k] + L]])
    return res, runs


def aln_cigar_to_gapped(q: np.ndarray, s: np.ndarray, result, runs, letters: Optional[str] = None):
    """The alignment as two gapped strings (host only).  result: one RESULT_DTYPE record (or a tuple-like
    with q_begin, s_begin); runs: [(length, op), ...].  Returns (q_aln, s_aln)."""
    qa = np.ascontiguousarray(q, dtype=np.uint8)
    sa = np.ascontiguousarray(s, dtype=np.uint8)
    words = np.array([(int(L) << 4) | int(op) for L, op in runs], dtype=np.uint32)
    rec = np.zeros(1, dtype=RESULT_DTYPE)
    rec["q_begin"] = int(result["q_begin"])
    rec["s_begin"] = int(result["s_begin"])
    rec["cigar_len"] = len(words)
    cap = int(sum(int(L) for L, _ in runs)) + 1
    qbuf = ctypes.create_string_buffer(cap)
    sbuf = ctypes.create_string_buffer(cap)
    st = lib().aln_cigar_to_gapped(qa.ctypes.data if len(qa) else None, len(qa), sa.ctypes.data if len(sa) else None,
                                   len(sa), rec.ctypes.data, words.ctypes.data if len(words) else None,
                                   letters.encode() if letters is not None else None, ctypes.addressof(qbuf),
                                   ctypes.addressof(sbuf), cap)
    if st != 0:
        raise AlnError(st, "aln_cigar_to_gapped")
    return qbuf.value.decode(), sbuf.value.decode()


def aln_set_traceback_budget(nbytes: int = 0) -> None:
    """Bytes of codes a linear-space traceback holds at once (0 = the library's default, 4 GiB)."""
    st = lib().aln_set_traceback_budget(nbytes)
    if st != 0:
        raise AlnError(st, "aln_set_traceback_budget")


def aln_batch_route(n_pairs: int, flags: int = SCORE_ONLY, config: Optional["BatchConfig"] = None):
    """The planner's routing rule for such a batch: (min_cells, max_side); a pair runs on the band
    wavefront when n*m >= min_cells or n or m > max_side (2**63 - 1: no bound)."""
    mc, ms = ctypes.c_int64(0), ctypes.c_int64(0)
    cfg = config.c() if config is not None else None
    st = lib().aln_batch_route(n_pairs, flags, ctypes.byref(cfg) if cfg is not None else None, ctypes.byref(mc),
                               ctypes.byref(ms))
    if st != 0:
        raise AlnError(st, "aln_batch_route")
    return int(mc.value), int(ms.value)


def aln_set_batch_code_arena(nbytes: int = 0) -> None:
    """Most bytes of a traceback batch's code arena (0 = the library's default, 16 GiB)."""
    st = lib().aln_set_batch_code_arena(nbytes)
    if st != 0:
        raise AlnError(st, "aln_set_batch_code_arena")


def aln_set_wait_limits(device_polls: int = 0, lds_polls: int = 0) -> None:
    """Poll counts of the bounded device-side waits (0 = the library's defaults); a diagnostic aid."""
    st = lib().aln_set_wait_limits(device_polls, lds_polls)
    if st != 0:
        raise AlnError(st, "aln_set_wait_limits")


def aln_status_string(status: int) -> str:
    return lib().aln_status_string(status).decode()


def aln_version() -> str:
    return lib().aln_version().decode()


def aln_align_batch_ex(scoring: Scoring, n_pairs: int, q, q_off, s, s_off, max_n: int, max_m: int, total_q: int,
                       total_s: int, flags: int, config: Optional[BatchConfig], out, cigar, cigar_off, workspace,
                       workspace_bytes: int, stream=None) -> int:
    """aln_align_batch with a BatchConfig (None = defaults).  Returns the status code."""
    sc = scoring.c()
    cfg = ctypes.byref(config.c()) if config is not None else None
    return int(lib().aln_align_batch_ex(ctypes.byref(sc), n_pairs, _ptr(q), _ptr(q_off), _ptr(s), _ptr(s_off),
                                        max_n, max_m, total_q, total_s, flags, cfg, _ptr(out), _ptr(cigar),
                                        _ptr(cigar_off), _ptr(workspace), workspace_bytes, _stream_handle(stream)))


class BatchAligner:
    """Owns the device buffers for repeated aln_align_batch calls over one set of device-resident pairs."""

    def __init__(self, scoring: Scoring, q, q_off, s, s_off, max_n: int, max_m: int, flags: int = SCORE_ONLY,
                 cigar_capacity=None, device="cuda", total_q=None, total_s=None, config: Optional[BatchConfig] = None,
                 workspace=None):
        """workspace: an optional caller-owned uint8 device tensor of at least the size query's bytes, for
        callers that run several aligners one after another on one stream and share one workspace."""
        import torch
        self.torch = torch
        self.config = config
        self.scoring = scoring
        self.q, self.q_off, self.s, self.s_off = q, q_off, s, s_off
        self.n_pairs = int(q_off.numel()) - 1
        self.max_n, self.max_m, self.flags = int(max_n), int(max_m), int(flags)
        self.total_q = int(q.numel()) if total_q is None else int(total_q)
        self.total_s = int(s.numel()) if total_s is None else int(total_s)
        self.out = torch.empty(self.n_pairs * 8, dtype=torch.int32, device=device)
        self.cigar = self.cigar_off = None
        if flags & TRACEBACK:
            if cigar_capacity is None:
                qo = q_off.to("cpu").numpy()
                so = s_off.to("cpu").numpy()
                cap = (qo[1:] - qo[:-1]) + (so[1:] - so[:-1])
                cap = np.maximum(cap, 1)
            else:
                cap = np.asarray(cigar_capacity, dtype=np.int64)
            coff = np.zeros(self.n_pairs + 1, dtype=np.int64)
            np.cumsum(cap, out=coff[1:])
            self.cigar_off = torch.from_numpy(coff).to(device)
            self.cigar = torch.empty(max(int(coff[-1]), 1), dtype=torch.int32, device=device)
        self.ws_bytes = aln_batch_workspace_size(scoring, self.n_pairs, self.max_n, self.max_m, self.total_q,
                                                 self.total_s, self.flags)
        if workspace is not None:
            if workspace.numel() < self.ws_bytes:
                raise ValueError("workspace of %d bytes, %d needed" % (workspace.numel(), self.ws_bytes))
            self.workspace = workspace
        else:
            self.workspace = torch.empty(max(self.ws_bytes, 256), dtype=torch.uint8, device=device)

    def run(self, stream=None):
        if self.config is None:
            st = aln_align_batch(self.scoring, self.n_pairs, self.q, self.q_off, self.s, self.s_off, self.max_n,
                                 self.max_m, self.total_q, self.total_s, self.flags, self.out, self.cigar,
                                 self.cigar_off, self.workspace, self.ws_bytes, stream)
        else:
            st = aln_align_batch_ex(self.scoring, self.n_pairs, self.q, self.q_off, self.s, self.s_off, self.max_n,
                                    self.max_m, self.total_q, self.total_s, self.flags, self.config, self.out,
                                    self.cigar, self.cigar_off, self.workspace, self.ws_bytes, stream)
        if st != 0:
            raise AlnError(st, "aln_align_batch")

    def results(self) -> np.ndarray:
        return self.out.to("cpu").numpy().view(RESULT_DTYPE)

    def cigars(self, idx=None):
        """CIGAR run lists [(length, op), ...] of all pairs, or of the pairs in idx (dict k -> runs)."""
        res = self.results()
        cig = self.cigar.to("cpu").numpy().view(np.uint32)
        coff = self.cigar_off.to("cpu").numpy()
        if idx is not None:
            got = {}
            for k in idx:
                k = int(k)
                L = int(res["cigar_len"][k])
                w = cig[coff[k]:coff[k] + min(L, coff[k + 1] - coff[k])]
                got[k] = [(int(x) >> 4, int(x) & 15) for x in w]
            return got
        out = []
        for k in range(self.n_pairs):
            L = int(res["cigar_len"][k])
            w = cig[coff[k]:coff[k] + min(L, coff[k + 1] - coff[k])]
            out.append([(int(x) >> 4, int(x) & 15) for x in w])
        return out


def to_device(workload, device="cuda"):
    """Copies a synth.Workload's arrays to the device (torch tensors)."""
    import torch
    q = torch.from_numpy(np.ascontiguousarray(workload.q) if len(workload.q) else np.zeros(1, np.uint8)).to(device)
    s = torch.from_numpy(np.ascontiguousarray(workload.s) if len(workload.s) else np.zeros(1, np.uint8)).to(device)
    qo = torch.from_numpy(np.ascontiguousarray(workload.q_off)).to(device)
    so = torch.from_numpy(np.ascontiguousarray(workload.s_off)).to(device)
    return q, qo, s, so


def scoring_of(workload) -> Scoring:
    return Scoring(workload.mode, workload.alphabet_size, workload.gap_open, workload.gap_extend,
                   match=workload.match or 0, mismatch=workload.mismatch or 0, subst=workload.subst)
