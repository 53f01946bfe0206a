"""The C-ABI library loads and exports every function include/mialign.h declares (no GPU calls)."""
import ctypes
import os
import re

import paper_2002_04561_amd as aln

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


def _declared():
    names = []
    for fn in sorted(os.listdir(os.path.join(ROOT, "include"))):
        if not fn.endswith(".h"):
            continue
        txt = open(os.path.join(ROOT, "include", fn)).read()
        txt = re.sub(r"/\*.*?\*/", "", txt, flags=re.S)
        names += re.findall(r"^\s*(?:const\s+)?[A-Za-z_][A-Za-z0-9_]*\s*\**\s+\**(aln_[a-z0-9_]+)\s*\(", txt, re.M)
    return sorted(set(names))


def test_header_declares_entry_points():
    d = _declared()
    for name in ("aln_align_batch", "aln_batch_workspace_size", "aln_status_string", "aln_version"):
        assert name in d


def test_library_exports_every_declared_symbol():
    L = ctypes.CDLL(aln.LIB_PATH)
    for name in _declared():
        assert hasattr(L, name), name
    for name in aln.exported_symbols():
        assert name in _declared(), name


def test_status_strings_and_version():
    assert "invalid" in aln.aln_status_string(-1)
    assert aln.aln_status_string(0) == "ok"
    assert "gfx950" in aln.aln_version()


def test_scoring_validation_on_host():
    """Invalid scoring is rejected before any device work (the size query touches no device memory)."""
    bad = [aln.Scoring(0, 1, 0, -1, 1, -1), aln.Scoring(0, 33, 0, -1, 1, -1), aln.Scoring(0, 4, 1, -1, 1, -1),
           aln.Scoring(0, 4, 0, 0, 1, -1), aln.Scoring(5, 4, 0, -1, 1, -1)]
    expect = [-2, -2, -3, -3, -1]
    for sc, e in zip(bad, expect):
        out = ctypes.c_size_t(0)
        c = sc.c()
        st = aln.lib().aln_batch_workspace_size(ctypes.byref(c), 10, 100, 100, 1000, 1000, 0, ctypes.byref(out))
        assert st == e, (sc, st)


def test_batch_config_validation_on_host():
    """aln_align_batch_ex rejects out-of-range execution choices before any device work."""
    sc = aln.Scoring(0, 4, 0, -1, 1, -1).c()
    cases = [(aln.BatchConfig(wf_waves_per_cu=33), -1), (aln.BatchConfig(wf_waves_per_cu=-1), -1),
             (aln.BatchConfig(wf_orient=3), -1), (aln.BatchConfig(wf_orient=-2), -1),
             (aln.BatchConfig(small_bits=8), -1), (aln.BatchConfig(), 0),
             (aln.BatchConfig(wf_min_cells=-1, wf_waves_per_cu=32, wf_orient=-1, small_bits=32), 0),
             (aln.BatchConfig(wf_orient=2), 0)]
    for cfg, e in cases:
        c = cfg.c()
        st = aln.lib().aln_align_batch_ex(ctypes.byref(sc), 0, None, None, None, None, 0, 0, 0, 0, 0, ctypes.byref(c),
                                          None, None, None, None, 0, None)
        assert st == e, (cfg, st)
    for bad in (aln.BatchConfig(wf_group=2), aln.BatchConfig(wf_bits=8)):
        c = bad.c()
        st = aln.lib().aln_align_batch_ex(ctypes.byref(sc), 0, None, None, None, None, 0, 0, 0, 0, 0, ctypes.byref(c),
                                          None, None, None, None, 0, None)
        assert st == -1, bad
    for ok in (aln.BatchConfig(wf_bits=16), aln.BatchConfig(wf_bits=32)):
        c = ok.c()
        st = aln.lib().aln_align_batch_ex(ctypes.byref(sc), 0, None, None, None, None, 0, 0, 0, 0, 0, ctypes.byref(c),
                                          None, None, None, None, 0, None)
        assert st == 0, ok
    c = aln.BatchConfig().c()
    c.reserved = 5
    st = aln.lib().aln_align_batch_ex(ctypes.byref(sc), 0, None, None, None, None, 0, 0, 0, 0, 0, ctypes.byref(c),
                                      None, None, None, None, 0, None)
    assert st == -1


def test_long_size_query_host_checks():
    """aln_long_workspace_size refuses, before any device query, an unknown flag, a score range beyond exact
    32-bit lanes (ALN_E_SCORING), an invalid mode and a negative length (ALN_E_INVALID).  A traceback
    above 64 GiB of codes is no longer refused: it runs in linear space."""
    cases = [(aln.Scoring(1, 4, -3, -1, 2, -3), 400000, 400000, aln.TRACEBACK | 32, -1),
             (aln.Scoring(1, 4, -3, -1, 100, -3), 3000000, 3000000, 0, -3),
             (aln.Scoring(5, 4, -3, -1, 2, -3), 10, 10, 0, -1),
             (aln.Scoring(1, 4, -3, -1, 2, -3), -1, 10, 0, -1)]
    for sc, n, m, flags, e in cases:
        c = sc.c()
        out = ctypes.c_size_t(0)
        st = aln.lib().aln_long_workspace_size(ctypes.byref(c), n, m, flags, ctypes.byref(out))
        assert st == e, (n, m, flags, st)


def test_wait_limits_host_checks():
    """aln_set_wait_limits refuses negative poll counts; 0 restores the defaults (no device work)."""
    assert aln.lib().aln_set_wait_limits(-1, 0) == -1
    assert aln.lib().aln_set_wait_limits(0, -5) == -1
    assert aln.lib().aln_set_wait_limits(0, 0) == 0


def test_traceback_budget_host_checks():
    assert aln.lib().aln_set_traceback_budget(-1) == -1
    assert aln.lib().aln_set_traceback_budget(0) == 0


def test_batch_code_arena_host_checks():
    """aln_set_batch_code_arena refuses a negative size; 0 restores the default (no device work)."""
    assert aln.lib().aln_set_batch_code_arena(-1) == -1
    assert aln.lib().aln_set_batch_code_arena(1 << 20) == 0
    assert aln.lib().aln_set_batch_code_arena(0) == 0
