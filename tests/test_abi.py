"""The C-ABI library loads, exports every symbol include/sdtw.h declares, and
rejects bad arguments before touching the device (no GPU needed)."""
import ctypes as C
import os
import re

import numpy as np
import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
HEADER = os.path.join(ROOT, "include", "sdtw.h")


def _declared():
    text = open(HEADER).read()
    text = re.sub(r"/\*.*?\*/", "", text, flags=re.S)
    return sorted(set(re.findall(r"\b(sdtw_\w+)\s*\(", text)))


@pytest.fixture(scope="module")
def lib():
    import paper_2211_07340_amd as sd
    if not os.path.exists(sd.library_path()):
        import __graft_entry__
        __graft_entry__.build()
    return sd.load_library()


def test_every_declared_symbol_is_exported(lib):
    names = _declared()
    assert len(names) >= 14
    raw = C.CDLL(os.path.join(ROOT, "paper_2211_07340_amd", "libsdtw.so"))
    missing = [n for n in names if not hasattr(raw, n)]
    assert not missing, missing


def test_version_and_error_string(lib):
    assert lib.sdtw_version() == 1
    assert isinstance(lib.sdtw_last_error(), bytes)


def _err(lib):
    return lib.sdtw_last_error().decode()


def test_plan_validation(lib):
    h = C.c_void_p()
    offs = np.array([0, 5, 5, 9], np.int64)  # read 1 is empty
    rc = lib.sdtw_plan_create(offs.ctypes.data_as(C.c_void_p), 3, 1, C.byref(h))
    assert rc == 1 and "read 1" in _err(lib)
    offs = np.array([0, 5000], np.int64)  # longer than SDTW_MAX_QUERY
    assert lib.sdtw_plan_create(offs.ctypes.data_as(C.c_void_p), 1, 1, C.byref(h)) == 1
    assert lib.sdtw_plan_create(offs.ctypes.data_as(C.c_void_p), 0, 1, C.byref(h)) == 1
    assert lib.sdtw_plan_create(offs.ctypes.data_as(C.c_void_p), 1, 7, C.byref(h)) == 1
    assert lib.sdtw_plan_create(None, 1, 1, C.byref(h)) == 1
    assert h.value is None


def test_argument_validation(lib):
    p = C.c_void_p(1)
    assert lib.sdtw_align_batch(None, None, p, p, p, None) == 1
    assert lib.sdtw_align_one(None, p, 5, p, p, None) == 1
    assert lib.sdtw_align_one_wide(None, p, 5, 0, p, p, None) == 1
    assert lib.sdtw_detect_events(None, p, 1, 0, 5, p, p, None) == 1
    assert lib.sdtw_detect_events(p, p, 0, 0, 5, p, p, None) == 1
    assert lib.sdtw_detect_events(p, p, 1, -1, 5, p, p, None) == 1
    assert lib.sdtw_detect_events(p, p, 1, 0, 0, p, p, None) == 1
    assert lib.sdtw_detect_events(p, p, 1, 3000, 4000, p, p, None) == 1
    assert lib.sdtw_detect_events_prefix(p, None, p, 1, 0, 5, p, p, None) == 1
    assert lib.sdtw_detect_events_prefix(p, p, p, 1, -1, 5, p, p, None) == 1
    assert lib.sdtw_detect_events_prefix(p, p, p, 1, 6000, 500, p, p, None) == 1
    assert lib.sdtw_event_state_bytes() > 0
    assert lib.sdtw_event_state_init(None, p, 1, None) == 1
    assert lib.sdtw_detect_events_continue(p, p, p, None, 1, 0, 5, p, p, None) == 1
    assert lib.sdtw_detect_events_continue(p, p, p, p, 1, 0, 5000, p, p, None) == 1
    assert lib.sdtw_align_one_wide(p, None, 5, 0, p, p, None) == 1
    assert lib.sdtw_load_reference(None, 10, 1, 0, None, C.byref(C.c_void_p())) == 1
    assert lib.sdtw_load_reference(p, 0, 1, 0, None, C.byref(C.c_void_p())) == 1
    assert lib.sdtw_load_reference(p, 10, 9, 0, None, C.byref(C.c_void_p())) == 1
    assert lib.sdtw_prepare_reference(p, 3, p, 6, 64.0, p, p, p, None) == 1  # L < k
    assert lib.sdtw_prepare_reference(p, 100, p, 6, -1.0, p, p, p, None) == 1
    assert lib.sdtw_prepare_queries(p, p, 0, 64.0, p, p, p, None) == 1
    assert lib.sdtw_plan_set_config(None, 16, 2, 1, 4, -1) == 1
    assert lib.sdtw_plan_autotune(None, None, p, p, p, 0, None) == 1
    assert lib.sdtw_plan_use_tuned(None, None, None) == 1
    assert lib.sdtw_stream_set_config(None, 0, 5) == 1
    assert lib.sdtw_stream_best_two(None, 1, 0, p, p, p, p, None) == 1
    assert lib.sdtw_stream_set_config(None, 8, 0) == 1
    assert lib.sdtw_free_reference(None) == 1
    assert lib.sdtw_plan_destroy(None) == 1
    assert "null" in _err(lib)


def test_stream_argument_validation(lib):
    p = C.c_void_p(1)
    assert lib.sdtw_stream_open(None, C.byref(C.c_void_p())) == 1
    assert lib.sdtw_stream_close(None) == 1
    assert lib.sdtw_stream_copy_row(None, p, None) == 1
    assert lib.sdtw_stream_info(None, None, None) == 1
    offs = np.array([0, 10], np.int64)
    assert lib.sdtw_stream_extend(None, 1, p, offs.ctypes.data_as(C.c_void_p), p, p, None) == 1
    arr = (C.c_void_p * 1)(None)
    assert lib.sdtw_stream_extend(arr, 0, p, offs.ctypes.data_as(C.c_void_p), p, p, None) == 1
    assert lib.sdtw_stream_extend(arr, 1, p, offs.ctypes.data_as(C.c_void_p), p, p, None) == 1
    assert lib.sdtw_set_row_budget(-5) == 1
    assert lib.sdtw_prepare_queries_ex(None, p, 1, 64.0, None, None, p, p, p, None) == 1


def test_probe_library_exports_its_header():
    # include/sdtw_probe.h: the issue-rate and LDS probes (libsdtw_probe.so)
    from paper_2211_07340_amd import build as hipbuild
    if not os.path.exists(hipbuild.PROBE_LIB):
        hipbuild.build_probe()
    text = open(os.path.join(ROOT, "include", "sdtw_probe.h")).read()
    text = re.sub(r"/\*.*?\*/", "", text, flags=re.S)
    names = sorted(set(re.findall(r"\b(sdtw_\w+)\s*\(", text)))
    assert names == ["sdtw_probe_issue", "sdtw_probe_lds", "sdtw_probe_placement"]
    raw = C.CDLL(hipbuild.PROBE_LIB)
    assert all(hasattr(raw, n) for n in names)
    # bad arguments are rejected before any device call
    raw.sdtw_probe_issue.argtypes = [C.c_int] * 4 + [C.c_void_p] * 2
    raw.sdtw_probe_lds.argtypes = [C.c_int] * 3 + [C.c_void_p] * 2
    raw.sdtw_probe_placement.argtypes = [C.c_int] * 5 + [C.c_void_p] * 2
    out = C.c_void_p(1)
    assert raw.sdtw_probe_issue(5, 1, 1, 1, out, None) == 1      # no such kind
    assert raw.sdtw_probe_issue(0, 3, 1, 1, out, None) == 1      # chains
    assert raw.sdtw_probe_issue(0, 1, 9, 1, out, None) == 1      # waves per SIMD
    assert raw.sdtw_probe_issue(0, 1, 1, 1, None, None) == 1     # no output
    assert raw.sdtw_probe_lds(0, 1, 1, out, None) == 1           # lanes
    assert raw.sdtw_probe_lds(65, 1, 1, out, None) == 1
    assert raw.sdtw_probe_lds(1, 1, 0, out, None) == 1           # iterations
    assert raw.sdtw_probe_placement(16, 96, 0, 0, 0, out, None) == 1  # not whole waves
    assert raw.sdtw_probe_placement(16, 128, 200000, 0, 0, out, None) == 1  # LDS
    assert raw.sdtw_probe_placement(16, 128, 0, 100, 0, out, None) == 1  # registers
    assert raw.sdtw_probe_placement(16, 128, 0, 0, 0, None, None) == 1
