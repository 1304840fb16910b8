"""Host-side checks of the C-ABI library (no GPU needed, no compute calls)."""
import ctypes
import os
import re

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


def declared_symbols():
    text = open(os.path.join(ROOT, "include", "gcr.h")).read()
    text = re.sub(r"/\*.*?\*/", "", text, flags=re.S)
    return sorted(set(re.findall(r"\b(gcr_[a-z_]+)\s*\(", text)))


def test_header_declares_the_boundary():
    syms = declared_symbols()
    for s in ("gcr_plan_create", "gcr_fill", "gcr_surface", "gcr_forces", "gcr_fill_adjoint",
              "gcr_batch_forward", "gcr_status_str"):
        assert s in syms


def test_library_exports_every_declared_symbol():
    import paper_2609_10165_amd as gcr
    if not os.path.exists(gcr.LIB_PATH):
        pytest.skip("libgcr.so not built (run __graft_entry__.build())")
    L = ctypes.CDLL(gcr.LIB_PATH)
    for s in declared_symbols():
        assert hasattr(L, s), s
    assert set(declared_symbols()) <= set(gcr.SYMBOLS) | {"gcr_version"}


def test_status_strings_and_argument_errors():
    """Error paths that need no device: null arguments are rejected before any
    HIP call."""
    import paper_2609_10165_amd as gcr
    if not os.path.exists(gcr.LIB_PATH):
        pytest.skip("libgcr.so not built")
    L = gcr.lib()
    assert L.gcr_status_str(0) == b"ok"
    assert b"argument" in L.gcr_status_str(1)
    h = ctypes.c_void_p()
    assert L.gcr_plan_create(None, None, 0, None, ctypes.byref(h)) == 1
    assert L.gcr_fill(None, 1, None, None, None, None, None) == 1
    assert L.gcr_plan_stats(None, None) == 1
    assert L.gcr_set_schedule(None, 0, 0) == 1
    g = gcr.make_grid(type("G", (), dict(dim=4, n=(8, 8, 8), lo=(0, 0, 0), h=(1, 1, 1)))())
    s, keep = gcr.make_shape(type("S", (), dict(kind=0, center=(0, 0, 0), r0=1.0))())
    assert L.gcr_plan_create(ctypes.byref(g), ctypes.byref(s), 0, None, ctypes.byref(h)) == 1
    assert L.gcr_plan_create(ctypes.byref(g), ctypes.byref(s), 7, None, ctypes.byref(h)) == 1


def test_process_wide_settings_validate_their_arguments():
    """The process-wide switches take no device call and reject values out of
    their documented ranges (and leave the setting as it was)."""
    import paper_2609_10165_amd as gcr
    if not os.path.exists(gcr.LIB_PATH):
        pytest.skip("libgcr.so not built")
    L = gcr.lib()
    for bad in ((100, 1), (32, 1), (2048, 1), (256, 0), (0, 1), (256, 5), (256, -129)):
        assert L.gcr_set_batch_shape(*bad) == 1, bad
    for ok in ((0, 0), (64, 1), (1024, 4), (256, -1), (512, -128)):
        assert L.gcr_set_batch_shape(*ok) == 0, ok
    assert L.gcr_set_batch_shape(0, 0) == 0
    assert L.gcr_set_batch_tiling(3) == 1 and L.gcr_set_batch_tiling(-1) == 1
    assert L.gcr_set_batch_tiling(1) == 0
    assert L.gcr_set_profiling(4) == 1 and L.gcr_set_profiling(0) == 0
    assert L.gcr_set_wave_residual(65) == 1 and L.gcr_set_wave_residual(-1) == 1
    assert L.gcr_set_wave_residual(64) == 0
    assert L.gcr_set_wide_buffer(4097) == 1 and L.gcr_set_wide_buffer(-1) == 1
    assert L.gcr_set_wide_buffer(0) == 0
