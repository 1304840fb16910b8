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
