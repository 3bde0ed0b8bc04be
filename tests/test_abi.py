"""The C ABI loads, exports what its headers declare, and rejects bad arguments
before touching a device (no GPU needed)."""
import ctypes
import os
import re

import pytest

from paper_1303_2285_amd import covest as cv

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
HEADERS = [os.path.join(ROOT, "include", h) for h in ("covest.h", "covest_plan.h")]


def declared_functions():
    names = set()
    for h in HEADERS:
        text = open(h).read()
        text = re.sub(r"/\*.*?\*/", "", text, flags=re.S)
        for m in re.finditer(r"^\s*(?:const\s+)?\w+\s*\*?\s*(covest_\w+)\s*\(", text, flags=re.M):
            names.add(m.group(1))
    return names


def test_every_declared_symbol_is_exported():
    names = declared_functions()
    assert len(names) >= 16
    L = ctypes.CDLL(cv.LIB_PATH)
    for n in sorted(names):
        assert hasattr(L, n), n
    # and the binding knows every one of them
    assert names == set(cv.SIGNATURES), names ^ set(cv.SIGNATURES)


def test_version():
    assert cv.version() == 2


def _opts(**kw):
    return ctypes.byref(cv.make_opts(**kw))


def test_workspace_query_errors():
    L = cv.lib()
    n = ctypes.c_size_t(0)
    assert L.covest_workspace_size(64, 64, 8, 8, _opts(), None) == cv.ERR_INVALID_ARG
    assert L.covest_workspace_size(64, 64, 65, 8, _opts(), ctypes.byref(n)) == cv.ERR_SHAPE
    assert L.covest_workspace_size(64, 64, 8, 0, _opts(), ctypes.byref(n)) == cv.ERR_SHAPE
    bad = cv.make_opts()
    bad.prec = 17
    assert L.covest_workspace_size(64, 64, 8, 8, ctypes.byref(bad), ctypes.byref(n)) == cv.ERR_INVALID_ARG
    assert "precision" in L.covest_last_error().decode()
    bad = cv.make_opts()
    bad.form = 9
    assert L.covest_workspace_size(64, 64, 8, 8, ctypes.byref(bad), ctypes.byref(n)) == cv.ERR_INVALID_ARG
    assert L.covest_workspace_size(300, 300, 80, 8, _opts(form="recurrence"), ctypes.byref(n)) \
        == cv.ERR_UNSUPPORTED
    bad = cv.make_opts(ring_cols=6)
    assert L.covest_workspace_size(64, 64, 8, 8, ctypes.byref(bad), ctypes.byref(n)) == cv.ERR_INVALID_ARG
    bad = cv.make_opts()
    bad.engine = 3
    assert L.covest_workspace_size(64, 64, 8, 8, ctypes.byref(bad), ctypes.byref(n)) == cv.ERR_INVALID_ARG
    assert "engine" in L.covest_last_error().decode()
    # the matrix-core engine: not where its kernel cannot run (Q < 4, N < 2P - 1);
    # its own plan where it can
    assert L.covest_workspace_size(64, 64, 8, 3, _opts(engine="matrix"), ctypes.byref(n)) == cv.ERR_UNSUPPORTED
    assert L.covest_workspace_size(64, 64, 40, 8, _opts(engine="matrix"), ctypes.byref(n)) == cv.ERR_UNSUPPORTED
    assert L.covest_workspace_size(64, 64, 8, 8, _opts(engine="matrix"), ctypes.byref(n)) == cv.OK
    assert n.value == cv.mfma_plan(64, 64, 8, 8)[0]["ws_bytes"]
    assert L.covest_workspace_size(1024, 1024, 32, 32, _opts(engine="matrix"), ctypes.byref(n)) == cv.OK
    assert n.value == cv.mfma_plan(1024, 1024, 32, 32)[0]["ws_bytes"]
    assert L.covest_workspace_size(1024, 1024, 32, 32, _opts(engine="vector"), ctypes.byref(n)) == cv.OK
    assert n.value == cv.plan_info(1024, 1024, 32, 32)["ws_bytes"]
    m = ctypes.c_size_t(0)
    assert L.covest_workspace_size(1024, 1024, 32, 32, _opts(), ctypes.byref(m)) == cv.OK
    assert m.value == max(n.value, cv.mfma_plan(1024, 1024, 32, 32)[0]["ws_bytes"])
    # AUTO takes the matrix cores for 8 x 8 too, and covers the vector plan it
    # falls back to for inputs too large for 32-bit offsets
    assert L.covest_workspace_size(64, 64, 8, 8, None, ctypes.byref(n)) == cv.OK
    assert n.value == max(cv.plan_info(64, 64, 8, 8)["ws_bytes"], cv.mfma_plan(64, 64, 8, 8)[0]["ws_bytes"])
    # ... but not for a 64 x 4 window (8 tiles, three quarters padding)
    assert L.covest_workspace_size(300, 300, 64, 4, None, ctypes.byref(n)) == cv.OK
    assert n.value == cv.plan_info(300, 300, 64, 4)["ws_bytes"]


def test_forward_argument_errors_before_device_use():
    L = cv.lib()
    o = _opts()
    # null A / R
    assert L.covest_forward(None, 64, 64, 8, 8, ctypes.c_void_p(16), o, None, 0, None) == cv.ERR_INVALID_ARG
    assert L.covest_forward(ctypes.c_void_p(16), 64, 64, 8, 8, None, o, None, 0, None) == cv.ERR_INVALID_ARG
    # shapes
    assert L.covest_forward(ctypes.c_void_p(16), 4, 4, 5, 1, ctypes.c_void_p(16), o, None, 0, None) == cv.ERR_SHAPE
    # leading dimensions
    assert L.covest_forward_ex(ctypes.c_void_p(16), 63, 64, 64, 8, 8, ctypes.c_void_p(16), 64, o, None, 0,
                               None) == cv.ERR_INVALID_ARG
    assert L.covest_forward_ex(ctypes.c_void_p(16), 64, 64, 64, 8, 8, ctypes.c_void_p(16), 63, o, None, 0,
                               None) == cv.ERR_INVALID_ARG
    assert "ldr" in L.covest_last_error().decode()


def test_counts_need_output():
    assert cv.lib().covest_counts(4, 4, 2, 2, None) == cv.ERR_INVALID_ARG


def test_timing_calls_without_device():
    cv.timing_enable(True)
    cv.timing_reset()
    assert cv.timing_read() == {}
    cv.timing_enable(False)
