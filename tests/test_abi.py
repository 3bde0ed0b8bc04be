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
    assert cv.version() == 5


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
    bad.engine = 4
    assert L.covest_workspace_size(64, 64, 8, 8, ctypes.byref(bad), ctypes.byref(n)) == cv.ERR_INVALID_ARG
    assert "engine" in L.covest_last_error().decode()
    # the lane engine needs no workspace; it refuses windows beyond its
    # register array (Q > 16), too many lags and rows too long for its LDS
    n.value = 99
    assert L.covest_workspace_size(100, 90, 10, 10, _opts(engine="lane"), ctypes.byref(n)) == cv.OK
    assert n.value == 0
    for shape in [(64, 64, 8, 17), (64, 64, 23, 16), (40, 1000, 10, 10)]:
        assert L.covest_workspace_size(*shape, _opts(engine="lane"), ctypes.byref(n)) == cv.ERR_UNSUPPORTED, shape
        assert "lane engine" in L.covest_last_error().decode()
    assert L.covest_workspace_size(64, 64, 8, 8, _opts(engine="lane", precision="bf16x3", form="recurrence"),
                                   ctypes.byref(n)) == cv.ERR_UNSUPPORTED
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


def test_batched_and_aperture_argument_errors_before_device_use():
    L = cv.lib()
    o = _opts()
    plan = ctypes.c_void_p(0)
    p = cv.covest_problem_ex(16, 16, 64, 64, 64, 64, 8, 8)
    arr = (cv.covest_problem_ex * 1)(p)
    assert L.covest_plan_batched_create_ex(None, arr, 1, o, None) == cv.ERR_INVALID_ARG
    assert L.covest_plan_batched_create_ex(ctypes.byref(plan), arr, 0, o, None) == cv.ERR_INVALID_ARG
    arr[0].lda = 63
    assert L.covest_plan_batched_create_ex(ctypes.byref(plan), arr, 1, o, None) == cv.ERR_INVALID_ARG
    assert "lda" in L.covest_last_error().decode()
    arr[0].lda, arr[0].ldr = 64, 63
    assert L.covest_plan_batched_create_ex(ctypes.byref(plan), arr, 1, o, None) == cv.ERR_INVALID_ARG
    arr[0].ldr, arr[0].P = 64, 65
    assert L.covest_plan_batched_create_ex(ctypes.byref(plan), arr, 1, o, None) == cv.ERR_SHAPE
    assert L.covest_plan_batched_create_ex(ctypes.byref(plan), arr, 1, _opts(form="hankel", precision="fp32"),
                                           None) == cv.ERR_UNSUPPORTED
    assert plan.value is None

    def grid(**kw):
        g = dict(ld=1600, H=1600, W=1600, ap_rows=100, ap_cols=100, row_step=62, col_step=62, n_rows=25,
                 n_cols=25)
        g.update(kw)
        return cv.covest_aperture_grid(16, *[g[k] for k in ("ld", "H", "W", "ap_rows", "ap_cols", "row_step",
                                                            "col_step", "n_rows", "n_cols")])

    def create(g, P=10, Q=10, R=16, opts=o):
        return L.covest_plan_apertures_create(ctypes.byref(plan), ctypes.byref(g), P, Q, ctypes.c_void_p(R),
                                              opts, None)

    assert L.covest_plan_apertures_create(ctypes.byref(plan), None, 10, 10, ctypes.c_void_p(16), o, None) \
        == cv.ERR_INVALID_ARG
    assert create(grid(), R=0) == cv.ERR_INVALID_ARG
    assert create(grid(ld=1599)) == cv.ERR_INVALID_ARG
    assert create(grid(row_step=0)) == cv.ERR_INVALID_ARG
    assert create(grid(n_cols=0)) == cv.ERR_INVALID_ARG
    # the last aperture row starts at 24 * 63 = 1512 and ends at 1612 > 1600
    assert create(grid(row_step=63)) == cv.ERR_SHAPE
    assert "leave" in L.covest_last_error().decode()
    assert create(grid(col_step=63)) == cv.ERR_SHAPE
    assert create(grid(ap_rows=1601)) == cv.ERR_SHAPE
    assert create(grid(), P=101) == cv.ERR_SHAPE
    assert create(grid(ld=1 << 20, H=1 << 20, W=1 << 20, ap_rows=1, ap_cols=1, row_step=1, col_step=1,
                       n_rows=1 << 16, n_cols=1 << 16), P=1, Q=1) == cv.ERR_SHAPE
    assert "2^31" in L.covest_last_error().decode()
    assert create(grid(), P=80, Q=80) == cv.ERR_UNSUPPORTED
    assert create(grid(), opts=_opts(form="hankel", precision="fp32")) == cv.ERR_UNSUPPORTED
    # the lane engine: windows it cannot hold, and no batched plans
    assert create(grid(), P=10, Q=17, opts=_opts(engine="lane")) == cv.ERR_UNSUPPORTED
    assert "lane engine" in L.covest_last_error().decode()
    assert create(grid(), opts=_opts(engine="lane", precision="bf16x3")) == cv.ERR_UNSUPPORTED
    arr[0].P = 8
    assert L.covest_plan_batched_create_ex(ctypes.byref(plan), arr, 1, _opts(engine="lane"), None) \
        == cv.ERR_UNSUPPORTED
    assert "lane" in L.covest_last_error().decode()
    # the largest grid that fits: the last aperture ends exactly at the image edge
    assert create(grid(row_step=62, n_rows=25, H=24 * 62 + 100), opts=_opts(precision="fp16")) \
        == cv.ERR_UNSUPPORTED
    assert plan.value is None


def test_binding_short_names():
    import torch
    assert cv.forward is cv.covest_forward and cv.backward is cv.covest_backward
    assert issubclass(cv.CovEst, torch.autograd.Function)
    assert cv.CovEst is cv.CovEst
    with pytest.raises(AttributeError):
        cv.no_such_name


def test_backward_argument_errors_before_device_use():
    """covest_backward_ex checks pointers, strides, overlap, shape and the
    workspace before any device call; opts->prec picks the element types
    (complex128 for FP64, the NULL-opts default), so the overlap check uses
    16-byte elements there."""
    L = cv.lib()
    A, G, D = ctypes.c_void_p(1 << 20), ctypes.c_void_p(1 << 30), ctypes.c_void_p(1 << 40)
    n = ctypes.c_size_t(0)
    assert L.covest_backward_workspace_size(64, 64, 8, 8, None, ctypes.byref(n)) == cv.OK
    ws, need = ctypes.c_void_p(1 << 44), n.value
    for prec in ("fp64", "fp32"):
        for fill in ("full", "upper"):
            o = _opts(precision=prec, fill=fill)
            # strides
            assert L.covest_backward_ex(A, 63, G, 64, D, 64, 64, 64, 8, 8, o, ws, need, None) == cv.ERR_INVALID_ARG
            assert L.covest_backward_ex(A, 64, G, 63, D, 64, 64, 64, 8, 8, o, ws, need, None) == cv.ERR_INVALID_ARG
            assert "ldr" in L.covest_last_error().decode()
            assert L.covest_backward_ex(A, 64, G, 64, D, 63, 64, 64, 8, 8, o, ws, need, None) == cv.ERR_INVALID_ARG
            # null pointers, shapes, P above the limit
            assert L.covest_backward(None, G, D, 64, 64, 8, 8, o, ws, need, None) == cv.ERR_INVALID_ARG
            assert L.covest_backward(A, G, D, 64, 64, 65, 8, o, ws, need, None) == cv.ERR_SHAPE
            assert L.covest_backward(A, G, D, 300, 300, 65, 8, o, ws, 1 << 40, None) == cv.ERR_UNSUPPORTED
            # workspace
            assert L.covest_backward(A, G, D, 64, 64, 8, 8, o, ws, need - 1, None) == cv.ERR_WORKSPACE
            assert L.covest_backward(A, G, D, 64, 64, 8, 8, o, None, need, None) == cv.ERR_WORKSPACE
    # dA overlapping A (strided: its last row reaches A) or dR, by element size
    o64, o32 = _opts(precision="fp64"), _opts(precision="fp32")
    base = 1 << 20
    # A spans [base, base + 64*64*8); a complex128 dA of 64 x 64 starting 32 KiB
    # before A ends overlaps it
    assert L.covest_backward(ctypes.c_void_p(base), G, ctypes.c_void_p(base + 64 * 64 * 8 - 32768), 64, 64, 8, 8,
                             o64, ws, need, None) == cv.ERR_INVALID_ARG
    assert "overlap" in L.covest_last_error().decode()
    # dR is 64 x 64 complex128 = 64 KiB: a dA right after a complex64-sized dR
    # overlaps only under FP64
    dr_c64 = 64 * 64 * 8
    assert L.covest_backward(A, ctypes.c_void_p(base << 4), ctypes.c_void_p((base << 4) + dr_c64), 64, 64, 8, 8,
                             o64, ws, need, None) == cv.ERR_INVALID_ARG
    assert L.covest_backward(A, ctypes.c_void_p(base << 4), ctypes.c_void_p((base << 4) + dr_c64), 64, 64, 8, 8,
                             o32, None, need, None) == cv.ERR_WORKSPACE   # passes the overlap check
    assert L.covest_backward(A, G, A, 64, 64, 8, 8, None, ws, need, None) == cv.ERR_INVALID_ARG


def test_noalloc_rejections_before_device_work():
    """covest_forward_noalloc checks its arguments and the fixed scratch's
    limit on the host; every case here returns before any device call."""
    L = cv.lib()
    fake = ctypes.c_void_p(0x1000)   # never dereferenced: each call is rejected first
    assert L.covest_forward_noalloc(None, 64, 64, 64, 8, 8, fake, 64, None, None) == cv.ERR_INVALID_ARG
    assert L.covest_forward_noalloc(fake, 63, 64, 64, 8, 8, fake, 64, None, None) == cv.ERR_INVALID_ARG
    assert L.covest_forward_noalloc(fake, 64, 64, 64, 8, 8, fake, 63, None, None) == cv.ERR_INVALID_ARG
    assert L.covest_forward_noalloc(fake, 64, 64, 64, 65, 8, fake, 520, None, None) == cv.ERR_SHAPE
    assert L.covest_forward_noalloc(fake, 64, 64, 64, 8, 8, fake, 64, _opts(form="hankel", precision="fp32"),
                                    None) == cv.ERR_UNSUPPORTED
    assert L.covest_forward_noalloc(fake, 64, 64, 64, 8, 8, fake, 64, _opts(precision="bf16"),
                                    None) == cv.ERR_UNSUPPORTED
    # tables plus workspace beyond the 32 MiB array
    assert L.covest_forward_noalloc(fake, 4096, 4096, 4096, 64, 64, fake, 4096, None, None) == cv.ERR_WORKSPACE
    assert "scratch" in L.covest_last_error().decode()
    n = ctypes.c_size_t(0)
    assert L.covest_workspace_size(4096, 4096, 64, 64, None, ctypes.byref(n)) == cv.OK
    assert n.value > (32 << 20)
    # the headline shape fits
    assert L.covest_workspace_size(1024, 1024, 32, 32, None, ctypes.byref(n)) == cv.OK
    assert n.value < (32 << 20) - (1 << 20)
