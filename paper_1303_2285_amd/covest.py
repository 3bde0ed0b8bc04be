"""Thin ctypes binding of libcovest (include/covest.h).

Argument marshalling only: every step of the computation runs in the library's
HIP kernels.  PyTorch supplies device memory and the current stream.  If the
built library is missing the import fails loudly; there is no fallback path.

    R = covest_forward(A, P, Q)                 # complex128 R on A's device
    dA = covest_backward(A, dR, P, Q)
    plan = BatchedPlan([(A0, P0, Q0), ...]); plan.run(); plan.outputs
    plan = AperturePlan(image, 100, 100, 62, 62, 25, 25, 10, 10); plan.run()
"""
from __future__ import annotations

import ctypes
import os
from dataclasses import dataclass

HERE = os.path.dirname(os.path.abspath(__file__))
# the in-tree build; COVEST_LIB names another build of the same library (e.g. to compare two)
LIB_PATH = os.environ.get("COVEST_LIB") or os.path.join(HERE, "libcovest.so")

OK = 0
ERR_INVALID_ARG = -1
ERR_SHAPE = -2
ERR_WORKSPACE = -3
ERR_HIP = -4
ERR_UNSUPPORTED = -5
ERR_PLAN_MISMATCH = -6

FORMS = {"auto": 0, "recurrence": 1, "hankel": 2, "hankel_mfma": 2}
PRECS = {"fp64": 0, "fp32": 1, "bf16x3": 2, "fp16x3": 3, "bf16": 4, "fp16": 5}
FILLS = {"full": 0, "upper": 1}
ENGINES = {"auto": 0, "vector": 1, "matrix": 2, "lane": 3}


class CovestError(RuntimeError):
    def __init__(self, status: int, message: str):
        super().__init__(f"libcovest status {status}: {message}")
        self.status = status


class covest_opts(ctypes.Structure):
    _fields_ = [("form", ctypes.c_int), ("prec", ctypes.c_int), ("fill", ctypes.c_int),
                ("normalize", ctypes.c_int), ("ring_cols", ctypes.c_int), ("ring_rows", ctypes.c_int),
                ("engine", ctypes.c_int)]


class covest_counts_t(ctypes.Structure):
    _fields_ = [("K", ctypes.c_int64), ("n_uc", ctypes.c_int64), ("um", ctypes.c_int64),
                ("eta", ctypes.c_int64), ("segments", ctypes.c_int64)]


class covest_problem(ctypes.Structure):
    _fields_ = [("A", ctypes.c_void_p), ("R", ctypes.c_void_p), ("N", ctypes.c_int32),
                ("M", ctypes.c_int32), ("P", ctypes.c_int32), ("Q", ctypes.c_int32)]


class covest_problem_ex(ctypes.Structure):
    _fields_ = [("A", ctypes.c_void_p), ("R", ctypes.c_void_p), ("lda", ctypes.c_int64),
                ("ldr", ctypes.c_int64), ("N", ctypes.c_int32), ("M", ctypes.c_int32),
                ("P", ctypes.c_int32), ("Q", ctypes.c_int32)]


class covest_aperture_grid(ctypes.Structure):
    _fields_ = [("image", ctypes.c_void_p)] + \
               [(n, ctypes.c_int64) for n in ("ld", "H", "W", "ap_rows", "ap_cols", "row_step", "col_step",
                                              "n_rows", "n_cols")]


class covest_timing_record(ctypes.Structure):
    _fields_ = [("name", ctypes.c_char * 48), ("launches", ctypes.c_int64),
                ("total_ms", ctypes.c_double)]


class covest_plan_info(ctypes.Structure):
    _fields_ = [(n, ctypes.c_int32) for n in ("W0", "W1", "Rm0", "Rm1", "Cm0", "Cm1", "n_ir", "n_ic",
                                               "lag_stride", "bandw", "n_bulk", "n_jobs", "n_groups",
                                               "n_items")] + \
               [(n, ctypes.c_int64) for n in ("ws_bytes", "lds_main", "lds_fin", "main_products",
                                               "fin_products")]


class covest_mfma_plan_info(ctypes.Structure):
    _fields_ = [(n, ctypes.c_int32) for n in ("mt", "nt", "Rm0", "Rm1", "Cm0", "Cm1", "n_ir", "n_ic",
                                               "lag_stride", "n_bulk", "n_jobs", "n_items", "zpieces")] + \
               [(n, ctypes.c_int64) for n in ("ws_bytes", "lds_main", "lds_fin", "main_products",
                                              "fin_products")]


class covest_lane_plan_info(ctypes.Structure):
    _fields_ = [(n, ctypes.c_int32) for n in ("fits", "qmax", "ring", "gstride", "chunk", "chain", "n_blocks",
                                               "threads")] + [("lds", ctypes.c_int64)]


class covest_hankel_plan_info(ctypes.Structure):
    _fields_ = [(n, ctypes.c_int32) for n in ("pb", "qb", "stride_a", "stride_b", "tm", "tn", "npl", "ldp",
                                               "n_items", "n_tiles", "n_index")] + \
               [(n, ctypes.c_int64) for n in ("lds", "ws_bytes", "planes_bytes")]


# Every symbol the headers declare, with its ctypes signature.
_i64 = ctypes.c_int64
_vp = ctypes.c_void_p
_int = ctypes.c_int
SIGNATURES = {
    "covest_counts": (_int, [_i64, _i64, _i64, _i64, ctypes.POINTER(covest_counts_t)]),
    "covest_workspace_size": (_int, [_i64, _i64, _i64, _i64, ctypes.POINTER(covest_opts),
                                     ctypes.POINTER(ctypes.c_size_t)]),
    "covest_forward": (_int, [_vp, _i64, _i64, _i64, _i64, _vp, ctypes.POINTER(covest_opts), _vp,
                              ctypes.c_size_t, _vp]),
    "covest_forward_ex": (_int, [_vp, _i64, _i64, _i64, _i64, _i64, _vp, _i64,
                                 ctypes.POINTER(covest_opts), _vp, ctypes.c_size_t, _vp]),
    "covest_forward_noalloc": (_int, [_vp, _i64, _i64, _i64, _i64, _i64, _vp, _i64,
                                      ctypes.POINTER(covest_opts), _vp]),
    "covest_backward_workspace_size": (_int, [_i64, _i64, _i64, _i64, ctypes.POINTER(covest_opts),
                                              ctypes.POINTER(ctypes.c_size_t)]),
    "covest_backward": (_int, [_vp, _vp, _vp, _i64, _i64, _i64, _i64, ctypes.POINTER(covest_opts),
                               _vp, ctypes.c_size_t, _vp]),
    "covest_backward_ex": (_int, [_vp, _i64, _vp, _i64, _vp, _i64, _i64, _i64, _i64, _i64,
                                  ctypes.POINTER(covest_opts), _vp, ctypes.c_size_t, _vp]),
    "covest_plan_batched_create": (_int, [ctypes.POINTER(_vp), ctypes.POINTER(covest_problem), _i64,
                                          ctypes.POINTER(covest_opts), _vp]),
    "covest_plan_batched_create_ex": (_int, [ctypes.POINTER(_vp), ctypes.POINTER(covest_problem_ex), _i64,
                                             ctypes.POINTER(covest_opts), _vp]),
    "covest_plan_apertures_create": (_int, [ctypes.POINTER(_vp), ctypes.POINTER(covest_aperture_grid), _i64,
                                            _i64, _vp, ctypes.POINTER(covest_opts), _vp]),
    "covest_forward_batched": (_int, [_vp, _vp]),
    "covest_capon_workspace_size": (_int, [_i64, _i64, _i64, _i64, ctypes.POINTER(ctypes.c_size_t)]),
    "covest_capon_spectrum": (_int, [_vp, _i64, _i64, _i64, _i64, _i64, _vp, _vp, ctypes.c_size_t, _vp]),
    "covest_plan_destroy": (_int, [_vp]),
    "covest_timing_enable": (_int, [_int]),
    "covest_timing_reset": (_int, []),
    "covest_timing_read": (_int, [ctypes.POINTER(covest_timing_record), _int]),
    "covest_last_error": (ctypes.c_char_p, []),
    "covest_version": (_int, []),
    # include/covest_plan.h
    "covest_plan_info_get": (_int, [_i64, _i64, _i64, _i64, ctypes.c_int32, ctypes.c_int32,
                                    ctypes.c_int32, ctypes.POINTER(covest_plan_info)]),
    "covest_plan_tables": (_int, [_i64, _i64, _i64, _i64, ctypes.c_int32, ctypes.c_int32,
                                  ctypes.c_int32, ctypes.c_void_p, ctypes.c_void_p, ctypes.c_void_p]),
    "covest_mfma_plan_get": (_int, [_i64, _i64, _i64, _i64, ctypes.c_int32,
                                    ctypes.POINTER(covest_mfma_plan_info), ctypes.c_void_p, ctypes.c_void_p]),
    "covest_forward_stamped": (_int, [_vp, _i64, _i64, _i64, _i64, _vp, ctypes.POINTER(covest_opts), _vp,
                                      ctypes.c_size_t, _vp, _i64, _vp, _vp]),
    "covest_hankel_plan_get": (_int, [_i64, _i64, _i64, _i64, ctypes.c_int32, ctypes.c_int32,
                                      ctypes.POINTER(covest_hankel_plan_info), _vp, _vp, _vp]),
    "covest_engine_choice": (_int, [_i64, _i64, _i64, _i64, ctypes.c_int32, ctypes.POINTER(ctypes.c_int32),
                                    ctypes.POINTER(ctypes.c_int32)]),
    "covest_lane_plan_get": (_int, [_i64, _i64, _i64, _i64, _i64, _i64, _i64, ctypes.c_int32,
                                    ctypes.POINTER(covest_lane_plan_info)]),
}

_lib = None


def lib():
    """Load libcovest.so (built in-tree by __graft_entry__.build())."""
    global _lib
    if _lib is None:
        if not os.path.exists(LIB_PATH):
            raise ImportError(f"libcovest.so is not built ({LIB_PATH}); run __graft_entry__.build()")
        # PyTorch ships its own HIP runtime under the same soname.  Load it
        # first so that libcovest binds to that one copy; a second runtime in
        # the process would not see the device.
        import torch  # noqa: F401
        L = ctypes.CDLL(LIB_PATH)
        for name, (res, args) in SIGNATURES.items():
            f = getattr(L, name)
            f.restype = res
            f.argtypes = args
        _lib = L
    return _lib


def _check(status: int):
    if status != OK:
        msg = lib().covest_last_error().decode(errors="replace")
        raise CovestError(status, msg)


def make_opts(form="auto", precision="fp64", fill="full", normalize=True, ring_cols=0,
              ring_rows=0, engine="auto") -> covest_opts:
    o = covest_opts()
    o.form = FORMS[form] if isinstance(form, str) else int(form)
    o.prec = PRECS[precision] if isinstance(precision, str) else int(precision)
    o.fill = FILLS[fill] if isinstance(fill, str) else int(fill)
    o.normalize = 1 if normalize else 0
    o.ring_cols = int(ring_cols)
    o.ring_rows = int(ring_rows)
    o.engine = ENGINES[engine] if isinstance(engine, str) else int(engine)
    return o


def counts(N: int, M: int, P: int, Q: int) -> dict:
    """K, |UC|, UM, eta and the segment count of the method for one shape (host only)."""
    c = covest_counts_t()
    _check(lib().covest_counts(N, M, P, Q, ctypes.byref(c)))
    return {"K": c.K, "n_uc": c.n_uc, "um": c.um, "eta": c.eta, "segments": c.segments}


_ws_cache: dict = {}


def workspace_size(N, M, P, Q, **kw) -> int:
    key = (N, M, P, Q, tuple(sorted(kw.items())))
    if key not in _ws_cache:
        o = make_opts(**kw)
        n = ctypes.c_size_t(0)
        _check(lib().covest_workspace_size(N, M, P, Q, ctypes.byref(o), ctypes.byref(n)))
        _ws_cache[key] = int(n.value)
    return _ws_cache[key]


def backward_workspace_size(N, M, P, Q, **kw) -> int:
    o = make_opts(**kw)
    n = ctypes.c_size_t(0)
    _check(lib().covest_backward_workspace_size(N, M, P, Q, ctypes.byref(o), ctypes.byref(n)))
    return int(n.value)


def _torch():
    import torch
    return torch


def _stream_handle(device):
    torch = _torch()
    return ctypes.c_void_p(torch.cuda.current_stream(device).cuda_stream)


def _check_input(A):
    torch = _torch()
    if not isinstance(A, torch.Tensor) or not A.is_cuda:
        raise TypeError("A must be a CUDA (HIP) tensor")
    if A.dtype != torch.complex64:
        raise TypeError("A must be complex64")
    if A.dim() != 2:
        raise ValueError("A must be 2-D (N x M)")
    if A.stride(1) != 1:
        raise ValueError("A must have unit column stride")


def _workspace(nbytes: int, device):
    torch = _torch()
    if nbytes == 0:
        return None, 0
    return torch.empty(nbytes, dtype=torch.uint8, device=device), nbytes


def covest_forward(A, P: int, Q: int, *, form="auto", precision="fp64", fill="full",
                   normalize=True, out=None, workspace=None, ring_cols=0, ring_rows=0, engine="auto"):
    """R = (1/K) sum_{p,q} V^{p,q} (V^{p,q})^H for the complex64 N x M tensor A.

    Returns a PQ x PQ tensor (complex128 for precision "fp64", complex64
    otherwise) on A's device, computed on the current stream.  `engine`
    ("auto", "vector", "matrix") picks the units of the recurrence's main pass.
    """
    torch = _torch()
    _check_input(A)
    N, M = A.shape
    o = make_opts(form, precision, fill, normalize, ring_cols, ring_rows, engine)
    PQ = P * Q
    rdtype = torch.complex128 if o.prec == 0 else torch.complex64
    if out is None:
        R = torch.empty((PQ, PQ), dtype=rdtype, device=A.device)
        if fill == "upper":
            R.zero_()
    else:
        R = out
        if R.dtype != rdtype or R.shape != (PQ, PQ) or R.stride(1) != 1:
            raise ValueError("out has the wrong dtype, shape or layout")
    need = workspace_size(N, M, P, Q, form=form, precision=precision, fill=fill,
                          normalize=normalize, ring_cols=ring_cols, ring_rows=ring_rows, engine=engine)
    if workspace is None or workspace.numel() < need:
        ws, nbytes = _workspace(need, A.device)
    else:
        ws, nbytes = workspace, workspace.numel()
    _check(lib().covest_forward_ex(
        ctypes.c_void_p(A.data_ptr()), A.stride(0), N, M, P, Q, ctypes.c_void_p(R.data_ptr()),
        R.stride(0), ctypes.byref(o), ctypes.c_void_p(ws.data_ptr() if ws is not None else 0),
        nbytes, _stream_handle(A.device)))
    return R


def covest_forward_noalloc(A, P: int, Q: int, out, *, precision="fp64", fill="full", normalize=True,
                           engine="auto"):
    """covest_forward's recurrence into the caller's `out` (PQ x PQ, complex128
    for "fp64", complex64 for "fp32", unit column stride) with no device
    allocation: the library's fixed per-GPU scratch holds its tables and
    workspace.  Calls on one GPU share that scratch, so they must not overlap."""
    _check_input(A)
    N, M = A.shape
    o = make_opts("recurrence", precision, fill, normalize, 0, 0, engine)
    torch = _torch()
    rdtype = torch.complex128 if o.prec == 0 else torch.complex64
    if out.dtype != rdtype or tuple(out.shape) != (P * Q, P * Q) or out.stride(1) != 1:
        raise ValueError("out has the wrong dtype, shape or layout")
    if out.device != A.device:
        raise ValueError("out must be on A's device")
    _check(lib().covest_forward_noalloc(
        ctypes.c_void_p(A.data_ptr()), A.stride(0), N, M, P, Q, ctypes.c_void_p(out.data_ptr()),
        out.stride(0), ctypes.byref(o), _stream_handle(A.device)))
    return out


def covest_backward(A, dR, P: int, Q: int, *, normalize=True, fill="full", precision=None, out=None,
                    workspace=None):
    """dA = fold(H X) / K with H = dR + dR^H (fill "full") or triu(dR) + triu(dR)^H
    (fill "upper": the gradient of an upper-only R).

    precision "fp64" takes a complex128 dR and returns complex128 dA; "fp32"
    takes and returns complex64; None follows dR's dtype.  A and dR may be
    strided views with unit column stride; `out` (N x M, the same dtype,
    unit column stride) receives dA if given.
    """
    torch = _torch()
    _check_input(A)
    N, M = A.shape
    if precision is None:
        precision = "fp64" if dR.dtype == torch.complex128 else "fp32"
    if precision not in ("fp64", "fp32"):
        raise ValueError("the adjoint's precision is fp64 or fp32")
    gdtype = torch.complex128 if precision == "fp64" else torch.complex64
    o = make_opts("auto", precision, fill, normalize)
    if dR.dtype != gdtype or dR.stride(-1) != 1:
        dR = dR.to(gdtype).contiguous()
    if dR.shape != (P * Q, P * Q):
        raise ValueError("dR must be PQ x PQ")
    if out is None:
        dA = torch.empty((N, M), dtype=gdtype, device=A.device)
    else:
        dA = out
        if dA.dtype != gdtype or dA.shape != (N, M) or dA.stride(1) != 1:
            raise ValueError("out has the wrong dtype, shape or layout")
    need = backward_workspace_size(N, M, P, Q, precision=precision, normalize=normalize)
    ws, nbytes = _workspace(need, A.device) if workspace is None else (workspace, workspace.numel())
    _check(lib().covest_backward_ex(
        ctypes.c_void_p(A.data_ptr()), A.stride(0), ctypes.c_void_p(dR.data_ptr()), dR.stride(0),
        ctypes.c_void_p(dA.data_ptr()), dA.stride(0), N, M, P, Q, ctypes.byref(o),
        ctypes.c_void_p(ws.data_ptr() if ws is not None else 0), nbytes, _stream_handle(A.device)))
    return dA


@dataclass
class _Problem:
    A: object
    P: int
    Q: int


class _PlanHandle:
    """Owns a covest_plan: run() replays its graph on the current stream."""

    def run(self):
        _check(lib().covest_forward_batched(self._handle, _stream_handle(self._device)))
        return self.outputs

    def close(self):
        if self._handle and self._handle.value:
            lib().covest_plan_destroy(self._handle)
            self._handle = ctypes.c_void_p(0)

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass


class BatchedPlan(_PlanHandle):
    """Many (A, P, Q) problems computed by one graph launch (covest_forward_batched).

    Each A may be a strided view (unit column stride, any row stride), e.g. a
    block of a larger image."""

    def __init__(self, problems, precision="fp64", fill="full", normalize=True, ring_cols=0,
                 ring_rows=0, engine="auto"):
        torch = _torch()
        self._handle = ctypes.c_void_p(0)
        self._problems = [_Problem(A, int(P), int(Q)) for (A, P, Q) in problems]
        o = make_opts("recurrence", precision, fill, normalize, ring_cols, ring_rows, engine)
        rdtype = torch.complex128 if o.prec == 0 else torch.complex64
        arr = (covest_problem_ex * len(self._problems))()
        self.outputs = []
        for i, pr in enumerate(self._problems):
            _check_input(pr.A)
            N, M = pr.A.shape
            R = torch.empty((pr.P * pr.Q, pr.P * pr.Q), dtype=rdtype, device=pr.A.device)
            if fill == "upper":
                R.zero_()
            self.outputs.append(R)
            arr[i] = covest_problem_ex(pr.A.data_ptr(), R.data_ptr(), pr.A.stride(0), pr.P * pr.Q,
                                       N, M, pr.P, pr.Q)
        dev = self._problems[0].A.device if self._problems else torch.device("cuda")
        self._device = dev
        _check(lib().covest_plan_batched_create_ex(ctypes.byref(self._handle), arr, len(self._problems),
                                                   ctypes.byref(o), _stream_handle(dev)))


class AperturePlan(_PlanHandle):
    """R of every aperture of one image (covest_plan_apertures_create).

    Aperture (a, b) is image[a*row_step : a*row_step + ap_rows,
    b*col_step : b*col_step + ap_cols]; `outputs` is one tensor of shape
    (n_rows, n_cols, PQ, PQ), complex128 for precision "fp64"."""

    def __init__(self, image, ap_rows, ap_cols, row_step, col_step, n_rows, n_cols, P, Q,
                 precision="fp64", fill="full", normalize=True, engine="auto"):
        torch = _torch()
        self._handle = ctypes.c_void_p(0)
        _check_input(image)
        o = make_opts("recurrence", precision, fill, normalize, 0, 0, engine)
        rdtype = torch.complex128 if o.prec == 0 else torch.complex64
        PQ = int(P) * int(Q)
        alloc = torch.zeros if fill == "upper" else torch.empty
        self.outputs = alloc((int(n_rows), int(n_cols), PQ, PQ), dtype=rdtype, device=image.device)
        self.image = image
        self._device = image.device
        g = covest_aperture_grid(image.data_ptr(), image.stride(0), image.shape[0], image.shape[1],
                                 int(ap_rows), int(ap_cols), int(row_step), int(col_step), int(n_rows),
                                 int(n_cols))
        _check(lib().covest_plan_apertures_create(ctypes.byref(self._handle), ctypes.byref(g), int(P), int(Q),
                                                  ctypes.c_void_p(self.outputs.data_ptr()), ctypes.byref(o),
                                                  _stream_handle(image.device)))


def covest_capon_spectrum(R, P: int, Q: int, F1: int, F2: int, *, workspace=None):
    """Minimum-variance (Capon) spectrum 1 / Re(a^H R^{-1} a) of each R on the
    grid w = -pi + 2 pi f / F (covest_capon_spectrum).  R: complex128 tensor of
    shape (PQ, PQ) or (count, PQ, PQ), or a (n_rows, n_cols, PQ, PQ) aperture
    output; returns float64 of shape R.shape[:-2] + (F1, F2)."""
    torch = _torch()
    if not isinstance(R, torch.Tensor) or not R.is_cuda or R.dtype != torch.complex128:
        raise TypeError("R must be a complex128 CUDA (HIP) tensor")
    PQ = int(P) * int(Q)
    if R.dim() < 2 or R.shape[-2:] != (PQ, PQ):
        raise ValueError("R must end in PQ x PQ")
    lead = tuple(R.shape[:-2])
    Rc = R.reshape(-1, PQ, PQ).contiguous()
    count = Rc.shape[0]
    S = torch.empty((count, int(F1), int(F2)), dtype=torch.float64, device=R.device)
    n = ctypes.c_size_t(0)
    _check(lib().covest_capon_workspace_size(count, P, Q, F1, ctypes.byref(n)))
    ws, nbytes = _workspace(int(n.value), R.device) if workspace is None else (workspace, workspace.numel())
    _check(lib().covest_capon_spectrum(ctypes.c_void_p(Rc.data_ptr()), count, P, Q, F1, F2,
                                       ctypes.c_void_p(S.data_ptr()),
                                       ctypes.c_void_p(ws.data_ptr() if ws is not None else 0), nbytes,
                                       _stream_handle(R.device)))
    return S.reshape(lead + (int(F1), int(F2)))


def covest_forward_batched(plan: BatchedPlan):
    return plan.run()


def _make_autograd():
    import torch

    class CovEst(torch.autograd.Function):
        """R = covest_forward(A, P, Q) with the hand-written adjoint as backward.

        The forward returns the full Hermitian R (complex128 for precision
        "fp64").  The backward receives dL/dR in PyTorch's convention and returns
        dL/dA = fold((dR + dR^H) X) / K from covest_backward (complex64).
        """

        @staticmethod
        def forward(ctx, A, P, Q, precision="fp64", normalize=True):
            R = covest_forward(A.detach(), P, Q, precision=precision, fill="full", normalize=normalize)
            ctx.save_for_backward(A)
            ctx.P, ctx.Q, ctx.normalize = int(P), int(Q), bool(normalize)
            return R

        @staticmethod
        def backward(ctx, gR):
            (A,) = ctx.saved_tensors
            dA = covest_backward(A.detach(), gR.to(torch.complex64).contiguous(), ctx.P, ctx.Q,
                                 normalize=ctx.normalize, precision="fp32")
            return dA, None, None, None, None

    return CovEst


_covest_fn = None


def _autograd_fn():
    global _covest_fn
    if _covest_fn is None:
        _covest_fn = _make_autograd()
    return _covest_fn


def covest_apply(A, P, Q, precision="fp64", normalize=True):
    """Differentiable forward: CovEst.apply(A, P, Q, precision, normalize)."""
    return _autograd_fn().apply(A, P, Q, precision, normalize)


# short names: covest.forward(A, P, Q), covest.backward(A, dR, P, Q), covest.CovEst.apply(A, P, Q)
forward = covest_forward
backward = covest_backward


def __getattr__(name):
    if name == "CovEst":
        return _autograd_fn()
    raise AttributeError(f"module {__name__!r} has no attribute {name!r}")


# ---------------------------------------------------------------- timing ----

def timing_enable(on: bool = True):
    _check(lib().covest_timing_enable(1 if on else 0))


def timing_reset():
    _check(lib().covest_timing_reset())


def timing_read() -> dict:
    recs = (covest_timing_record * 64)()
    n = lib().covest_timing_read(recs, 64)
    if n < 0:
        _check(n)
    return {recs[i].name.decode(): (int(recs[i].launches), float(recs[i].total_ms))
            for i in range(min(n, 64))}


def plan_info(N, M, P, Q, n_slots=512, w0=0, w1=0) -> dict:
    """The recurrence plan's geometry for one shape (host only)."""
    info = covest_plan_info()
    _check(lib().covest_plan_info_get(N, M, P, Q, n_slots, w0, w1, ctypes.byref(info)))
    return {name: getattr(info, name) for name, _ in covest_plan_info._fields_}


def plan_tables(N, M, P, Q, n_slots=512, w0=0, w1=0):
    """(jobs[n,12], groups[n,14], items[n,5]) int32 arrays of the recurrence plan."""
    import numpy as np
    info = plan_info(N, M, P, Q, n_slots, w0, w1)
    jobs = np.zeros((info["n_jobs"], 12), dtype=np.int32)
    groups = np.zeros((info["n_groups"], 14), dtype=np.int32)
    items = np.zeros((info["n_items"], 5), dtype=np.int32)
    _check(lib().covest_plan_tables(N, M, P, Q, n_slots, w0, w1, jobs.ctypes.data,
                                    groups.ctypes.data, items.ctypes.data))
    return info, jobs, groups, items


def version() -> int:
    return int(lib().covest_version())


def mfma_plan(N, M, P, Q, n_cu=256):
    """(info, jobs[n,16], items[n,5]) of the matrix-core engine's plan (host only)."""
    import numpy as np
    info = covest_mfma_plan_info()
    _check(lib().covest_mfma_plan_get(N, M, P, Q, n_cu, ctypes.byref(info), None, None))
    d = {name: getattr(info, name) for name, _ in covest_mfma_plan_info._fields_}
    jobs = np.zeros((d["n_jobs"], 16), dtype=np.int32)
    items = np.zeros((d["n_items"], 5), dtype=np.int32)
    _check(lib().covest_mfma_plan_get(N, M, P, Q, n_cu, ctypes.byref(info), jobs.ctypes.data,
                                      items.ctypes.data))
    return d, jobs, items


def covest_forward_stamped(A, P: int, Q: int, *, engine="auto"):
    """covest_forward (FP64) plus, per finalize item (one unique combination),
    the 100 MHz wall clock at its workgroup's start and end.  Returns
    (R, stamps[n_uc, 2] int64 on the device, items[n_uc, 5] int32 host:
    inst, dr, dc, bulk0, bulk1).  A measurement call."""
    import numpy as np
    torch = _torch()
    _check_input(A)
    N, M = A.shape
    o = make_opts("recurrence", "fp64", "full", True, 0, 0, engine)
    n_uc = counts(N, M, P, Q)["n_uc"]
    R = torch.empty((P * Q, P * Q), dtype=torch.complex128, device=A.device)
    stamps = torch.zeros((n_uc, 2), dtype=torch.int64, device=A.device)
    items = np.zeros((n_uc, 5), dtype=np.int32)
    need = workspace_size(N, M, P, Q, form="recurrence", engine=engine)
    ws, nbytes = _workspace(need, A.device)
    _check(lib().covest_forward_stamped(
        ctypes.c_void_p(A.data_ptr()), N, M, P, Q, ctypes.c_void_p(R.data_ptr()), ctypes.byref(o),
        ctypes.c_void_p(ws.data_ptr() if ws is not None else 0), nbytes, ctypes.c_void_p(stamps.data_ptr()),
        2 * n_uc, items.ctypes.data, _stream_handle(A.device)))
    return R, stamps, items


def lane_plan(N, M, P, Q, row_step=1, n_rows=1, n_cols=1, n_cu=256):
    """Plan of the lane engine for a grid of inputs (covest_lane_plan_get, host only) as a dict."""
    info = covest_lane_plan_info()
    _check(lib().covest_lane_plan_get(N, M, P, Q, row_step, n_rows, n_cols, n_cu, ctypes.byref(info)))
    return {name: getattr(info, name) for name, _ in covest_lane_plan_info._fields_}


def hankel_plan(N, M, P, Q, precision, n_cu=256):
    """(info, items[n,6], tiles[n,4], item_index) of the 16-bit plain-form plan (host only)."""
    import numpy as np
    info = covest_hankel_plan_info()
    prec = PRECS[precision] if isinstance(precision, str) else int(precision)
    _check(lib().covest_hankel_plan_get(N, M, P, Q, prec, n_cu, ctypes.byref(info), None, None, None))
    d = {name: getattr(info, name) for name, _ in covest_hankel_plan_info._fields_}
    items = np.zeros((d["n_items"], 6), dtype=np.int32)
    tiles = np.zeros((d["n_tiles"], 4), dtype=np.int32)
    index = np.zeros(d["n_index"], dtype=np.int32)
    _check(lib().covest_hankel_plan_get(N, M, P, Q, prec, n_cu, ctypes.byref(info), items.ctypes.data,
                                        tiles.ctypes.data, index.ctypes.data))
    return d, items, tiles, index


def engine_choice(N, M, P, Q, batch=False):
    """(engine AUTO picks: "vector" or "matrix", whether the matrix cores can run the shape)."""
    e, f = ctypes.c_int32(0), ctypes.c_int32(0)
    _check(lib().covest_engine_choice(N, M, P, Q, 1 if batch else 0, ctypes.byref(e), ctypes.byref(f)))
    return ("matrix" if e.value == ENGINES["matrix"] else "vector"), bool(f.value)


def mfma_fits(N, M, P, Q) -> bool:
    return engine_choice(N, M, P, Q)[1]


def mfma_preferred(N, M, P, Q, batch=False) -> bool:
    return engine_choice(N, M, P, Q, batch)[0] == "matrix"
