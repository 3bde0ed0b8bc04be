"""CPU oracle for the sliding-window estimated covariance matrix.

TEST INFRASTRUCTURE ONLY.  Only ``tests/``, ``__graft_entry__.smoke()`` and the
CPU-baseline leg of ``bench.py`` may import this module.  It shares no code with
the GPU library and never imports it.

Two independent formulations live here:

* ``forward`` / ``entries`` / ``adjoint`` wrap ``covest_oracle.c``: the direct
  definition of eq. 2.2 (Sec. 2.2) as plain FP64 loops, and the adjoint written
  from the definition one window position at a time.
* ``hankel_X`` / ``forward_blas`` / ``adjoint_blas`` build the explicit matrix
  X whose columns are the column-stacked windows V^{p,q} (eq. 2.1) and use
  NumPy's BLAS matrix product: R = X X^H / K and dA = fold(H X) / K.  They are a
  second, separately written route to the same numbers, used to pin the C loops
  and to reach sizes where the loops are too slow.

Readings of the paper used throughout (also listed in the design notes):
K = (N-P+1)(M-Q+1) positions; R = C / K; window index k = i + P*j; entry
(k1, k2) conjugates the second factor; A is row-major with the paper's first
index as the row.
"""
from __future__ import annotations

import ctypes
import os
import subprocess

import numpy as np

HERE = os.path.dirname(os.path.abspath(__file__))
SRC = os.path.join(HERE, "covest_oracle.c")
LIB = os.path.join(HERE, "libcovest_oracle.so")

_lib = None


def build(force: bool = True) -> str:
    """Compile the C oracle with gcc (-O2, no FMA contraction, OpenMP)."""
    if force or not os.path.exists(LIB):
        tmp = LIB + ".tmp"
        cmd = ["gcc", "-O2", "-ffp-contract=off", "-fno-fast-math", "-fopenmp",
               "-shared", "-fPIC", "-std=c99", "-Wall", "-o", tmp, SRC]
        subprocess.run(cmd, check=True)
        os.replace(tmp, LIB)
    return LIB


def _load():
    global _lib
    if _lib is None:
        if not os.path.exists(LIB):
            build(force=False)
        lib = ctypes.CDLL(LIB)
        dp = ctypes.POINTER(ctypes.c_double)
        i64 = ctypes.c_int64
        lib.covest_oracle_fwd.argtypes = [dp, i64, i64, i64, i64, ctypes.c_int, dp, ctypes.c_int]
        lib.covest_oracle_entries.argtypes = [dp, i64, i64, i64, i64, ctypes.c_int,
                                              ctypes.POINTER(i64), ctypes.POINTER(i64), i64,
                                              dp, ctypes.c_int]
        lib.covest_oracle_adj.argtypes = [dp, dp, i64, i64, i64, i64, ctypes.c_int, dp]
        lib.covest_oracle_max_threads.argtypes = []
        for f in (lib.covest_oracle_fwd, lib.covest_oracle_entries, lib.covest_oracle_adj,
                  lib.covest_oracle_max_threads):
            f.restype = ctypes.c_int
        _lib = lib
    return _lib


def _c128(A) -> np.ndarray:
    a = np.ascontiguousarray(np.asarray(A), dtype=np.complex128)
    if a.ndim != 2:
        raise ValueError("A must be 2-D")
    return a


def _ptr(a: np.ndarray):
    return a.ctypes.data_as(ctypes.POINTER(ctypes.c_double))


def _check(rc: int):
    if rc == -2:
        raise ValueError("bad shape: need 1 <= P <= N and 1 <= Q <= M")
    if rc != 0:
        raise RuntimeError(f"oracle returned {rc}")


def max_threads() -> int:
    return int(_load().covest_oracle_max_threads())


def forward(A, P: int, Q: int, normalize: bool = True, threads: int = 1) -> np.ndarray:
    """R (PQ x PQ complex128) by the direct loops of eq. 2.2."""
    a = _c128(A)
    N, M = a.shape
    R = np.empty((P * Q, P * Q), dtype=np.complex128)
    _check(_load().covest_oracle_fwd(_ptr(a), N, M, P, Q, int(bool(normalize)), _ptr(R),
                                     int(threads)))
    return R


def entries(A, P: int, Q: int, k1, k2, normalize: bool = True, threads: int = 1) -> np.ndarray:
    """R[k1[t], k2[t]] for every t, each summed directly over all K positions."""
    a = _c128(A)
    N, M = a.shape
    k1 = np.ascontiguousarray(np.asarray(k1, dtype=np.int64).ravel())
    k2 = np.ascontiguousarray(np.asarray(k2, dtype=np.int64).ravel())
    if k1.shape != k2.shape:
        raise ValueError("k1 and k2 must have the same length")
    out = np.empty(k1.shape[0], dtype=np.complex128)
    p64 = ctypes.POINTER(ctypes.c_int64)
    rc = _load().covest_oracle_entries(_ptr(a), N, M, P, Q, int(bool(normalize)),
                                       k1.ctypes.data_as(p64), k2.ctypes.data_as(p64),
                                       k1.shape[0], _ptr(out), int(threads))
    if rc == -1:
        raise IndexError("entry index out of range")
    _check(rc)
    return out


def adjoint(A, G, P: int, Q: int, normalize: bool = True) -> np.ndarray:
    """dA for a real loss with dL/dR = G (full PQ x PQ), direct definition."""
    a = _c128(A)
    N, M = a.shape
    g = np.ascontiguousarray(np.asarray(G), dtype=np.complex128)
    if g.shape != (P * Q, P * Q):
        raise ValueError("G must be PQ x PQ")
    dA = np.empty_like(a)
    _check(_load().covest_oracle_adj(_ptr(a), _ptr(g), N, M, P, Q, int(bool(normalize)),
                                     _ptr(dA)))
    return dA


# ---------------------------------------------------------------------------
# Explicit-matrix (BLAS) route.
# ---------------------------------------------------------------------------

def hankel_X(A, P: int, Q: int, p0: int = 0, p1: int | None = None) -> np.ndarray:
    """X[:, t] = V^{p,q} for positions with p in [p0, p1), q in [0, M-Q].

    Column t = (p - p0) * Kc + q.  Row k = i + P*j holds A[p+i, q+j] (eq. 2.1).
    """
    a = np.asarray(A, dtype=np.complex128)
    N, M = a.shape
    if not (1 <= P <= N and 1 <= Q <= M):
        raise ValueError("bad shape")
    Kr, Kc = N - P + 1, M - Q + 1
    p1 = Kr if p1 is None else p1
    X = np.empty((P * Q, (p1 - p0) * Kc), dtype=np.complex128)
    for j in range(Q):
        for i in range(P):
            X[i + P * j] = a[p0 + i:p1 + i, j:j + Kc].reshape(-1)
    return X


def _chunk_rows(P: int, Q: int, N: int, M: int, budget: int = 1 << 24) -> int:
    Kc = M - Q + 1
    return max(1, budget // max(1, P * Q * Kc))


def forward_blas(A, P: int, Q: int, normalize: bool = True) -> np.ndarray:
    """R = X X^H / K with X built explicitly, summed over row chunks of positions.

    R is Hermitian by its definition (eq. 2.2: a sum of V V^H), so only its
    upper triangle is accumulated, by BLAS's Hermitian rank-k update (zherk),
    and the lower triangle is its exact conjugate mirror.  zherk is handed
    X^T (Fortran order, no copy) with the conjugate-transpose option, which
    gives conj(X X^H); the conjugate is taken once at the end."""
    from scipy.linalg import blas

    a = np.asarray(A, dtype=np.complex128)
    N, M = a.shape
    Kr, Kc = N - P + 1, M - Q + 1
    PQ = P * Q
    C = np.zeros((PQ, PQ), dtype=np.complex128, order="F")
    step = _chunk_rows(P, Q, N, M)
    for p0 in range(0, Kr, step):
        X = hankel_X(a, P, Q, p0, min(Kr, p0 + step))
        C = blas.zherk(1.0, X.T, beta=1.0, c=C, trans=2, lower=0, overwrite_c=1)
    U = np.triu(np.conj(C))
    R = U + np.triu(U, 1).conj().T
    R[np.diag_indices(PQ)] = U.diagonal().real
    if normalize:
        R /= float(Kr * Kc)
    return np.ascontiguousarray(R)


def forward_blas_cached(A, P: int, Q: int, normalize: bool = True) -> np.ndarray:
    """forward_blas, kept on disk between calls of one session (the headline
    1024 x 1024 / 32 x 32 case costs ~10^12 complex multiply-adds): a file in
    the system temp folder keyed by a hash of A's bytes, P, Q, normalize and
    this module's source.  Never in the repository."""
    import hashlib
    import tempfile

    a = np.ascontiguousarray(np.asarray(A))
    h = hashlib.sha256()
    h.update(a.dtype.str.encode())
    h.update(repr(a.shape).encode())
    h.update(a.tobytes())
    h.update(f"{P},{Q},{int(bool(normalize))}".encode())
    with open(os.path.abspath(__file__), "rb") as f:
        h.update(f.read())
    folder = os.path.join(tempfile.gettempdir(), "covest_oracle_cache")
    path = os.path.join(folder, h.hexdigest()[:24] + ".npy")
    if os.path.exists(path):
        try:
            return np.load(path, allow_pickle=False)
        except (OSError, ValueError):
            pass
    R = forward_blas(a, P, Q, normalize)
    os.makedirs(folder, exist_ok=True)
    tmp = f"{path}.{os.getpid()}.tmp.npy"
    np.save(tmp, R, allow_pickle=False)
    os.replace(tmp, path)
    return R


def adjoint_blas(A, G, P: int, Q: int, normalize: bool = True) -> np.ndarray:
    """dA = fold(H X) / K with H = G + G^H; fold adds row k = i + P*j of the
    product back onto A[p+i, q+j] for every position (p, q)."""
    a = np.asarray(A, dtype=np.complex128)
    N, M = a.shape
    Kr, Kc = N - P + 1, M - Q + 1
    g = np.asarray(G, dtype=np.complex128)
    H = g + g.conj().T
    dA = np.zeros((N, M), dtype=np.complex128)
    step = _chunk_rows(P, Q, N, M)
    for p0 in range(0, Kr, step):
        p1 = min(Kr, p0 + step)
        U = (H @ hankel_X(a, P, Q, p0, p1)).reshape(P * Q, p1 - p0, Kc)
        for j in range(Q):
            for i in range(P):
                dA[p0 + i:p1 + i, j:j + Kc] += U[i + P * j]
    if normalize:
        dA /= float(Kr * Kc)
    return dA


def capon(R, P: int, Q: int, F1: int, F2: int) -> np.ndarray:
    """Minimum-variance (Capon) spectrum of one R (Sec. 2.3 names the MVM /
    Capon estimator as the consumer of R): S[f1][f2] = 1 / Re(a^H R^{-1} a)
    with a[i + P*j] = exp(1j (w1 i + w2 j)) (the window index map of eq. 2.1)
    on the grid w = -pi + 2 pi f / F.  Written from the definition: every grid
    vector a is formed, R^{-1} a comes from LAPACK's linear solve, then the
    quadratic form."""
    R = np.asarray(R, dtype=np.complex128)
    PQ = P * Q
    w1 = -np.pi + 2 * np.pi * np.arange(F1) / F1
    w2 = -np.pi + 2 * np.pi * np.arange(F2) / F2
    k = np.arange(PQ)
    i, j = k % P, k // P
    phase = i[:, None, None] * w1[None, :, None] + j[:, None, None] * w2[None, None, :]
    a = np.exp(1j * phase).reshape(PQ, F1 * F2)
    x = np.linalg.solve(R, a)
    q = np.sum(a.conj() * x, axis=0).real
    return (1.0 / q).reshape(F1, F2)

