"""Seeded synthetic inputs for the sliding-window covariance workloads.

This module only draws numbers.  It holds none of the covariance method's
arithmetic, so both the CPU oracle tests and the GPU path can take their inputs
from here without sharing any computation.

Every generator draws in float64 with ``numpy.random.default_rng(seed)``
(PCG64) and casts once to complex64; those complex64 values are the inputs to
both sides.  Indices n (row) and m (column) are 0-based.

Workloads (the paper's problem statement, Sec. 2.2: an N x M complex input and a
P x Q sliding window):

* ``gaussian``      re, im i.i.d. N(0, 1)                     (64x64, P=Q=8)
* ``small_int``     re, im uniform on the integers -8..8     (exact FP64 sums)
* ``exponentials``  3 unit-amplitude 2-D complex exponentials plus complex
                    Gaussian noise at 10 dB SNR per exponential (256x256, 16x16)
* ``wide_range``    N(0,1) noise plus one exponential of amplitude 1e3
                    (1024x1024, 32x32)
* ``batch``         512 Gaussian inputs, N, M uniform in [64, 512], P, Q drawn
                    from {4, 8, 12, 16}
* ``adjoint``       512x512 Gaussian A, a random Hermitian W and the R of an
                    independent input (loss of the differentiation workload)
* ``aperture_image`` one large image of 2-D exponentials plus noise, cut into
                    a grid of overlapping apertures (the many-matrix imaging
                    workload of Sec. 2.3: a 1600x1600 image, 25x25 apertures of
                    100x100, a 10x10 window)

The 2-D exponentials stand in for the spectral-estimation signals the paper
cites (Sec. 2.3); no SAR data or benchmark suite is involved.
"""
from __future__ import annotations

import numpy as np

__all__ = [
    "gaussian", "small_int", "exponentials", "wide_range", "batch_shapes",
    "batch", "adjoint_inputs", "hermitian", "aperture_image", "CONFIGS", "APERTURE_GRIDS",
]


def _rng(seed: int) -> np.random.Generator:
    return np.random.default_rng(int(seed))


def gaussian(N: int, M: int, seed: int) -> np.ndarray:
    """complex64 N x M, real and imaginary parts i.i.d. N(0, 1)."""
    g = _rng(seed)
    re = g.standard_normal((N, M))
    im = g.standard_normal((N, M))
    return (re + 1j * im).astype(np.complex64)


def small_int(N: int, M: int, seed: int, lo: int = -8, hi: int = 8) -> np.ndarray:
    """complex64 N x M whose parts are integers uniform on [lo, hi]."""
    g = _rng(seed)
    re = g.integers(lo, hi + 1, size=(N, M))
    im = g.integers(lo, hi + 1, size=(N, M))
    return (re + 1j * im).astype(np.complex64)


def _exp2d(N, M, w1, w2, phi):
    n = np.arange(N, dtype=np.float64)[:, None]
    m = np.arange(M, dtype=np.float64)[None, :]
    return np.exp(1j * (w1 * n + w2 * m + phi))


def exponentials(N: int, M: int, seed: int, n_exp: int = 3,
                 noise_var: float = 0.1) -> np.ndarray:
    """Sum of unit-amplitude 2-D complex exponentials plus complex noise.

    Frequencies are uniform on [-pi, pi)^2 and phases uniform on [0, 2 pi).
    ``noise_var`` is the total complex noise variance (0.1 = 10 dB below one
    unit-amplitude exponential), split equally between the two parts.
    """
    g = _rng(seed)
    w = g.uniform(-np.pi, np.pi, size=(n_exp, 2))
    phi = g.uniform(0.0, 2 * np.pi, size=n_exp)
    a = np.zeros((N, M), dtype=np.complex128)
    for t in range(n_exp):
        a += _exp2d(N, M, w[t, 0], w[t, 1], phi[t])
    s = np.sqrt(noise_var / 2.0)
    a += s * g.standard_normal((N, M)) + 1j * s * g.standard_normal((N, M))
    return a.astype(np.complex64)


def exponential_params(seed: int, n_exp: int = 3):
    """The (w1, w2, phi) triples ``exponentials`` draws for ``seed``."""
    g = _rng(seed)
    w = g.uniform(-np.pi, np.pi, size=(n_exp, 2))
    phi = g.uniform(0.0, 2 * np.pi, size=n_exp)
    return w, phi


def wide_range(N: int, M: int, seed: int, amp: float = 1e3) -> np.ndarray:
    """N(0,1) complex noise plus one 2-D exponential of amplitude ``amp``."""
    g = _rng(seed)
    re = g.standard_normal((N, M))
    im = g.standard_normal((N, M))
    w1, w2 = g.uniform(-np.pi, np.pi, size=2)
    phi = g.uniform(0.0, 2 * np.pi)
    a = (re + 1j * im) + amp * _exp2d(N, M, w1, w2, phi)
    return a.astype(np.complex64)


def hermitian(n: int, seed: int) -> np.ndarray:
    """complex128 (B + B^H)/2 with B complex Gaussian n x n."""
    g = _rng(seed)
    b = g.standard_normal((n, n)) + 1j * g.standard_normal((n, n))
    return (b + b.conj().T) / 2.0


def batch_shapes(count: int = 512, seed: int = 4, nm_lo: int = 64,
                 nm_hi: int = 512, windows=(4, 8, 12, 16)):
    """Draw (N, M, P, Q) for every instance first, from one generator stream."""
    g = _rng(seed)
    N = g.integers(nm_lo, nm_hi + 1, size=count)
    M = g.integers(nm_lo, nm_hi + 1, size=count)
    P = g.choice(np.asarray(windows), size=count)
    Q = g.choice(np.asarray(windows), size=count)
    P = np.minimum(P, N)
    Q = np.minimum(Q, M)
    return g, [(int(N[i]), int(M[i]), int(P[i]), int(Q[i])) for i in range(count)]


def batch(count: int = 512, seed: int = 4, **kw):
    """Shapes first, then every instance's Gaussian data from the same stream."""
    g, shapes = batch_shapes(count, seed, **kw)
    out = []
    for (N, M, P, Q) in shapes:
        re = g.standard_normal((N, M))
        im = g.standard_normal((N, M))
        out.append(((re + 1j * im).astype(np.complex64), P, Q))
    return out


def adjoint_inputs(N: int = 512, M: int = 512, P: int = 16, Q: int = 16,
                   seed_a: int = 5, seed_w: int = 56, seed_t: int = 55):
    """A, the Hermitian weight W (PQ x PQ) and the independent input A_t."""
    A = gaussian(N, M, seed_a)
    W = hermitian(P * Q, seed_w)
    At = gaussian(N, M, seed_t)
    return A, W, At


def aperture_image(H: int, W: int, seed: int, n_exp: int = 8, noise_var: float = 0.1) -> np.ndarray:
    """An H x W image for the aperture workload: ``n_exp`` unit-amplitude 2-D
    exponentials (point scatterers seen in the frequency domain) plus complex
    noise 10 dB below one of them.  A synthetic stand-in for imaging data."""
    return exponentials(H, W, seed, n_exp, noise_var)


# name -> (H, W, ap_rows, ap_cols, row_step, col_step, n_rows, n_cols, P, Q, seed):
# aperture (a, b) is image[a*row_step : a*row_step + ap_rows, b*col_step : ...]
APERTURE_GRIDS = {
    "sar_1600": (1600, 1600, 100, 100, 62, 62, 25, 25, 10, 10, 6),
}


# name -> (N, M, P, Q, generator, seed)
CONFIGS = {
    "small": (64, 64, 8, 8, gaussian, 1),
    "small_int": (64, 64, 8, 8, small_int, 101),
    "medium": (256, 256, 16, 16, exponentials, 2),
    "large": (1024, 1024, 32, 32, wide_range, 3),
    "adjoint": (512, 512, 16, 16, gaussian, 5),
}


def config_input(name: str) -> tuple[np.ndarray, int, int]:
    N, M, P, Q, fn, seed = CONFIGS[name]
    return fn(N, M, seed), P, Q
