"""Minimum-variance (Capon) spectrum of R: the oracle pinned to closed forms
(CPU), the GPU kernel against the oracle (GPU).

S(w1, w2) = 1 / Re(a^H R^{-1} a), a[i + P*j] = exp(i (w1 i + w2 j)), on the
grid w = -pi + 2 pi f / F.  Tolerance of the GPU parity: both sides solve in
FP64 (the GPU through a Cholesky factor and the lag sums of R^{-1}, the oracle
through LAPACK's solve per grid vector); their difference is bounded by about
cond(R) * PQ * 2^-53 relative, below 1e-11 for the condition numbers here
(R = B B^H / n + I has cond < 1e3), so 1e-10 is asserted.
"""
import ctypes
import sys

import numpy as np
import pytest

from paper_1303_2285_amd import synth

TOL = 1e-10


def _note(*a):
    print("[gpu-case]", *a, flush=True)
    sys.stdout.flush()


def grid(F):
    return -np.pi + 2 * np.pi * np.arange(F) / F


def dirichlet(n, dw):
    """|sum_{t<n} exp(i dw t)|^2 by direct summation."""
    t = np.arange(n)
    return np.abs(np.exp(1j * np.multiply.outer(dw, t)).sum(axis=-1)) ** 2


def hpd(n, seed):
    g = np.random.default_rng(seed)
    B = g.standard_normal((n, n)) + 1j * g.standard_normal((n, n))
    return B @ B.conj().T / n + np.eye(n)


# ------------------------------------------------------------------ oracle --

def test_oracle_white_noise(oracle_mod):
    for (P, Q) in [(1, 1), (3, 4), (8, 8)]:
        S = oracle_mod.capon(2.5 * np.eye(P * Q), P, Q, 16, 12)
        assert np.allclose(S, 2.5 / (P * Q), rtol=1e-14, atol=0)


def test_oracle_rank_one_plus_noise(oracle_mod):
    """R = s2 I + p a0 a0^H: by Sherman-Morrison
    a^H R^{-1} a = (PQ - p |a^H a0|^2 / (s2 + p PQ)) / s2, with |a^H a0|^2 the
    product of two Dirichlet kernels."""
    P, Q, F1, F2 = 5, 7, 32, 24
    s2, p = 0.3, 4.0
    w01, w02 = 0.7, -1.9
    k = np.arange(P * Q)
    a0 = np.exp(1j * (w01 * (k % P) + w02 * (k // P)))
    R = s2 * np.eye(P * Q) + p * np.outer(a0, a0.conj())
    g1, g2 = grid(F1), grid(F2)
    overlap = dirichlet(P, g1 - w01)[:, None] * dirichlet(Q, g2 - w02)[None, :]
    want = s2 / (P * Q - p * overlap / (s2 + p * P * Q))
    assert np.allclose(oracle_mod.capon(R, P, Q, F1, F2), want, rtol=1e-12, atol=0)


def peak_checks(S, freqs, F1, F2):
    """Each generated frequency sits on a peak: S at its nearest grid point is
    a local maximum (3 x 3, circular) and exceeds the median of S tenfold."""
    med = np.median(S)
    for (w1, w2) in freqs:
        f1 = int(np.round((w1 + np.pi) * F1 / (2 * np.pi))) % F1
        f2 = int(np.round((w2 + np.pi) * F2 / (2 * np.pi))) % F2
        nb = S[np.ix_([(f1 - 1) % F1, f1, (f1 + 1) % F1], [(f2 - 1) % F2, f2, (f2 + 1) % F2])]
        assert S[f1, f2] == nb.max(), (w1, w2)
        assert S[f1, f2] > 10 * med, (w1, w2, S[f1, f2], med)


def test_oracle_peaks_at_generated_frequencies(oracle_mod):
    """Two exponentials 10 dB above the noise: the spectrum of the oracle's R
    peaks at their frequencies."""
    n_exp, seed = 2, 12
    A = synth.exponentials(96, 96, seed, n_exp=n_exp)
    w, _ = synth.exponential_params(seed, n_exp)
    R = oracle_mod.forward(A, 8, 8, threads=oracle_mod.max_threads())
    peak_checks(oracle_mod.capon(R, 8, 8, 64, 64), w, 64, 64)


def test_capon_argument_errors_before_device_use():
    from paper_1303_2285_amd import covest as cv
    L = cv.lib()
    n = ctypes.c_size_t(0)
    assert L.covest_capon_workspace_size(4, 17, 16, 64, ctypes.byref(n)) == cv.ERR_UNSUPPORTED
    assert L.covest_capon_workspace_size(1, 16, 16, 64, ctypes.byref(n)) == cv.OK
    assert n.value == 16 * (64 * 31 + 256 * 257 // 2)   # the factor in the workspace above PQ = 128
    assert L.covest_capon_workspace_size(4, 10, 10, 0, ctypes.byref(n)) == cv.ERR_SHAPE
    assert L.covest_capon_workspace_size(4, 10, 10, 64, None) == cv.ERR_INVALID_ARG
    assert L.covest_capon_workspace_size(4, 10, 10, 64, ctypes.byref(n)) == cv.OK
    need = n.value
    assert need == 4 * 16 * 64 * 19
    fake = ctypes.c_void_p(256)
    assert L.covest_capon_spectrum(fake, 4, 10, 10, 64, 64, fake, fake, need - 1, None) == cv.ERR_WORKSPACE
    assert L.covest_capon_spectrum(None, 4, 10, 10, 64, 64, fake, fake, need, None) == cv.ERR_INVALID_ARG
    assert L.covest_capon_spectrum(fake, 4, 10, 10, 64, 5000, fake, fake, need, None) == cv.ERR_SHAPE
    assert L.covest_capon_spectrum(fake, 4, 16, 17, 64, 64, fake, fake, need, None) == cv.ERR_UNSUPPORTED
    assert L.covest_capon_spectrum(fake, 4, 16, 16, 64, 64, fake, fake, need, None) == cv.ERR_WORKSPACE
    assert L.covest_capon_spectrum(None, 0, 10, 10, 64, 64, None, None, 0, None) == cv.OK


# -------------------------------------------------------------------- GPU --

@pytest.fixture(scope="module")
def tdev():
    import torch
    assert torch.cuda.is_available(), "GPU tests need a ROCm device"
    return torch, torch.device("cuda:0")


@pytest.fixture(scope="module")
def cv():
    from paper_1303_2285_amd import covest
    covest.lib()
    return covest


@pytest.mark.gpu
@pytest.mark.parametrize("shape", [(1, 1, 8, 8), (3, 4, 16, 12), (8, 8, 64, 64), (10, 10, 64, 48),
                                   (16, 8, 32, 32), (11, 11, 40, 40), (2, 64, 16, 64), (7, 1, 33, 1),
                                   (12, 11, 24, 24), (16, 16, 32, 32), (4, 64, 8, 32)],
                         ids=lambda s: "x".join(map(str, s)))
def test_gpu_random_hpd(cv, tdev, oracle_mod, shape):
    torch, dev = tdev
    P, Q, F1, F2 = shape
    Rs = np.stack([hpd(P * Q, seed=100 * P + Q + c) for c in range(3)])
    _note("capon random HPD", shape)
    S = cv.covest_capon_spectrum(torch.from_numpy(Rs).to(dev), P, Q, F1, F2).cpu().numpy()
    assert S.shape == (3, F1, F2)
    for c in range(3):
        ref = oracle_mod.capon(Rs[c], P, Q, F1, F2)
        assert np.max(np.abs(S[c] - ref) / np.abs(ref)) <= TOL, (shape, c)


@pytest.mark.gpu
def test_gpu_not_positive_definite_gives_nan(cv, tdev):
    torch, dev = tdev
    Rs = np.stack([hpd(16, seed=5), -np.eye(16), hpd(16, seed=6)])
    _note("capon NaN for a non-PD matrix")
    S = cv.covest_capon_spectrum(torch.from_numpy(Rs).to(dev), 4, 4, 8, 8).cpu().numpy()
    assert np.all(np.isnan(S[1]))
    assert np.all(np.isfinite(S[0])) and np.all(np.isfinite(S[2]))


@pytest.mark.gpu
def test_gpu_aperture_pipeline(cv, tdev, oracle_mod):
    """Image -> R of every aperture (GPU) -> spectrum of each (GPU), against the
    oracle's R of the aperture -> the oracle's spectrum; and every aperture's
    spectrum peaks at the image's generated frequencies."""
    torch, dev = tdev
    n_exp, seed = 2, 12
    img = synth.exponentials(240, 240, seed, n_exp=n_exp)
    w, _ = synth.exponential_params(seed, n_exp)
    ap, step, n, P, Q, F = (100, 100), (70, 70), (3, 3), 10, 10, 64
    _note("capon aperture pipeline 240x240, 3x3 apertures of 100x100, 10x10 window")
    plan = cv.AperturePlan(torch.from_numpy(img).to(dev), ap[0], ap[1], step[0], step[1], n[0], n[1], P, Q)
    R = plan.run()
    S = cv.covest_capon_spectrum(R, P, Q, F, F).cpu().numpy()
    plan.close()
    assert S.shape == (3, 3, F, F)
    for a in range(n[0]):
        for b in range(n[1]):
            sub = np.ascontiguousarray(img[a * step[0]:a * step[0] + ap[0], b * step[1]:b * step[1] + ap[1]])
            ref = oracle_mod.capon(oracle_mod.forward(sub, P, Q, threads=oracle_mod.max_threads()), P, Q, F, F)
            assert np.max(np.abs(S[a, b] - ref) / np.abs(ref)) <= 1e-9, (a, b)
            peak_checks(S[a, b], w, F, F)


@pytest.mark.gpu
def test_gpu_three_exponentials_16x16(cv, tdev):
    """The 256 x 256 input of three exponentials 10 dB above the noise with a
    16 x 16 window (PQ = 256, the factor in the workspace): R on the GPU, its
    spectrum on the GPU, peaks at the three generated frequencies."""
    torch, dev = tdev
    A, P, Q = synth.config_input("medium")
    w, _ = synth.exponential_params(2, 3)
    _note("capon 256x256 three exponentials, 16x16 window")
    R = cv.covest_forward(torch.from_numpy(A).to(dev), P, Q)
    S = cv.covest_capon_spectrum(R, P, Q, 128, 128).cpu().numpy()
    peak_checks(S, w, 128, 128)



@pytest.mark.gpu
@pytest.mark.parametrize("P,Q", [(10, 10), (16, 16)])
def test_gpu_upper_fill_input(cv, tdev, oracle_mod, P, Q):
    """R from the forward with fill='upper' (the lower triangle left as the
    caller's zeros) gives the same spectrum as the full R: the kernel reads
    only the upper triangle."""
    torch, dev = tdev
    img = synth.exponentials(120, 110, 21, n_exp=2)
    _note("capon of an upper-fill R", P, Q)
    At = torch.from_numpy(img).to(dev)
    Ru = cv.covest_forward(At, P, Q, fill="upper")
    Rf = cv.covest_forward(At, P, Q, fill="full")
    assert torch.count_nonzero(torch.tril(Ru, -1)).item() == 0
    Su = cv.covest_capon_spectrum(Ru, P, Q, 48, 40).cpu().numpy()
    Sf = cv.covest_capon_spectrum(Rf, P, Q, 48, 40).cpu().numpy()
    assert np.array_equal(Su, Sf)
    ref = oracle_mod.capon(oracle_mod.forward(img, P, Q, threads=oracle_mod.max_threads()), P, Q, 48, 40)
    assert np.max(np.abs(Su - ref) / np.abs(ref)) <= 1e-9
