"""Full-matrix parity at the headline size: A 1024 x 1024 (N(0,1) noise plus
one 2-D exponential of amplitude 1e3, seed 3), 32 x 32 window, every entry of
the 1024 x 1024 R of every form against the oracle's R.

The oracle's R comes from its explicit-X route (X X^H / K by BLAS, the pinned
second formulation of eq. 2.2), computed once and kept in the system temp
folder for the session.  Bars (relative Frobenius error over the whole
Hermitian matrix, eq. 2.2 as the reference):
  * FP64 recurrence, both engines: max |R - R_oracle| <= 1e-12 max |diag|;
  * FP32, BF16x3, FP16x3 on the matrix cores: rel-F <= 1e-5;
  * plain FP16: rel-F <= 2^-9, plain BF16: rel-F <= 2^-6 (four unit
    roundoffs of the input format).
The error of the noise component (R - R_oracle over the noise power, since
the exponential's rank-1 part dominates every norm) is printed per form.
"""
import sys

import numpy as np
import pytest

from paper_1303_2285_amd import synth

pytestmark = pytest.mark.gpu

P = Q = 32
TOL = {"fp32": 1e-5, "bf16x3": 1e-5, "fp16x3": 1e-5, "fp16": 2.0 ** -9, "bf16": 2.0 ** -6}


def _note(*a):
    print("[gpu-case]", *a, flush=True)
    sys.stdout.flush()


@pytest.fixture(scope="module")
def torch_dev():
    import torch
    assert torch.cuda.is_available(), "GPU tests need a ROCm device"
    return torch, torch.device("cuda:0")


@pytest.fixture(scope="module")
def cv():
    from paper_1303_2285_amd import covest
    covest.lib()
    return covest


@pytest.fixture(scope="module")
def cfg3(oracle_mod):
    A, p, q = synth.config_input("large")
    assert (p, q) == (P, Q)
    _note("cfg3 oracle R (explicit-X route, cached for the session)")
    R = oracle_mod.forward_blas_cached(A, P, Q)
    noise = float(np.mean(np.abs(synth.wide_range(1024, 1024, seed=3, amp=0.0)) ** 2))
    return A, R, noise


def _relF(a, b):
    return float(np.linalg.norm(a - b) / np.linalg.norm(b))


@pytest.mark.parametrize("engine", ["matrix", "vector"])
def test_cfg3_fp64_recurrence_full(cv, torch_dev, cfg3, engine):
    torch, dev = torch_dev
    A, Rref, noise = cfg3
    _note("cfg3 full matrix, FP64 recurrence", engine)
    R = cv.covest_forward(torch.from_numpy(A).to(dev), P, Q, engine=engine).cpu().numpy()
    scale = np.abs(np.diag(Rref)).max()
    err = np.abs(R - Rref).max()
    _note(f"  max abs err {err / scale:.3e} of max|diag|, rel-F {_relF(R, Rref):.3e}, "
          f"noise-component err {err / noise:.3e} noise powers")
    assert err <= 1e-12 * scale
    assert np.array_equal(R, R.conj().T) and np.all(np.diag(R).imag == 0)


def test_cfg3_fp32_output_full(cv, torch_dev, cfg3):
    """The recurrence with complex64 output: its FP64 sums rounded once."""
    torch, dev = torch_dev
    A, Rref, noise = cfg3
    _note("cfg3 full matrix, FP64 recurrence, complex64 output")
    R = cv.covest_forward(torch.from_numpy(A).to(dev), P, Q, precision="fp32").cpu().numpy()
    assert _relF(R.astype(np.complex128), Rref) <= 2.0 ** -23


@pytest.mark.parametrize("prec", list(TOL))
def test_cfg3_plain_forms_full(cv, torch_dev, cfg3, prec):
    torch, dev = torch_dev
    A, Rref, noise = cfg3
    _note("cfg3 full matrix, plain form", prec)
    R = cv.covest_forward(torch.from_numpy(A).to(dev), P, Q, form="hankel",
                          precision=prec).cpu().numpy().astype(np.complex128)
    err = _relF(R, Rref)
    _note(f"  rel-F {err:.3e}, noise-component max err {np.abs(R - Rref).max() / noise:.3e} noise powers")
    assert err <= TOL[prec], err
    assert np.array_equal(R, R.conj().T)
