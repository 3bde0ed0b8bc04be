"""GPU parity of the plain form (R = X X^H / K on the matrix cores) against the
CPU oracle.

Bars: relative Frobenius error <= 1e-5 for FP32, BF16x3 and FP16x3; the stated
figures 2^-9 (FP16) and 2^-6 (BF16) for the plain 16-bit forms (first-order
bounds of four unit roundoffs on the input rounding).  On small-integer inputs
every product and every FP32 partial sum is an exact integer below 2^24, so all
forms are bit-exact there.
"""
import sys

import numpy as np
import pytest

from paper_1303_2285_amd import synth

pytestmark = pytest.mark.gpu

TOL = {"fp32": 1e-5, "bf16x3": 1e-5, "fp16x3": 1e-5, "fp16": 2.0 ** -9, "bf16": 2.0 ** -6}
PRECS = list(TOL)


def _note(*a):
    print("[gpu-case]", *a, flush=True)
    sys.stdout.flush()


@pytest.fixture(scope="module")
def torch_dev():
    import torch
    assert torch.cuda.is_available()
    return torch, torch.device("cuda:0")


@pytest.fixture(scope="module")
def cv():
    from paper_1303_2285_amd import covest
    covest.lib()
    return covest


def hankel(cv, torch_dev, A, P, Q, precision, **kw):
    torch, dev = torch_dev
    At = torch.from_numpy(np.ascontiguousarray(A)).to(dev)
    R = cv.covest_forward(At, P, Q, form="hankel", precision=precision, **kw)
    torch.cuda.synchronize()
    return R.cpu().numpy()


def relF(a, b):
    return np.linalg.norm(a - b) / np.linalg.norm(b)


@pytest.mark.parametrize("prec", PRECS)
def test_small_gaussian(cv, torch_dev, oracle_mod, prec):
    A, P, Q = synth.config_input("small")
    _note("hankel small", prec)
    R = hankel(cv, torch_dev, A, P, Q, prec)
    assert R.dtype == np.complex64
    ref = oracle_mod.forward(A, P, Q)
    err = relF(R.astype(np.complex128), ref)
    assert err <= TOL[prec], err
    assert np.array_equal(R, R.conj().T)
    assert np.all(np.diag(R).imag == 0)


@pytest.mark.parametrize("prec", PRECS)
def test_small_integer_exact(cv, torch_dev, oracle_mod, prec):
    A, P, Q = synth.config_input("small_int")
    _note("hankel small_int", prec)
    C = hankel(cv, torch_dev, A, P, Q, prec, normalize=False)
    ref = oracle_mod.forward(A, P, Q, normalize=False)
    assert np.array_equal(C.astype(np.complex128), ref)


def test_medium_fp32(cv, torch_dev, oracle_mod):
    A, P, Q = synth.config_input("medium")
    _note("hankel medium fp32")
    R = hankel(cv, torch_dev, A, P, Q, "fp32")
    ref = oracle_mod.forward(A, P, Q, threads=oracle_mod.max_threads())
    assert relF(R.astype(np.complex128), ref) <= 1e-5


@pytest.mark.parametrize("prec", PRECS)
def test_large_sampled(cv, torch_dev, oracle_mod, prec):
    """1024 x 1024, 32 x 32 window: relative error over a sample of entries
    (all diagonal entries plus random ones) against the oracle's direct sums."""
    A, P, Q = synth.config_input("large")
    _note("hankel large", prec)
    R = hankel(cv, torch_dev, A, P, Q, prec)
    PQ = P * Q
    rng = np.random.default_rng(5)
    k1 = np.concatenate([np.arange(0, PQ, 8), rng.integers(0, PQ, 400)])
    k2 = np.concatenate([np.arange(0, PQ, 8), rng.integers(0, PQ, 400)])
    ref = oracle_mod.entries(A, P, Q, k1, k2, threads=oracle_mod.max_threads())
    got = R[k1, k2].astype(np.complex128)
    err = np.linalg.norm(got - ref) / np.linalg.norm(ref)
    assert err <= TOL[prec], err


EDGE = [(5, 7, 5, 7), (9, 4, 3, 4), (33, 17, 1, 16), (17, 33, 16, 1), (40, 33, 4, 16),
        (97, 131, 12, 4), (131, 97, 5, 13), (64, 64, 32, 32), (70, 66, 33, 2), (100, 90, 9, 11),
        (1, 1, 1, 1), (30, 200, 24, 24)]


@pytest.mark.parametrize("shape", EDGE, ids=lambda s: "x".join(map(str, s)))
def test_edge_integer_exact(cv, torch_dev, oracle_mod, shape):
    N, M, P, Q = shape
    A = synth.small_int(N, M, seed=N * 7 + M * 3 + P)
    _note("hankel edge", shape)
    for prec in PRECS:
        C = hankel(cv, torch_dev, A, P, Q, prec, normalize=False)
        ref = oracle_mod.forward(A, P, Q, normalize=False)
        assert np.array_equal(C.astype(np.complex128), ref), prec


@pytest.mark.parametrize("prec", PRECS)
def test_fill_upper(cv, torch_dev, oracle_mod, prec):
    torch, dev = torch_dev
    A = synth.small_int(40, 44, seed=12)
    P, Q = 5, 6
    out = torch.full((P * Q, P * Q), complex(3.0, 4.0), dtype=torch.complex64, device=dev)
    _note("hankel fill upper", prec)
    cv.covest_forward(torch.from_numpy(A).to(dev), P, Q, form="hankel", precision=prec,
                      fill="upper", normalize=False, out=out)
    torch.cuda.synchronize()
    R = out.cpu().numpy().astype(np.complex128)
    ref = oracle_mod.forward(A, P, Q, normalize=False)
    iu = np.triu_indices(P * Q)
    il = np.tril_indices(P * Q, -1)
    assert np.array_equal(R[iu], ref[iu])
    assert np.all(R[il] == complex(3.0, 4.0))


@pytest.mark.parametrize("prec", ["bf16", "bf16x3", "fp16", "fp16x3"])
def test_long_rows_integer_exact(cv, torch_dev, oracle_mod, prec):
    """Rows of more positions than one item sums (16384 for the split forms,
    32768 for the plain ones): items split along the row; integer input, exact."""
    A = synth.small_int(6, 33000, seed=31)
    P, Q = 3, 5
    _note("hankel long rows", prec)
    C = hankel(cv, torch_dev, A, P, Q, prec, normalize=False)
    ref = oracle_mod.forward(A, P, Q, normalize=False, threads=oracle_mod.max_threads())
    assert np.array_equal(C.astype(np.complex128), ref)


@pytest.mark.parametrize("prec", ["bf16", "bf16x3", "fp16", "fp16x3"])
def test_strided_input(cv, torch_dev, oracle_mod, prec):
    """A strided view of A (lda > M) through the split pass."""
    torch, dev = torch_dev
    full = synth.small_int(90, 120, seed=32)
    P, Q = 7, 9
    _note("hankel strided", prec)
    At = torch.from_numpy(full).to(dev)[:, 5:105]
    C = cv.covest_forward(At, P, Q, form="hankel", precision=prec, normalize=False)
    torch.cuda.synchronize()
    ref = oracle_mod.forward(full[:, 5:105], P, Q, normalize=False)
    assert np.array_equal(C.cpu().numpy().astype(np.complex128), ref)


def test_fp64_not_offered(cv, torch_dev):
    torch, dev = torch_dev
    A = torch.zeros((16, 16), dtype=torch.complex64, device=dev)
    with pytest.raises(cv.CovestError) as e:
        cv.covest_forward(A, 4, 4, form="hankel", precision="fp64")
    assert e.value.status == cv.ERR_UNSUPPORTED
