"""Batched forward (one persistent launch captured in a HIP graph) and the
recurrence's tile-shape choices, on the GPU, against the CPU oracle.

The batch workload: 512 Gaussian inputs, N and M uniform in [64, 512], P and Q
drawn from {4, 8, 12, 16} (seed 4).  Checks: every instance's sampled entries
against the oracle's direct sums (FP64 bar 1e-12), full oracle comparison on
the smallest instances, bit-exactness on a small-integer batch, identical
results over repeated graph replays with eager work in between, and the
FILL_UPPER / complex64 variants.
"""
import sys

import numpy as np
import pytest

from paper_1303_2285_amd import synth

pytestmark = pytest.mark.gpu


def _note(*a):
    print("[gpu-case]", *a, flush=True)
    sys.stdout.flush()


@pytest.fixture(scope="module")
def tdev():
    import torch
    assert torch.cuda.is_available()
    return torch, torch.device("cuda:0")


@pytest.fixture(scope="module")
def cv():
    from paper_1303_2285_amd import covest
    covest.lib()
    return covest


def int_batch(n, seed):
    rng = np.random.default_rng(seed)
    out = []
    for i in range(n):
        P = int(rng.choice([4, 8, 12, 16]))
        Q = int(rng.choice([4, 8, 12, 16]))
        N = int(rng.integers(P, 120))
        M = int(rng.integers(Q, 120))
        out.append((synth.small_int(N, M, seed=seed * 1000 + i), P, Q))
    return out


def test_integer_batch_bit_exact(cv, tdev, oracle_mod):
    torch, dev = tdev
    batch = int_batch(40, 7)
    _note("batched integer x40")
    plan = cv.BatchedPlan([(torch.from_numpy(A).to(dev), P, Q) for (A, P, Q) in batch])
    outs = plan.run()
    torch.cuda.synchronize()
    for (A, P, Q), R in zip(batch, outs):
        ref = oracle_mod.forward(A, P, Q)
        got = R.cpu().numpy()
        assert np.array_equal(got.real, ref.real) and np.array_equal(got.imag, ref.imag), (A.shape, P, Q)
    plan.close()


@pytest.mark.parametrize("workers", [1, 3])
def test_worker_cap_bit_exact(cv, tdev, oracle_mod, monkeypatch, workers):
    """COVEST_WORKERS caps the persistent kernel's workgroups (the worker
    study); every job still runs, so every result is still the oracle's."""
    torch, dev = tdev
    batch = int_batch(12, 11) + [(synth.small_int(32, 32, seed=1300), 13, 13),
                                 (synth.small_int(20, 20, seed=1301), 8, 8)]
    monkeypatch.setenv("COVEST_WORKERS", str(workers))
    _note("batched integer x14, workers", workers)
    plan = cv.BatchedPlan([(torch.from_numpy(A).to(dev), P, Q) for (A, P, Q) in batch], engine="vector")
    outs = plan.run()
    torch.cuda.synchronize()
    for (A, P, Q), R in zip(batch, outs):
        ref = oracle_mod.forward(A, P, Q)
        got = R.cpu().numpy()
        assert np.array_equal(got.real, ref.real) and np.array_equal(got.imag, ref.imag), (A.shape, P, Q)
    plan.close()


def test_workload_batch(cv, tdev, oracle_mod):
    torch, dev = tdev
    batch = synth.batch(512, seed=4)
    _note("batched workload x512")
    As = [torch.from_numpy(A).to(dev) for (A, P, Q) in batch]
    plan = cv.BatchedPlan([(At, P, Q) for At, (A, P, Q) in zip(As, batch)])
    first = [R.clone() for R in plan.run()]
    torch.cuda.synchronize()
    # eager work and a synchronisation between replays, then replay twice more
    junk = torch.randn(1 << 20, device=dev).cumsum(0)
    torch.cuda.synchronize()
    for _ in range(2):
        outs = plan.run()
        torch.cuda.synchronize()
        for R0, R in zip(first, outs):
            assert torch.equal(R0, R)
    del junk
    thr = oracle_mod.max_threads()
    rng = np.random.default_rng(11)
    order = np.argsort([A.shape[0] * A.shape[1] * P * Q for (A, P, Q) in batch])
    smallest = set(order[:12].tolist())
    worst = 0.0
    for i, ((A, P, Q), R) in enumerate(zip(batch, first)):
        got = R.cpu().numpy()
        if i in smallest:
            ref = oracle_mod.forward(A, P, Q, threads=thr)
            err = np.linalg.norm(got - ref) / np.linalg.norm(ref)
        else:
            PQ = P * Q
            k1 = np.concatenate([rng.integers(0, PQ, 10), [0, PQ - 1]])
            k2 = np.concatenate([rng.integers(0, PQ, 10), [PQ - 1, PQ - 1]])
            ref = oracle_mod.entries(A, P, Q, k1, k2, threads=thr)
            err = np.abs(got[k1, k2] - ref).max() / np.abs(np.diag(got)).max()
        worst = max(worst, err)
        assert err <= 1e-12, (i, A.shape, P, Q, err)
    # the batched result equals the single-problem path up to summation order
    for i in order[-3:]:
        A, P, Q = batch[i]
        R1 = cv.covest_forward(As[i], P, Q).cpu().numpy()
        Rb = first[i].cpu().numpy()
        assert np.linalg.norm(R1 - Rb) / np.linalg.norm(R1) <= 1e-13
    plan.close()


def test_batch_fp32_upper(cv, tdev, oracle_mod):
    torch, dev = tdev
    batch = int_batch(12, 9)
    _note("batched fp32 upper")
    plan = cv.BatchedPlan([(torch.from_numpy(A).to(dev), P, Q) for (A, P, Q) in batch],
                          precision="fp32", fill="upper", normalize=False)
    outs = plan.run()
    torch.cuda.synchronize()
    for (A, P, Q), R in zip(batch, outs):
        assert R.dtype == torch.complex64
        ref = oracle_mod.forward(A, P, Q, normalize=False)
        got = R.cpu().numpy().astype(np.complex128)
        iu = np.triu_indices(P * Q)
        il = np.tril_indices(P * Q, -1)
        assert np.array_equal(got[iu], ref[iu])        # integers below 2^24: exact in float
        assert np.all(got[il] == 0)
    plan.close()


def fit_int_batch(n, seed):
    """Small-integer problems, most of which fit the matrix-core engine."""
    rng = np.random.default_rng(seed)
    out = []
    for i in range(n):
        P = int(rng.choice([8, 12, 16, 24]))
        Q = int(rng.choice([8, 12, 16, 32]))
        N = int(rng.integers(2 * P - 1, 2 * P + 150))
        M = int(rng.integers(2 * Q - 1, 2 * Q + 150))
        out.append((synth.small_int(N, M, seed=seed * 1000 + i), P, Q))
    return out


@pytest.mark.parametrize("engine", ["auto", "vector"])
def test_batch_engines_bit_exact(cv, tdev, oracle_mod, engine):
    """Mixed batches: with engine auto the problems that fit go to the
    matrix-core kernel (one launch per lag-block shape), the rest to the
    vector kernel; every result is the oracle's, bit for bit."""
    torch, dev = tdev
    batch = fit_int_batch(36, 21)
    _note("batched integer x36, engine", engine)
    plan = cv.BatchedPlan([(torch.from_numpy(A).to(dev), P, Q) for (A, P, Q) in batch], engine=engine)
    outs = plan.run()
    torch.cuda.synchronize()
    thr = oracle_mod.max_threads()
    for (A, P, Q), R in zip(batch, outs):
        ref = oracle_mod.forward(A, P, Q, threads=thr)
        got = R.cpu().numpy()
        assert np.array_equal(got.real, ref.real) and np.array_equal(got.imag, ref.imag), (A.shape, P, Q)
    plan.close()


def test_batch_matrix_engine_forced(cv, tdev, oracle_mod):
    torch, dev = tdev
    batch = [(synth.gaussian(70, 90, seed=1), 16, 16), (synth.gaussian(120, 64, seed=2), 24, 16),
             (synth.gaussian(200, 220, seed=3), 16, 32)]
    _note("batched matrix engine forced x3")
    plan = cv.BatchedPlan([(torch.from_numpy(A).to(dev), P, Q) for (A, P, Q) in batch], engine="matrix")
    outs = plan.run()
    torch.cuda.synchronize()
    for (A, P, Q), R in zip(batch, outs):
        ref = oracle_mod.forward(A, P, Q, threads=oracle_mod.max_threads())
        got = R.cpu().numpy()
        assert np.linalg.norm(got - ref) / np.linalg.norm(ref) <= 1e-12
        assert np.array_equal(got, got.conj().T)
    plan.close()
    with pytest.raises(cv.CovestError) as e:   # Q < 4: no matrix-core kernel for it
        cv.BatchedPlan([(torch.zeros((64, 64), dtype=torch.complex64, device=dev), 16, 16),
                        (torch.zeros((64, 64), dtype=torch.complex64, device=dev), 4, 3)], engine="matrix")
    assert e.value.status == cv.ERR_UNSUPPORTED


def test_batch_errors(cv, tdev):
    torch, dev = tdev
    with pytest.raises(cv.CovestError):
        cv.BatchedPlan([(torch.zeros((8, 8), dtype=torch.complex64, device=dev), 9, 2)])
    with pytest.raises(cv.CovestError):
        cv.BatchedPlan([(torch.zeros((8, 8), dtype=torch.complex64, device=dev), 2, 2)], precision="bf16")


WIDTH_CASES = [((97, 131, 12, 4), (8, 4)), ((97, 131, 12, 4), (16, 16)), ((131, 97, 5, 13), (8, 8)),
               ((200, 150, 20, 24), (8, 12)), ((64, 64, 8, 8), (4, 4)), ((300, 64, 16, 12), (12, 8)),
               ((256, 256, 16, 16), (8, 16)), ((256, 256, 16, 16), (16, 8))]


@pytest.mark.parametrize("case", WIDTH_CASES, ids=lambda c: "x".join(map(str, c[0])) + f"_w{c[1][0]}_{c[1][1]}")
def test_ring_width_overrides(cv, tdev, oracle_mod, case):
    torch, dev = tdev
    (N, M, P, Q), (w0, w1) = case
    A = synth.small_int(N, M, seed=N + M + w0 + w1)
    _note("ring widths", case)
    R = cv.covest_forward(torch.from_numpy(A).to(dev), P, Q, ring_cols=w0, ring_rows=w1)
    torch.cuda.synchronize()
    ref = oracle_mod.forward(A, P, Q, threads=oracle_mod.max_threads())
    got = R.cpu().numpy()
    assert np.array_equal(got.real, ref.real) and np.array_equal(got.imag, ref.imag)
