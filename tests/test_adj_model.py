"""CPU model of the adjoint's matrix-core interior (adj_int_mfma and
adj_bnd_combine): the kernels' own index arithmetic -- weight and operand
lanes, the clamped and zeroed second-operand columns, each wave's ring of
output rows, the workgroup sum in wave order, the rows two spans share and
their combination -- replayed with numpy tile products in the
three-multiplication form, against the oracle's adjoint (its direct loops).
Every address the kernels would touch is checked against its buffer, and
every interior output must be written exactly once.
"""
import numpy as np
import pytest

from paper_1303_2285_amd import synth

SPAN, WROWS, WAVES = 64, 8, 8


def full_lag_weights(G, P, Q):
    """W[a][b]: sum over the window offsets of H[k(i1, j1)][k(i1+dr, j1+dc)],
    H = G + G^H (the lag's sum over every offset that keeps both inside)."""
    H = G + G.conj().T
    W = np.zeros((2 * P - 1, 2 * Q - 1), np.complex128)
    for a in range(2 * P - 1):
        dr = a - (P - 1)
        for b in range(2 * Q - 1):
            dc = b - (Q - 1)
            for i1 in range(max(0, -dr), min(P, P - dr)):
                for j1 in range(max(0, -dc), min(Q, Q - dc)):
                    W[a, b] += H[i1 + P * j1, (i1 + dr) + P * (j1 + dc)]
    return W


def model(A, G, P, Q):
    N, M = A.shape
    nlr, nlc = 2 * P - 1, 2 * Q - 1
    Kr, Kc = N - P + 1, M - Q + 1
    ny, nx = Kr - P + 1, Kc - Q + 1
    mtiles, mranges = (nx + 15) // 16, (N + SPAN - 1) // SPAN
    Hh = 2 * P - 2
    brows = WROWS + Hh
    MT = 1 if nlr <= 16 else 2
    ks_n = (nlc + 3) // 4
    xpad = 16 * mtiles
    W = full_lag_weights(G, P, Q)
    # first operand: lane (n, g) of k-step ks holds W[16 mt + n][4 ks + g], zero past the lags
    Wp = np.zeros((16 * MT, 4 * 8), np.complex128)
    Wp[:nlr, :nlc] = W
    Wp = Wp[:, :4 * ks_n]
    bnd = np.full((max(mranges - 1, 0), 2, Hh, xpad), np.nan + 0j)
    out = np.full((N, M), np.nan + 0j)
    writes = np.zeros((N, M), int)
    K = float(Kr * Kc)
    n_idx = np.arange(16)
    b_idx = np.arange(4 * ks_n)
    for blk in range(mtiles * mranges):
        tile, rng = blk % mtiles, blk // mtiles
        x0, rho0 = 16 * tile, SPAN * rng
        ring = np.zeros((WAVES, brows, 16), np.complex128)
        for w in range(WAVES):
            rw = rho0 + WROWS * w
            for t in range(min(WROWS, N - rw)):
                rho = rw + t
                assert 0 <= rho < N
                cols = np.minimum(x0 + n_idx[None, :] + b_idx[:, None], M - 1)   # [b, n]
                assert cols.min() >= 0 and cols.max() < M
                X = A[rho, cols].astype(np.complex128)
                X[b_idx >= nlc, :] = 0
                xr, xi = X.real, X.imag
                k1 = (Wp.real + Wp.imag) @ xr
                k2 = Wp.real @ (xi - xr)
                k3 = Wp.imag @ (xr + xi)
                Y = (k1 - k3) + 1j * (k1 + k2)
                for a in range(nlr):
                    r = t - a + Hh
                    assert 0 <= r < brows
                    ring[w, r] += Y[a]
        for row in range(SPAN + Hh):
            y = rho0 - Hh + row
            for nn in range(16):
                x = x0 + nn
                if y < 0 or y >= ny or x >= nx:
                    continue
                s = 0j
                for w in range(WAVES):
                    br = y - (rho0 + WROWS * w - Hh)
                    if 0 <= br < brows:
                        s += ring[w, br, nn]
                if rng > 0 and y < rho0:
                    br = y - (rho0 - Hh)
                    assert 0 <= br < Hh and x < xpad
                    bnd[rng - 1, 1, br, x] = s
                elif y + Hh >= rho0 + SPAN:
                    br = y - (rho0 + SPAN - Hh)
                    assert rng < mranges - 1 and 0 <= br < Hh
                    bnd[rng, 0, br, x] = s
                else:
                    out[y + P - 1, x + Q - 1] = s / K
                    writes[y + P - 1, x + Q - 1] += 1
    for b in range(mranges - 1):
        for br in range(Hh):
            y = SPAN * (b + 1) - Hh + br
            if y >= ny:
                continue
            for x in range(nx):
                u, v = bnd[b, 0, br, x], bnd[b, 1, br, x]
                assert np.isfinite(u) and np.isfinite(v), (b, br, x)
                out[y + P - 1, x + Q - 1] = (u + v) / K
                writes[y + P - 1, x + Q - 1] += 1
    inner = (slice(P - 1, Kr), slice(Q - 1, Kc))
    assert np.all(writes[inner] == 1)
    assert writes.sum() == ny * nx
    return out[inner]


SHAPES = [(9, 11, 3, 4), (20, 18, 4, 4), (64, 64, 8, 8), (70, 50, 16, 12), (150, 70, 9, 13),
          (200, 90, 16, 16), (65, 40, 16, 16), (130, 37, 1, 5), (129, 20, 2, 1), (97, 47, 16, 1)]


@pytest.mark.parametrize("shape", SHAPES, ids=lambda s: "x".join(map(str, s)))
def test_mfma_interior_model(oracle_mod, shape):
    N, M, P, Q = shape
    A = synth.gaussian(N, M, seed=N + 7 * M + P)
    rng = np.random.default_rng(N * M + Q)
    G = rng.standard_normal((P * Q, P * Q)) + 1j * rng.standard_normal((P * Q, P * Q))
    got = model(A, G, P, Q)
    ref = oracle_mod.adjoint(A, G, P, Q)[P - 1:N - 2 * P + 2 + P - 1, Q - 1:M - 2 * Q + 2 + Q - 1]
    assert np.linalg.norm(got - ref) <= 1e-12 * np.linalg.norm(ref)
