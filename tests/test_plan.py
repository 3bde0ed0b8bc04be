"""Host-side plan layer of libcovest (no GPU needed).

* Counts against the paper: |UC| = 113 and 313 (Sec. 5.1), 626 for two
  matrices, eq. 3.4, the closed form of UM (eq. 4.6), the coverage identity
  sum of eta = PQ(PQ+1)/2 (eqs. 4.18-4.23) and SM / UM_hat = 45.125 (eq. 4.9).
* Ownership: every product of every unique combination is owned by exactly one
  job of the main kernel or by the finalize step, and every upper-triangle entry
  by exactly one finalize item (single writer, Sec. 3.3 proposition and
  Sec. 4.2-4.3), for the tile choices the planner makes.
* Decomposition: a NumPy model of the job split and of the finalize recurrence
  (middle sums, strip sums, corner products, sliding box) reproduces the oracle
  exactly on small-integer inputs.
"""
import itertools
import json
import os

import numpy as np
import pytest

from paper_1303_2285_amd import covest as cv
from paper_1303_2285_amd import synth

GOLDEN = os.path.join(os.path.dirname(__file__), "golden", "paper_counts.json")


def uc_set(P, Q):
    """Unique combinations (eq. 3.3)."""
    s = {(dr, dc) for dr in range(0, P) for dc in range(0, Q)}
    s |= {(dr, dc) for dr in range(-(P - 1), 0) for dc in range(1, Q)}
    return s


def upper_owner(P, Q):
    """Owner combination of every upper entry, from the index map (eq. 2.1)."""
    own = {}
    for k1 in range(P * Q):
        for k2 in range(k1, P * Q):
            i1, j1, i2, j2 = k1 % P, k1 // P, k2 % P, k2 // P
            own[(k1, k2)] = (i2 - i1, j2 - j1)
    return own


@pytest.fixture(scope="module")
def golden():
    with open(GOLDEN) as f:
        return json.load(f)


def test_paper_combination_counts(golden):
    for e in golden["unique_combinations"]:
        c = cv.counts(e["N"], e["M"], e["P"], e["Q"])
        assert c["n_uc"] == e["value"], e["cite"]
        assert len(uc_set(e["P"], e["Q"])) == e["value"], e["cite"]
    e = golden["second_combination_count"][0]
    assert 2 * cv.counts(e["N"], e["M"], e["P"], e["Q"])["n_uc"] == e["value"]


def test_sm_over_um_hat(golden):
    e = golden["sm_over_um_hat"]
    N, M, P, Q = e["N"], e["M"], e["P"], e["Q"]
    sm = (N - P) * (M - Q) * P * P * Q * Q                           # eq. 4.1
    um_hat = 2 * (P / 2) * (2 * N - (P - 1)) * (Q / 2) * (2 * M - (Q - 1))  # eq. 4.7
    assert sm / um_hat == e["value"]
    # the bound really bounds UM (eq. 4.7)
    assert cv.counts(N, M, P, Q)["um"] <= um_hat


@pytest.mark.parametrize("shape", [(20, 20, 8, 8), (32, 32, 13, 13), (64, 64, 8, 8), (256, 256, 16, 16),
                                   (1024, 1024, 32, 32), (512, 300, 12, 4), (7, 9, 7, 1), (5, 5, 1, 5)])
def test_counts_closed_forms(shape):
    N, M, P, Q = shape
    c = cv.counts(N, M, P, Q)
    assert c["K"] == (N - P + 1) * (M - Q + 1)
    assert c["n_uc"] == P * Q + (P - 1) * (Q - 1)                     # eq. 3.4
    um1 = P * (2 * N - P + 1) * Q * (2 * M - Q + 1) // 4               # eq. 4.4
    um2 = (P - 1) * (2 * N - P) * (Q - 1) * (2 * M - Q) // 4          # eq. 4.5
    assert c["um"] == um1 + um2                                        # eq. 4.6
    assert c["um"] == sum((N - abs(dr)) * (M - abs(dc)) for dr, dc in uc_set(P, Q))  # eq. 3.6
    eta = sum((P - abs(dr)) * (Q - abs(dc)) for dr, dc in uc_set(P, Q))  # eq. 3.8
    assert eta == c["eta"] == P * Q * (P * Q + 1) // 2                  # eqs. 4.22, 4.23
    assert c["segments"] == sum(Q - abs(dc) for dr, dc in uc_set(P, Q))


def test_uc_owns_each_upper_entry_once():
    """Sec. 4.2-4.3: the combinations' write sets partition the upper triangle."""
    for P, Q in [(3, 4), (4, 3), (5, 5), (1, 6), (6, 1)]:
        own = upper_owner(P, Q)
        assert set(own.values()) == uc_set(P, Q)
        per = {}
        for (k1, k2), d in own.items():
            per[d] = per.get(d, 0) + 1
        for (dr, dc), n in per.items():
            assert n == (P - abs(dr)) * (Q - abs(dc))   # eta (eq. 3.8)


def test_count_errors():
    with pytest.raises(cv.CovestError) as e:
        cv.counts(4, 4, 5, 1)
    assert e.value.status == cv.ERR_SHAPE
    with pytest.raises(cv.CovestError) as e:
        cv.counts(4, 4, 0, 1)
    assert e.value.status == cv.ERR_SHAPE


# ---------------------------------------------------------------------------
# Ownership of products by the plan's jobs
# ---------------------------------------------------------------------------

def group_lags(g):
    orient, W, d1lo, d1hi, ch0, nch, v2lo, v2hi, lanes, slots = g[:10]
    out = []
    for li in range(lanes):
        d1 = d1lo + li // nch
        base = ch0 + (li % nch) * W
        for w in range(W):
            d2 = base + w
            if v2lo <= d2 < v2hi:
                out.append((d2, d1) if orient else (d1, d2))
    return out


def coverage(info, jobs, groups, N, M):
    """Per group: how many times each B position is covered by its jobs."""
    cov = {}
    for gid, g in enumerate(groups):
        orient = g[0]
        shape = (M, N) if orient else (N, M)
        cov[gid] = np.zeros(shape, dtype=np.int32)
    for j in jobs:
        mode, inst, gid, out, u0, u1, x0, x1, c0, c1, tr, tc = j
        g = groups[gid]
        if mode == 0:
            S = g[9]
            nrg = -(-(info["Rm1"] - info["Rm0"]) // S)
            for u in range(u0, u1):
                band, rg = divmod(u, nrg)
                r0 = info["Rm0"] + rg * S
                r1 = min(info["Rm1"], r0 + S)
                cc = info["Cm0"] + band * info["bandw"]
                cov[gid][r0:r1, cc:cc + info["bandw"]] += 1
        else:
            assert x1 - x0 <= 4 * g[9]
            assert (c1 - c0) % g[1] == 0 and tc % g[1] == 0
            cov[gid][x0:x1, c0:c1] += 1
    return cov


SHAPES = [(64, 64, 8, 8), (256, 256, 16, 16), (1024, 1024, 32, 32), (512, 512, 16, 16),
          (97, 131, 12, 4), (40, 33, 4, 16), (9, 9, 5, 5), (6, 7, 6, 7), (300, 64, 16, 12),
          (130, 200, 3, 1), (50, 50, 1, 1), (200, 200, 40, 24)]


WIDTHS = [(0, 0), (8, 8), (4, 16), (16, 4), (12, 12)]


@pytest.mark.parametrize("shape", SHAPES)
@pytest.mark.parametrize("n_slots", [512, 64, 1])
@pytest.mark.parametrize("widths", WIDTHS, ids=lambda w: f"w{w[0]}_{w[1]}")
def test_plan_ownership(shape, n_slots, widths):
    N, M, P, Q = shape
    info, jobs, groups, items = cv.plan_tables(N, M, P, Q, n_slots, *widths)
    Rm0, Rm1, Cm0, Cm1 = info["Rm0"], info["Rm1"], info["Cm0"], info["Cm1"]
    assert P - 1 <= Rm0 <= Rm1 <= max(Rm0, N - P + 1)
    assert Q - 1 <= Cm0 <= Cm1 <= max(Cm0, M - Q + 1)
    assert (Rm1 - Rm0) % info["W1"] == 0 and (Cm1 - Cm0) % info["bandw"] == 0
    UC = uc_set(P, Q)
    # every UC lag in exactly one group of each orientation, nothing else
    for orient in (0, 1):
        seen = []
        for g in groups:
            if g[0] == orient:
                seen += group_lags(g)
                assert g[8] <= 64 and g[9] == 64 // g[8]
        assert sorted(seen) == sorted(UC)
    cov = coverage(info, jobs, groups, N, M)
    mid_r = np.zeros(N, bool)
    mid_r[Rm0:Rm1] = True
    mid_c = np.zeros(M, bool)
    mid_c[Cm0:Cm1] = True
    for gid, g in enumerate(groups):
        if g[0] == 0:   # bulk: middle x middle; row strips: individual rows x middle cols
            want = np.where(mid_c[None, :], 1, 0) * np.ones((N, 1), int)
        else:           # column strips: individual cols x middle rows (B = A^T)
            want = np.where(mid_r[None, :], 1, 0) * np.where(~mid_c[:, None], 1, 0)
        assert np.array_equal(cov[gid], want), gid
    # outputs: bulk rows unique per group, strip rows = individual index
    bulk_outs = {}
    for j in jobs:
        if j[0] == 0:
            bulk_outs.setdefault(j[2], []).append(j[3])
        else:
            g = groups[j[2]]
            lo = Rm0 if g[0] == 0 else Cm0
            hi = Rm1 if g[0] == 0 else Cm1
            for t in range(j[6], j[7]):
                idx = t if t < lo else lo + (t - hi)
                assert j[3] + (t - j[6]) == idx
    all_outs = sorted(o for v in bulk_outs.values() for o in v)
    assert all_outs == list(range(info["n_bulk"]))
    # finalize items: the UC set once each, pointing at their group's partial rows
    assert sorted((int(i[1]), int(i[2])) for i in items) == sorted(UC)
    for it in items:
        dr, b0, b1 = it[1], it[3], it[4]
        owners = [gid for gid, g in enumerate(groups)
                  if g[0] == 0 and g[2] <= dr < g[3] and (dr >= 0) == (g[2] >= 0)]
        assert len(owners) == 1
        assert sorted(bulk_outs.get(owners[0], [])) == list(range(b0, b1))
    # products: the main kernel keeps all but the corner products
    c = cv.counts(N, M, P, Q)
    assert info["main_products"] + info["fin_products"] == c["um"]


def test_width_errors():
    with pytest.raises(cv.CovestError) as e:
        cv.plan_info(64, 64, 8, 8, 512, 5, 0)
    assert e.value.status == cv.ERR_INVALID_ARG


def test_plan_cfg3_fills_the_gpu():
    info = cv.plan_info(1024, 1024, 32, 32, 512)
    assert info["n_jobs"] == 512
    assert info["lds_main"] <= 80 * 1024      # two workgroups per compute unit


# ---------------------------------------------------------------------------
# The decomposition itself, modelled on the CPU
# ---------------------------------------------------------------------------

def model_forward(A, P, Q, info):
    """R from middle sums, strip sums, corner products and sliding boxes."""
    A = np.asarray(A, dtype=np.complex128)
    N, M = A.shape
    Kr, Kc = N - P + 1, M - Q + 1
    Rm0, Rm1, Cm0, Cm1 = info["Rm0"], info["Rm1"], info["Cm0"], info["Cm1"]
    ind_r = [r for r in range(N) if r < Rm0 or r >= Rm1]
    ind_c = [c for c in range(M) if c < Cm0 or c >= Cm1]
    rho = {r: i for i, r in enumerate(ind_r)}
    gam = {c: i for i, c in enumerate(ind_c)}
    R = np.zeros((P * Q, P * Q), dtype=np.complex128)
    for dr, dc in uc_set(P, Q):
        Pi = np.zeros((N, M), dtype=np.complex128)
        r0, r1 = max(0, -dr), N - max(0, dr)
        Pi[r0:r1, :M - dc] = A[r0:r1, :M - dc] * A[r0 + dr:r1 + dr, dc:].conj()
        zm = Pi[Rm0:Rm1, Cm0:Cm1].sum()
        zr = {r: Pi[r, Cm0:Cm1].sum() for r in ind_r}
        zc = {c: Pi[Rm0:Rm1, c].sum() for c in ind_c}
        nr, nc = P - abs(dr), Q - dc
        rlo = max(0, -dr)
        cs = {}
        for cls in ["mid"] + [r for r in ind_r if r0 <= r < r1]:
            if cls == "mid":
                base, ind = zm, (lambda c: zc[c])
            else:
                base, ind = zr[cls], (lambda c, r=cls: Pi[r, c])
            s = base + sum(ind(c) for c in ind_c if c < Kc)
            row = [s]
            for b in range(nc - 1):
                s = s - ind(b) + ind(b + Kc)
                row.append(s)
            cs[cls] = row
        for b in range(nc):
            s = cs["mid"][b] + sum(cs[r][b] for r in ind_r if rlo <= r < rlo + Kr)
            for a in range(nr):
                i1 = rlo + a
                k1, k2 = i1 + P * b, i1 + dr + P * (b + dc)
                K = float(Kr * Kc)
                v = complex(s.real / K, 0.0 if k1 == k2 else s.imag / K)
                R[k1, k2] = v
                R[k2, k1] = v.conjugate()
                if a + 1 < nr:
                    s = s - cs[i1][b] + cs[i1 + Kr][b]
    return R


@pytest.mark.parametrize("shape", [(64, 64, 8, 8), (40, 33, 4, 16), (9, 9, 5, 5), (6, 7, 6, 7),
                                   (130, 64, 3, 1), (20, 20, 1, 1), (72, 70, 12, 4)])
def test_decomposition_reproduces_oracle(oracle_mod, shape):
    N, M, P, Q = shape
    A = synth.small_int(N, M, seed=N + 7 * M)
    for widths in WIDTHS:
        info = cv.plan_info(N, M, P, Q, 512, *widths)
        R = model_forward(A, P, Q, info)
        ref = oracle_mod.forward(A, P, Q)
        assert np.array_equal(R.real, ref.real) and np.array_equal(R.imag, ref.imag), widths
    info = cv.plan_info(N, M, P, Q)
    R = model_forward(A, P, Q, info)
    ref = oracle_mod.forward(A, P, Q)
    assert np.array_equal(R.real, ref.real)
    assert np.array_equal(R.imag, ref.imag)
