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

def model_finalize(A, P, Q, info, sums):
    """R from the middle, strip and corner sums by sliding boxes (the finalize).

    sums(dr, dc) -> (zm, zr, zc): the middle sum, {individual row: sum over
    the middle columns} and {individual column: sum over the middle rows}."""
    A = np.asarray(A, dtype=np.complex128)
    N, M = A.shape
    Kr, Kc = N - P + 1, M - Q + 1
    Rm0, Rm1, Cm0, Cm1 = info["Rm0"], info["Rm1"], info["Cm0"], info["Cm1"]
    ind_r = [r for r in range(N) if r < Rm0 or r >= Rm1]
    ind_c = [c for c in range(M) if c < Cm0 or c >= Cm1]
    R = np.zeros((P * Q, P * Q), dtype=np.complex128)
    for dr, dc in uc_set(P, Q):
        Pi = np.zeros((N, M), dtype=np.complex128)
        r0, r1 = max(0, -dr), N - max(0, dr)
        Pi[r0:r1, :M - dc] = A[r0:r1, :M - dc] * A[r0 + dr:r1 + dr, dc:].conj()
        zm, zr, zc = sums(dr, dc)
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


def model_forward(A, P, Q, info):
    """R from middle sums, strip sums, corner products and sliding boxes."""
    A = np.asarray(A, dtype=np.complex128)
    N, M = A.shape
    Rm0, Rm1, Cm0, Cm1 = info["Rm0"], info["Rm1"], info["Cm0"], info["Cm1"]

    def sums(dr, dc):
        Pi = np.zeros((N, M), dtype=np.complex128)
        r0, r1 = max(0, -dr), N - max(0, dr)
        Pi[r0:r1, :M - dc] = A[r0:r1, :M - dc] * A[r0 + dr:r1 + dr, dc:].conj()
        zm = Pi[Rm0:Rm1, Cm0:Cm1].sum()
        zr = {r: Pi[r, Cm0:Cm1].sum() for r in range(N) if r < Rm0 or r >= Rm1}
        zc = {c: Pi[Rm0:Rm1, c].sum() for c in range(M) if c < Cm0 or c >= Cm1}
        return zm, zr, zc

    return model_finalize(A, P, Q, info, sums)


def dpp_scan(v):
    """The wave-scan finalize's prefix sum over 64 lanes, step by step: row
    shifts by 1, 2 and 3 of the original values, row shifts by 4 and 8 of the
    running sums (a lane whose source lies before its row of 16 reads zero),
    then the total of row 0 into row 1 and of row 2 into row 3, and the total
    of rows 0-1 into rows 2 and 3; lanes a step does not reach add zero."""
    v = np.asarray(v, dtype=complex)
    i = np.arange(64)
    s = v.copy()
    for k in (1, 2, 3):
        s = s + np.where(i % 16 >= k, np.roll(v, k), 0)
    s = s + np.where(i % 16 >= 4, np.roll(s, 4), 0)
    s = s + np.where(i % 16 >= 8, np.roll(s, 8), 0)
    s = s + np.where(np.isin(i // 16, (1, 3)), s[(i // 16) * 16 - 1], 0)
    s = s + np.where(i // 16 >= 2, s[31], 0)
    return s


def test_dpp_scan_is_a_prefix_sum():
    rng = np.random.default_rng(5)
    for _ in range(20):
        v = rng.integers(-1000, 1000, 64) + 1j * rng.integers(-1000, 1000, 64)
        assert np.array_equal(dpp_scan(v), np.cumsum(v))


def model_finalize_scan(A, P, Q, info, sums):
    """R from the same sums as the wave-scan finalize takes them: per class
    (the middle rows, then each individual row) a prefix sum over the
    individual columns, read at the ends of each offset's column range; per
    column offset a prefix sum over the individual rows, read at the ends of
    each row offset's range; rows and columns a lag cannot use zeroed.  The
    prefix sums are np.cumsum (test_dpp_scan_is_a_prefix_sum pins the lane
    pattern to it; on integer inputs the order of the additions is moot)."""
    A = np.asarray(A, dtype=np.complex128)
    N, M = A.shape
    Kr, Kc = N - P + 1, M - Q + 1
    Rm0, Rm1, Cm0, Cm1 = info["Rm0"], info["Rm1"], info["Cm0"], info["Cm1"]
    ind_r = [r for r in range(N) if r < Rm0 or r >= Rm1]
    ind_c = [c for c in range(M) if c < Cm0 or c >= Cm1]
    nir = len(ind_r)

    def span(x0, n, m0, m1):
        lo = x0 if x0 < m0 else m0 + max(0, x0 - m1)
        hi = m0 + x0 + n - m1 if x0 + n > m1 else min(m0, x0 + n)
        return lo, hi

    def at(p, i):
        return p[i] if i >= 0 else 0

    R = np.zeros((P * Q, P * Q), dtype=np.complex128)
    for dr, dc in uc_set(P, Q):
        rlo, rhi = max(0, -dr), N - max(0, dr)
        zm, zr, zc = sums(dr, dc)
        zm = zm if Rm1 > Rm0 else 0
        nr, nc = P - abs(dr), Q - dc
        St = np.zeros((nc, 1 + nir), complex)
        cols = np.array(ind_c, dtype=int)
        col_ok = cols + dc < M
        for cls in range(1 + nir):
            v = np.zeros(64, complex)
            base = 0
            if cls == 0:
                if Rm1 > Rm0:
                    v[:len(cols)] = [zc[c] if ok else 0 for c, ok in zip(ind_c, col_ok)]
            else:
                r = ind_r[cls - 1]
                if rlo <= r < rhi:
                    base = zr[r] if Cm1 > Cm0 else 0
                    cc = np.where(col_ok, cols, 0)
                    v[:len(cols)] = np.where(col_ok, A[r, cc] * np.conj(A[r + dr, cc + dc]), 0)
            pre = np.cumsum(v)
            for b in range(nc):
                glo, ghi = span(b, Kc, Cm0, Cm1)
                St[b, cls] = base + (at(pre, ghi - 1) - at(pre, glo - 1))
        for b in range(nc):
            u = np.zeros(64, complex)
            u[:nir] = St[b, 1:]
            pre = np.cumsum(u)
            for a in range(nr):
                ra, rb = span(rlo + a, Kr, Rm0, Rm1)
                v = zm + St[b, 0] + (at(pre, rb - 1) - at(pre, ra - 1))
                i1 = rlo + a
                k1, k2 = i1 + P * b, i1 + dr + P * (b + dc)
                K = float(Kr * Kc)
                v = complex(v.real / K, 0.0 if k1 == k2 else v.imag / K)
                R[k1, k2] = v
                R[k2, k1] = v.conjugate()
    return R


@pytest.mark.parametrize("shape", [(64, 64, 8, 8), (40, 33, 4, 16), (9, 9, 5, 5), (6, 7, 6, 7),
                                   (72, 70, 12, 4), (31, 31, 16, 16), (80, 90, 32, 32)])
def test_scan_finalize_reproduces_oracle(oracle_mod, shape):
    """The wave-scan finalize's index ranges and prefix sums, for every plan
    whose individual rows and columns fit one wave."""
    N, M, P, Q = shape
    A = synth.small_int(N, M, seed=N + 5 * M)
    ref = oracle_mod.forward(A, P, Q)
    infos = [cv.plan_info(N, M, P, Q, 512, *w) for w in WIDTHS]
    if N >= 2 * P - 1 and M >= 2 * Q - 1 and Q >= 4:
        infos.append(cv.mfma_plan(N, M, P, Q)[0])
    A128 = np.asarray(A, dtype=np.complex128)
    checked = 0
    for info in infos:
        Rm0, Rm1, Cm0, Cm1 = info["Rm0"], info["Rm1"], info["Cm0"], info["Cm1"]
        if info["n_ir"] > 63 or info["n_ic"] > 64:
            continue

        def sums(dr, dc):
            Pi = np.zeros((N, M), dtype=np.complex128)
            r0, r1 = max(0, -dr), N - max(0, dr)
            Pi[r0:r1, :M - dc] = A128[r0:r1, :M - dc] * A128[r0 + dr:r1 + dr, dc:].conj()
            zm = Pi[Rm0:Rm1, Cm0:Cm1].sum()
            zr = {r: Pi[r, Cm0:Cm1].sum() for r in range(N) if r < Rm0 or r >= Rm1}
            zc = {c: Pi[Rm0:Rm1, c].sum() for c in range(M) if c < Cm0 or c >= Cm1}
            return zm, zr, zc

        R = model_finalize_scan(A, P, Q, info, sums)
        assert np.array_equal(R.real, ref.real) and np.array_equal(R.imag, ref.imag), info
        checked += 1
    assert checked > 0


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


# ---------------------------------------------------------------------------
# The matrix-core engine's plan: ownership and a model of its kernel
# ---------------------------------------------------------------------------

MFMA_SHAPES = [(1024, 1024, 32, 32), (256, 256, 16, 16), (512, 512, 16, 16), (40, 36, 16, 16),
               (31, 31, 16, 16), (50, 47, 24, 24), (70, 40, 32, 16), (34, 64, 16, 32), (300, 64, 28, 28),
               (64, 64, 8, 8), (15, 7, 8, 4), (90, 70, 12, 12), (1, 9, 1, 4), (2, 7, 1, 4), (3, 7, 2, 4),
               (3, 200, 2, 64)]


def test_mfma_fits():
    # the planner takes any shape the kernel can run (tile padding only costs speed)
    for shape in [(1024, 1024, 32, 32), (256, 256, 16, 16), (50, 47, 24, 24), (70, 40, 32, 16),
                  (64, 64, 8, 8), (256, 256, 12, 12), (15, 7, 8, 4)]:
        cv.mfma_plan(*shape)
    for shape in [(300, 300, 48, 48), (30, 40, 16, 16), (40, 30, 16, 16), (64, 64, 8, 3), (14, 7, 8, 4)]:
        with pytest.raises(cv.CovestError) as e:
            cv.mfma_plan(*shape)
        assert e.value.status == cv.ERR_UNSUPPORTED, shape


def mfma_visits(job):
    """(line, k-group) pairs a job covers, per wave."""
    inst, o, kind, out, line0, line_end, b0, kg0, b1, kg1, nkg = job[:11]
    for bl in range(b0, b1 + 1):
        kga = kg0 if bl == b0 else 0
        kgb = kg1 if bl == b1 else nkg
        for w in range(8):
            line = line0 + 8 * bl + w
            if kga < kgb and line < line_end:
                for kg in range(kga, kgb):
                    yield w, line, kg


@pytest.mark.parametrize("shape", MFMA_SHAPES)
@pytest.mark.parametrize("n_cu", [256, 16, 3, 1])
def test_mfma_plan_ownership(shape, n_cu):
    N, M, P, Q = shape
    info, jobs, items = cv.mfma_plan(N, M, P, Q, n_cu)
    assert (info["Rm0"], info["Rm1"], info["Cm0"], info["Cm1"]) == (P - 1, N - P + 1, Q - 1, M - Q + 1)
    assert info["mt"] == -(-(2 * P - 1) // 16) and info["nt"] == -(-Q // 16)
    nkg = {0: -(-(info["Cm1"] - info["Cm0"] + Q - 1) // 4), 1: -(-(info["Rm1"] - info["Rm0"] + 2 * (P - 1)) // 4)}
    ind = {0: [r for r in range(N) if r < info["Rm0"] or r >= info["Rm1"]],
           1: [c for c in range(M) if c < info["Cm0"] or c >= info["Cm1"]]}
    zp = info["zpieces"]
    bulk = {}
    strip = {0: {}, 1: {}}
    bulk_outs = []
    for j in jobs:
        o, kind, out, line0 = int(j[1]), int(j[2]), int(j[3]), int(j[4])
        assert j[10] == nkg[o]
        assert (j[11], j[12]) == ((info["Cm0"], info["Cm1"]) if o == 0 else (info["Rm0"], info["Rm1"]))
        # orientation 0 ends at A's last column (its first operand is read
        # unchecked); orientation 1 starts at row 0
        assert j[13] == (info["Cm1"] + Q - 1 - 4 * nkg[0] if o == 0 else info["Rm0"] - (P - 1))
        assert j[13] >= 0 and j[13] + 4 * j[10] <= (M if o == 0 else N + 3)
        if kind == 0:
            assert o == 0 and (j[4], j[5]) == (info["Rm0"], info["Rm1"])
            bulk_outs.append(out)
            for w, line, kg in mfma_visits(j):
                bulk[(line, kg)] = bulk.get((line, kg), 0) + 1
        else:
            assert j[6] == j[8] == 0 and j[5] - j[4] <= 8
            # every piece of every strip line is written (the finalize adds them all)
            assert j[9] > j[7]
            for w, line, kg in mfma_visits(j):
                zrow = out + (line - line0)
                piece, idx = divmod(zrow, len(ind[o]))
                assert piece < zp and ind[o][idx] == line
                key = (line, kg)
                assert key not in strip[o]
                strip[o][key] = piece
    assert sorted(bulk_outs) == list(range(info["n_bulk"]))
    want = {(l, k) for l in range(info["Rm0"], info["Rm1"]) for k in range(nkg[0])}
    assert set(bulk) == want and all(v == 1 for v in bulk.values())
    for o in (0, 1):
        assert set(strip[o]) == {(l, k) for l in ind[o] for k in range(nkg[o])}
        # pieces cover consecutive k-groups in piece order
        for l in ind[o]:
            ps = [strip[o][(l, k)] for k in range(nkg[o])]
            assert ps == sorted(ps)
    assert sorted((int(i[1]), int(i[2])) for i in items) == sorted(uc_set(P, Q))
    assert all(i[3] == 0 and i[4] == info["n_bulk"] for i in items)
    c = cv.counts(N, M, P, Q)
    assert info["main_products"] + info["fin_products"] == c["um"]
    if n_cu == 256 and N * M >= 256 * 256:
        assert len(jobs) <= 256
        # cost of a job: (block, k-group) steps, its waves running side by side
        cost = [len({((line - j[4]) // 8, kg) for w, line, kg in mfma_visits(j)}) for j in jobs]
        assert max(cost) <= 1.15 * (sum(cost) / 256) + 1   # balanced to a few percent


def mfma_first_operand_rows_cols(job, info, N, M, P, Q, kin):
    """Every A element the matrix-core kernel's first-operand loads touch for
    one job, as (row, col) arrays: per visited (line, k-group), the 16*mt
    lines of each tile row, clamped to the input, at the k-group's 4
    positions, unclamped below kin and clamped to the line's end from kin on
    (the kernel's two loaders)."""
    o, kind, out, line0, line_end, b0, kg0, b1, kg1, nkg, plo, phi, k0 = [int(v) for v in job[1:14]]
    nlines, npos = (M, N) if o else (N, M)
    tm = info["nt"] if o else info["mt"]
    d1lo = 0 if o else -(P - 1)
    d1 = d1lo + np.arange(16 * tm)
    rows, cols = [], []
    for w, line, kg in mfma_visits(job):
        q = np.clip(line + d1, 0, nlines - 1)
        pos = k0 + 4 * kg + np.arange(4)
        if kg >= kin:
            pos = np.minimum(pos, npos - 1)
        qq, pp = np.meshgrid(q, pos, indexing="ij")
        rows.append(qq.ravel())
        cols.append(pp.ravel())
    if not rows:
        return np.zeros(0, int), np.zeros(0, int)
    lines, poss = np.concatenate(rows), np.concatenate(cols)
    return (poss, lines) if o else (lines, poss)


def c_trunc_div(a, b):
    return int(a / b)   # C's integer division truncates toward zero


# N <= 3 with P in {1, 2}: orientation-1 lines (columns of A) have fewer than
# 4 positions, so the one k-group of such a line must take the clamped loader
MFMA_THIN = [(N, 2 * Q - 1 + extra, P, Q) for N in (1, 2, 3) for P in (1, 2) for Q in (4, 5, 9, 16, 17, 33, 64)
             for extra in (0, 7) if N >= 2 * P - 1]


@pytest.mark.parametrize("shape", MFMA_THIN + [(64, 64, 8, 8), (5, 9, 3, 4), (1024, 1024, 32, 32),
                                               (7, 200, 4, 64), (4, 7, 2, 4)])
def test_mfma_first_operand_loads_stay_in_bounds(shape):
    N, M, P, Q = shape
    for n_cu in (256, 3):
        info, jobs, _ = cv.mfma_plan(N, M, P, Q, n_cu)
        for j in jobs:
            o, nkg, k0, kin = int(j[1]), int(j[10]), int(j[13]), int(j[14])
            npos = N if o else M
            # kin counts exactly the k-groups whose 4 positions lie inside the line
            assert kin == sum(1 for kg in range(nkg) if k0 + 4 * kg + 3 < npos)
            assert nkg - kin <= (1 if o else 0)
            r, c = mfma_first_operand_rows_cols(j, info, N, M, P, Q, kin)
            assert r.size == 0 or (r.min() >= 0 and r.max() < N and c.min() >= 0 and c.max() < M), (shape, j)


@pytest.mark.parametrize("shape", [(1, 9, 1, 4), (2, 7, 1, 4), (3, 7, 2, 4), (3, 200, 2, 64)])
def test_mfma_bounds_check_catches_truncating_kin(shape):
    """The count kin = (npos - 4 - k0) / 4 + 1 with C's truncating division is
    1, not 0, for a line of 1-3 positions; the bounds model must flag it."""
    N, M, P, Q = shape
    assert cv.mfma_fits(N, M, P, Q) and cv.mfma_preferred(N, M, P, Q)
    info, jobs, _ = cv.mfma_plan(N, M, P, Q, 256)
    bad = 0
    for j in jobs:
        o, k0 = int(j[1]), int(j[13])
        npos = N if o else M
        r, c = mfma_first_operand_rows_cols(j, info, N, M, P, Q, c_trunc_div(npos - 4 - k0, 4) + 1)
        bad += int(r.size > 0 and (r.max() >= N or c.max() >= M))
    assert bad > 0


def mfma_model_sums(A, P, Q, info, jobs):
    """What the matrix-core kernel computes, in NumPy: per job, the products of
    a block of lines (rows of A, or of A^T) with the Toeplitz band of the line,
    at clamped indices, summed over its k-groups; then the sums the finalize
    reads (bulk partials added, strip pieces added)."""
    A = np.asarray(A, dtype=np.complex128)
    N, M = A.shape
    mt, nt, zp = info["mt"], info["nt"], info["zpieces"]
    L = info["lag_stride"]
    # the workspace starts as garbage (NaN here): every sum the finalize reads
    # must have been written
    partial = np.full((info["n_bulk"], L), np.nan, dtype=np.complex128)
    z = {0: np.full((zp * info["n_ir"], L), np.nan, dtype=np.complex128),
         1: np.full((zp * info["n_ic"], L), np.nan, dtype=np.complex128)}

    def lag_rows(o, tm, tn):
        d1 = (0 if o else -(P - 1)) + np.arange(16 * tm)
        d2 = (-(P - 1) if o else 0) + np.arange(16 * tn)
        return d1, d2

    def store(row, o, d1, d2, T):
        for a, v1 in enumerate(d1):
            for b, v2 in enumerate(d2):
                dr, dc = (v2, v1) if o else (v1, v2)
                if 0 <= dc < Q and -P < dr < P and (dc > 0 or dr >= 0):
                    row[(dr + P - 1) * Q + dc] = T[a, b]

    for j in jobs:
        o, kind, out, line0, line_end, b0, kg0, b1, kg1, nkg, plo, phi, k0 = [int(v) for v in j[1:14]]
        B = A.T if o else A
        nlines, npos = B.shape
        tm, tn = (nt, mt) if o else (mt, nt)
        d1, d2 = lag_rows(o, tm, tn)
        acc = np.zeros((16 * tm, 16 * tn), dtype=np.complex128)
        for bl in range(b0, b1 + 1):
            kga = kg0 if bl == b0 else 0
            kgb = kg1 if bl == b1 else nkg
            for w in range(8):
                line = line0 + 8 * bl + w
                if kga >= kgb or line >= line_end:
                    continue
                cps = np.arange(k0 + 4 * kga, k0 + 4 * kgb)
                Y = B[np.clip(line + d1, 0, nlines - 1)][:, np.minimum(cps, npos - 1)]
                xp = cps[None, :] - d2[:, None]
                X = np.where((xp >= plo) & (xp < phi), B[line][np.clip(xp, 0, npos - 1)], 0)
                T = Y.conj() @ X.T
                if kind == 1:
                    store(z[o][out + line - line0], o, d1, d2, T)
                else:
                    acc += T
        if kind == 0:
            store(partial[out], o, d1, d2, acc)
    Rm0, Rm1, Cm0, Cm1 = info["Rm0"], info["Rm1"], info["Cm0"], info["Cm1"]
    ind_r = [r for r in range(N) if r < Rm0 or r >= Rm1]
    ind_c = [c for c in range(M) if c < Cm0 or c >= Cm1]

    def sums(dr, dc):
        lag = (dr + P - 1) * Q + dc
        zm = partial[:, lag].sum()
        zr = {r: sum(z[0][p * len(ind_r) + i, lag] for p in range(zp)) for i, r in enumerate(ind_r)}
        zc = {c: sum(z[1][p * len(ind_c) + i, lag] for p in range(zp)) for i, c in enumerate(ind_c)}
        return zm, zr, zc

    return sums


@pytest.mark.parametrize("shape", [(40, 36, 16, 16), (31, 31, 16, 16), (50, 47, 24, 24), (70, 40, 32, 16),
                                   (34, 64, 16, 32), (1, 9, 1, 4), (2, 7, 1, 4), (3, 7, 2, 4), (3, 200, 2, 64)])
@pytest.mark.parametrize("n_cu", [256, 5])
def test_mfma_model_reproduces_oracle(oracle_mod, shape, n_cu):
    N, M, P, Q = shape
    A = synth.small_int(N, M, seed=3 * N + M)
    info, jobs, items = cv.mfma_plan(N, M, P, Q, n_cu)
    R = model_finalize(A, P, Q, info, mfma_model_sums(A, P, Q, info, jobs))
    ref = oracle_mod.forward(A, P, Q)
    assert np.array_equal(R.real, ref.real) and np.array_equal(R.imag, ref.imag)
