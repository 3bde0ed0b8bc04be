"""CPU model of the plain form's 16-bit matrix-core path (B1-B3), no GPU.

`covest_hankel_plan_get` exposes the plan the library launches.  The model
replays what `hankel_main16` does with it -- staging rows of the packed
planes into LDS, each lane's row of X as an LDS offset, zero rows past PQ,
positions past a sub-block masked on both operands -- and

* checks every LDS offset and every plane element the kernel touches against
  the buffers the launch provides (the LDS bytes of the launch, the padded
  planes of the workspace);
* checks that an unmasked operand never reads an LDS word the current
  sub-block did not stage;
* sums the items' tiles the way `hankel_reduce16` does and compares R with
  the oracle (eq. 2.2) bit for bit on small-integer inputs (float64 sums of
  small integers are exact), so that a wrong row, column or position mapping
  fails here rather than on the device.

The model computes in float64 from the complex values: the 16-bit rounding is
the hardware's and is covered by the GPU tests.
"""
import numpy as np
import pytest

from paper_1303_2285_amd import covest as cv
from paper_1303_2285_amd import synth

PRECS = ["bf16", "bf16x3", "fp16", "fp16x3"]


def _geometry(info, it, P, Q, PQ):
    tr, tc = int(it[0]), int(it[1])
    tn = info["tn"]
    same = tn == 128 and tr == tc
    ja_lo, ja_hi = tr // P, min(Q - 1, min(PQ - 1, tr + 127) // P)
    jb_lo, jb_hi = tc // P, min(Q - 1, min(PQ - 1, tc + tn - 1) // P)
    rows = info["pb"] + P - 1
    sa, sb = info["stride_a"], info["stride_b"]
    plane_a, plane_b = (rows + 1) * sa, (rows + 1) * sb
    npl = info["npl"]
    lb = 0 if same else npl * plane_a
    return dict(tr=tr, tc=tc, tn=tn, same=same, ja=(ja_lo, ja_hi), jb=(jb_lo, jb_hi), rows=rows,
                sa=sa, sb=sb, plane_a=plane_a, plane_b=plane_b, lb=lb,
                lds_words=npl * plane_a + (0 if same else npl * plane_b))


def _lane_rows(k_first, count, P, PQ, jlo, s, rows):
    """LDS offset of X row k at position 0 of staged row 0, and its per-row step."""
    k = k_first + np.arange(count)
    valid = k < PQ
    base = np.where(valid, (k % P) * s + (k // P - jlo), rows * s)
    step = np.where(valid, s, 0)
    return k, valid, base, step


def model(A, P, Q, prec, n_cu, check_only=False):
    N, M = A.shape
    PQ, Kr, Kc = P * Q, N - P + 1, M - Q + 1
    info, items, tiles, index = cv.hankel_plan(N, M, P, Q, prec, n_cu)
    npl, ldp = info["npl"], info["ldp"]
    assert info["lds"] <= 160 * 1024
    assert info["planes_bytes"] >= npl * N * ldp * 4
    assert info["ws_bytes"] >= info["planes_bytes"] + len(items) * 128 * info["tn"] * 8
    # padded plane (one complex plane stands for every packed plane: same layout)
    plane = np.zeros((N, ldp), dtype=np.complex128)
    plane[:, :M] = A
    # every upper tile once; each item belongs to exactly one tile
    seen = np.zeros(len(items), dtype=np.int64)
    for t in tiles:
        seen[index[t[2]:t[3]]] += 1
    assert np.all(seen == 1)
    # items of a tile cover every position exactly once
    for t in tiles:
        cover = np.zeros((Kr, Kc), dtype=np.int64)
        for i in index[t[2]:t[3]]:
            it = items[i]
            assert it[0] == t[0] and it[1] == t[1]
            assert 0 <= it[2] < it[3] <= Kr and 0 <= it[4] < it[5] <= Kc
            limit = 32768 if prec in ("bf16", "fp16") else 16384
            assert (it[3] - it[2]) * (it[5] - it[4]) <= limit or (it[3] - it[2]) == 1
            cover[it[2]:it[3], it[4]:it[5]] += 1
        assert np.all(cover == 1)
    partial = {}
    for n_item, it in enumerate(items):
        g = _geometry(info, it, P, Q, PQ)
        assert g["lds_words"] * 4 <= info["lds"]
        rows, sa, sb = g["rows"], g["sa"], g["sb"]
        lds = np.full(g["lds_words"] if not check_only else 1, np.nan + 0j)
        # zero rows
        lds[rows * sa:(rows + 1) * sa] = 0
        if not g["same"] and not check_only:
            lds[g["lb"] + rows * sb:g["lb"] + (rows + 1) * sb] = 0
        kA, vA, baseA, stepA = _lane_rows(g["tr"], 128, P, PQ, g["ja"][0], sa, rows)
        kB, vB, baseB, stepB = _lane_rows(g["tc"], g["tn"], P, PQ, g["jb"][0], sb, rows)
        acc = np.zeros((128, g["tn"]), dtype=np.complex128)
        p0, p1, q0, q1 = (int(x) for x in it[2:])
        for ps in range(p0, p1, info["pb"]):
            n_p = min(p1, ps + info["pb"]) - ps
            nrows = n_p + P - 1
            for qs in range(q0, q1, info["qb"]):
                cw = min(q1, qs + info["qb"]) - qs
                steps = (cw + 7) // 8
                for side in (0, 1):
                    if side == 1 and g["same"]:
                        break
                    jlo, jhi = g["jb"] if side else g["ja"]
                    s = sb if side else sa
                    off0 = g["lb"] if side else 0
                    width = cw + jhi - jlo
                    assert width <= s - 16, (width, s)
                    assert nrows <= rows
                    # rows read from the planes stay inside A's rows; chunk reads inside the padded row
                    assert ps + nrows - 1 <= N - 1
                    chunks = (width + 63) // 64
                    assert chunks <= 5
                    assert qs + jlo + 64 * chunks - 1 < ldp, (qs, jlo, chunks, ldp)
                    if not check_only:
                        for rr in range(nrows):
                            lds[off0 + rr * s:off0 + rr * s + width] = plane[ps + rr, qs + jlo:qs + jlo + width]
                if check_only:
                    # only the address extremes
                    for base, step, s, off0 in ((baseA, stepA, sa, 0), (baseB, stepB, sb, g["lb"])):
                        # the last step's early read of a next step, 8 words past the last step
                        hi = off0 + base + (n_p - 1) * step + 8 * steps + 7
                        assert hi.max() + (npl - 1) * (g["plane_b"] if off0 else g["plane_a"]) < off0 + npl * (
                            g["plane_b"] if off0 else g["plane_a"])
                    continue
                # one step more than the sub-block has: the early read of a next
                # step (never used) must stay in bounds too
                pos = np.arange(8 * steps + 8)
                live = pos < cw
                for pr in range(n_p):
                    offA = baseA[:, None] + pr * stepA[:, None] + pos[None, :]
                    offB = g["lb"] + baseB[:, None] + pr * stepB[:, None] + pos[None, :]
                    for off, pl in ((offA, g["plane_a"]), (offB - g["lb"], g["plane_b"])):
                        assert off.min() >= 0 and off.max() + (npl - 1) * pl < npl * pl
                    XA = np.where(live[None, :], lds[offA], 0)
                    XB = np.where(live[None, :], lds[offB], 0)
                    assert not np.isnan(XA).any() and not np.isnan(XB).any(), "unstaged LDS word read"
                    acc += XA @ XB.conj().T
        partial[n_item] = acc
    if check_only:
        return None
    R = np.zeros((PQ, PQ), dtype=np.complex128)
    for t in tiles:
        tile = sum(partial[i] for i in index[t[2]:t[3]])
        tr, tc = int(t[0]), int(t[1])
        for r in range(128):
            k1 = tr + r
            if k1 >= PQ:
                break
            for c in range(info["tn"]):
                k2 = tc + c
                if k2 >= PQ:
                    break
                if k2 >= k1:
                    R[k1, k2] = tile[r, c]
    iu = np.triu_indices(PQ, 1)
    R[(iu[1], iu[0])] = R[iu].conj()
    return R


SHAPES = [(5, 7, 5, 7), (9, 4, 3, 4), (33, 17, 1, 16), (17, 33, 16, 1), (40, 33, 4, 16),
          (97, 131, 12, 4), (64, 64, 8, 8), (70, 66, 33, 2), (1, 1, 1, 1), (30, 200, 24, 24),
          (20, 300, 9, 11)]


@pytest.mark.parametrize("prec", PRECS)
@pytest.mark.parametrize("shape", SHAPES, ids=lambda s: "x".join(map(str, s)))
def test_model_matches_oracle(oracle_mod, shape, prec):
    N, M, P, Q = shape
    A = synth.small_int(N, M, seed=N * 11 + M + P * 3 + Q)
    R = model(A.astype(np.complex128), P, Q, prec, n_cu=4)
    ref = oracle_mod.forward(A, P, Q, normalize=False)
    assert np.array_equal(R, ref)


@pytest.mark.parametrize("prec", PRECS)
def test_model_many_items(oracle_mod, prec):
    """The full device count: many items per tile, split along position rows."""
    A = synth.small_int(48, 70, seed=5)
    R = model(A.astype(np.complex128), 6, 7, prec, n_cu=256)
    assert np.array_equal(R, oracle_mod.forward(A, 6, 7, normalize=False))


@pytest.mark.parametrize("prec", PRECS)
@pytest.mark.parametrize("shape", [(1024, 1024, 32, 32), (256, 256, 16, 16), (512, 512, 64, 64),
                                   (600, 700, 64, 3), (40, 20000, 4, 64), (33, 17000, 32, 5),
                                   (20, 40000, 3, 7)],
                         ids=lambda s: "x".join(map(str, s)))
def test_address_bounds_large(shape, prec):
    """Every item of the large plans (the headline size among them, and rows
    longer than one item's positions): staging, LDS and plane addresses stay
    inside their buffers."""
    N, M, P, Q = shape
    A = np.zeros((N, M), dtype=np.complex128)
    model(A, P, Q, prec, n_cu=256, check_only=True)
