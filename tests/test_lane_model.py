"""CPU model of the lane engine (one lane per unique combination), no GPU.

`covest_lane_plan_get` gives the plan the library launches: second-factor
rings of `ring` rows with a row stride of `gstride` elements,
chunks of `chunk` row steps, `chain` inputs per workgroup along a grid
column.  The model replays `lane_main` with that plan -- the staging of rows
into the rings (which ring slot holds which row of the chain at every row
step), the first and second factors each lane reads, the window sums over the
column offsets, the box that slides down the chain, and the entries each lane
writes (with their conjugates below the diagonal) -- and

* checks that every ring slot a lane reads holds the row it wants (a stale
  or not yet staged row would fail), that every LDS index stays inside the
  launch's buffers, and that the LDS bytes match the plan;
* checks that every entry of every input's R is written exactly once (upper
  triangle; the mirror once more for the full fill);
* compares R with the oracle (eq. 2.2) bit for bit on small-integer inputs,
  where every sum is exact whatever its order.
"""
import numpy as np
import pytest

from paper_1303_2285_amd import covest as cv
from paper_1303_2285_amd import synth


def _lags(P, Q, n_lags, threads):
    """(dr, dc, live) per thread: dr = 0 with dc in [0, Q), then dr >= 1 with dc in (-Q, Q)."""
    out = []
    for t in range(threads):
        if t >= n_lags:
            out.append((0, 0, False))
        elif t < Q:
            out.append((0, t, True))
        else:
            u = t - Q
            out.append((1 + u // (2 * Q - 1), u % (2 * Q - 1) - (Q - 1), True))
    return out


def model(img, N, M, P, Q, rs, cs, n_rows, n_cols, chain=None, fill_full=True, check_only=False):
    info = cv.lane_plan(N, M, P, Q, rs, n_rows, n_cols)
    assert info["fits"] == 1
    if chain is not None:
        info["chain"] = min(chain, n_rows)
    ring, gstride, CH, L0 = info["ring"], info["gstride"], info["chunk"], info["chain"]
    PQ, Kr, Kc = P * Q, N - P + 1, M - Q + 1
    n_lags = PQ + (P - 1) * (Q - 1)
    threads = -(-n_lags // 64) * 64
    assert info["threads"] == threads
    # LDS: two rings of complex64 second-factor rows, two chunks of FP64 first-factor rows
    assert info["lds"] == 2 * ring * gstride * 8 + 2 * CH * M * 16
    assert gstride >= M + 2 * Q - 2 and ring == CH + P - 1
    lags = _lags(P, Q, n_lags, threads)
    R = np.zeros((n_rows, n_cols, PQ, PQ), dtype=np.complex128)
    writes = np.zeros((n_rows, n_cols, PQ, PQ), dtype=np.int64)
    n_chains = -(-n_rows // L0)
    assert info["n_blocks"] == n_chains * n_cols or chain is not None
    for wg in range(n_chains * n_cols):
        b, a0 = wg % n_cols, (wg // n_cols) * L0
        L = min(L0, n_rows - a0)
        rows_walk = (L - 1) * rs + N
        r0, c0 = a0 * rs, b * cs
        # the chain's rows, zero below; Q-1 zero columns on each side
        padded = np.zeros((rows_walk + 2 * P + CH, M + 2 * Q - 2), dtype=np.complex128)
        if not check_only:
            padded[:rows_walk, Q - 1:Q - 1 + M] = img[r0:r0 + rows_walk, c0:c0 + M]
        ring_row = {"i": [-1] * ring, "o": [-1] * ring}
        nxt = {"i": 0, "o": 0}

        def stage(which, lo, hi, oldest_needed):
            assert hi - lo <= ring
            for r in range(lo, hi):
                slot = r % ring
                prev = ring_row[which][slot]
                assert prev < oldest_needed, "a ring row still in use is overwritten"
                ring_row[which][slot] = r

        def walk(B, ring_in, s, slide):
            """one row step of every lane: ring checks, then the window sums"""
            for t, (dr, dc, live) in enumerate(lags):
                gs = s % ring + dr
                gs -= ring if gs >= ring else 0
                assert 0 <= gs < ring and ring_row[ring_in][gs] == s + dr
                assert 0 <= dc + Q - 1 and dc + Q - 1 + M - 1 < gstride
                if slide:
                    go = (s - Kr) % ring + dr
                    go -= ring if go >= ring else 0
                    assert ring_row["o"][go] == s - Kr + dr
                if check_only:
                    continue
                z = padded[s, Q - 1:Q - 1 + M] * np.conj(padded[s + dr, Q - 1 + dc:Q - 1 + dc + M])
                if slide:
                    z = z - padded[s - Kr, Q - 1:Q - 1 + M] * np.conj(
                        padded[s - Kr + dr, Q - 1 + dc:Q - 1 + dc + M])
                c = np.concatenate([[0], np.cumsum(z)])
                B[t] += c[Kc:Kc + Q] - c[0:Q]

        def emit(B, tt):
            q_lo = (tt - P + rs) // rs if tt >= P else 0
            q_hi = min(L - 1, tt // rs)
            for q in range(q_lo, q_hi + 1):
                i1 = tt - q * rs
                assert 0 <= i1 < P
                for t, (dr, dc, live) in enumerate(lags):
                    if not live or i1 >= P - dr:
                        continue
                    for e in range(max(0, -dc), Q - max(0, dc)):
                        k1, k2 = i1 + P * e, i1 + dr + P * (e + dc)
                        v = B[t, e]
                        if dr == 0 and dc == 0:
                            v = complex(v.real, 0.0)
                        u1, u2 = (k2, k1) if k1 > k2 else (k1, k2)
                        vu = np.conj(v) if k1 > k2 else v
                        R[a0 + q, b, u1, u2] = vu
                        writes[a0 + q, b, u1, u2] += 1
                        if fill_full and u1 != u2:
                            R[a0 + q, b, u2, u1] = np.conj(vu)
                            writes[a0 + q, b, u2, u1] += 1

        def seed(B, which, frm, to):
            for s0 in range(frm, to, CH):
                s1 = min(to, s0 + CH)
                stage(which, nxt[which], s1 + P - 1, s0)
                nxt[which] = s1 + P - 1
                for s in range(s0, s1):
                    walk(B, which, s, False)

        B = np.zeros((threads, Q), dtype=np.complex128)
        seed(B, "i", 0, Kr)
        emit(B, 0)
        for s0 in range(Kr, rows_walk, CH):
            s1 = min(rows_walk, s0 + CH)
            stage("i", nxt["i"], s1 + P - 1, s0)
            nxt["i"] = s1 + P - 1
            stage("o", max(nxt["o"], s0 - Kr), s1 - Kr + P - 1, s0 - Kr)
            nxt["o"] = s1 - Kr + P - 1
            for s in range(s0, s1):
                walk(B, "i", s, True)
                emit(B, s - (Kr - 1))
    iu = np.triu_indices(PQ)
    assert np.all(writes[:, :, iu[0], iu[1]] == 1), "an upper-triangle entry is not written exactly once"
    if fill_full:
        assert np.all(writes == 1)
    return R


GRIDS = [
    # N, M, P, Q, row_step, col_step, n_rows, n_cols, chain
    (12, 11, 3, 4, 5, 4, 3, 2, 1),
    (12, 11, 3, 4, 5, 4, 3, 2, 3),      # chained: slides through the gaps
    (9, 9, 4, 3, 2, 3, 4, 2, 4),        # row step below P: box starts shared by two inputs
    (10, 7, 1, 1, 3, 2, 3, 3, 2),
    (8, 13, 8, 5, 1, 3, 3, 2, 3),       # one box row per input, step 1
    (16, 16, 5, 5, 6, 7, 3, 2, 2),
    (6, 20, 2, 16, 2, 1, 4, 1, 4),      # Q = 16 (the widest register array)
    (14, 9, 6, 9, 4, 1, 2, 1, 2),       # Q = M: one column offset box per row
]


@pytest.mark.parametrize("grid", GRIDS, ids=lambda g: "x".join(map(str, g)))
@pytest.mark.parametrize("fill", ["full", "upper"])
def test_model_matches_oracle(oracle_mod, grid, fill):
    N, M, P, Q, rs, cs, nr, nc, chain = grid
    H, W = (nr - 1) * rs + N + 2, (nc - 1) * cs + M + 1   # spare rows and columns the walk must not read
    img = synth.small_int(H, W, seed=H * 7 + W + P + Q).astype(np.complex128)
    R = model(img, N, M, P, Q, rs, cs, nr, nc, chain=chain, fill_full=(fill == "full"))
    for a in range(nr):
        for b in range(nc):
            ap = img[a * rs:a * rs + N, b * cs:b * cs + M].astype(np.complex64)
            ref = oracle_mod.forward(ap, P, Q, normalize=False)
            if fill == "upper":
                ref = np.triu(ref)
            assert np.array_equal(R[a, b], ref), (a, b)


@pytest.mark.parametrize("grid", [(100, 100, 10, 10, 62, 62, 25, 25, None),
                                  (100, 100, 10, 10, 16, 16, 94, 94, None),
                                  (100, 100, 10, 10, 16, 16, 21, 21, 21),
                                  (64, 96, 16, 16, 8, 8, 3, 1, 3),
                                  (40, 30, 13, 13, 3, 3, 9, 1, 9)],
                         ids=lambda g: "x".join(map(str, g)))
def test_ring_bookkeeping_large(grid):
    """The aperture grids of the measured workloads (and long chains): every
    ring slot a lane reads holds its row, and every entry is written once."""
    N, M, P, Q, rs, cs, nr, nc, chain = grid
    if chain is None:
        chain = cv.lane_plan(N, M, P, Q, rs, nr, nc)["chain"]
    # one grid column: every column has the same schedule
    model(None, N, M, P, Q, rs, cs, nr, 1, chain=chain, check_only=True)


def test_plan_choices():
    """Chains only where sliding through the gap is cheaper than a new box,
    and only as long as the grid keeps four workgroups per compute unit."""
    p = cv.lane_plan(100, 100, 10, 10, 62, 25, 25)
    assert p["chain"] == 1 and p["n_blocks"] == 625 and p["threads"] == 192
    p = cv.lane_plan(100, 100, 10, 10, 16, 94, 94)
    assert p["chain"] == 8 and p["n_blocks"] == 94 * 12
    p = cv.lane_plan(100, 100, 10, 10, 16, 21, 21)      # 441 apertures: too few to chain
    assert p["chain"] == 1
    assert cv.lane_plan(20, 200, 2, 17)["fits"] == 0     # Q above the register array
    assert cv.lane_plan(40, 40, 22, 16)["fits"] == 0     # more lags than one workgroup's lanes
    assert cv.lane_plan(40, 1000, 10, 10)["fits"] == 0   # rows too long for the LDS
