// plan.cpp -- host planning for the recurrence kernels.
#include "plan.hpp"

#include <algorithm>
#include <cmath>
#include <cstdlib>

namespace covest {

Counts method_counts(int64_t N, int64_t M, int64_t P, int64_t Q)
{
    Counts c{};
    c.K = (N - P + 1) * (M - Q + 1);
    c.n_uc = P * Q + (P - 1) * (Q - 1);
    c.eta = P * Q * (P * Q + 1) / 2;
    int64_t um = 0, seg = 0;
    for (int64_t dc = 0; dc < Q; ++dc) {
        for (int64_t dr = (dc == 0 ? 0 : -(P - 1)); dr < P; ++dr) {
            um += (N - std::llabs(dr)) * (M - dc);
            seg += Q - dc;
        }
    }
    c.um = um;
    c.segments = seg;
    return c;
}

static int ring_width(int n)
{
    if (n <= 4) return 4;
    if (n <= 8) return 8;
    if (n <= 12) return 12;
    return 16;
}

// Lanes (d1, chunk) for d1 in [d1lo, d1hi) and d2 chunks covering [v2lo, v2hi)
// from ch0, split so that a group has at most 64 lanes.
static void add_groups(std::vector<LagGroup> &gs, int orient, int W, int d1lo, int d1hi, int ch0,
                       int v2lo, int v2hi, std::vector<int> &ids)
{
    if (d1hi <= d1lo || v2hi <= v2lo) return;
    const int nch = (v2hi - ch0 + W - 1) / W;
    const int per = std::max(1, 64 / nch);
    const int nd1 = d1hi - d1lo;
    const int ngroups = (nd1 + per - 1) / per;
    // balance the d1 ranges of the groups
    for (int k = 0; k < ngroups; ++k) {
        LagGroup g{};
        g.orient = orient;
        g.W = W;
        g.d1lo = d1lo + (int)((int64_t)k * nd1 / ngroups);
        g.d1hi = d1lo + (int)((int64_t)(k + 1) * nd1 / ngroups);
        g.ch0 = ch0;
        g.nch = nch;
        g.v2lo = v2lo;
        g.v2hi = v2hi;
        g.lanes = (g.d1hi - g.d1lo) * nch;
        g.slots = 64 / g.lanes;
        g.hr_lo = std::min(0, g.d1lo);
        g.hr_hi = std::max(0, g.d1hi - 1);
        g.hc_lo = std::min(0, ch0);
        g.hc_hi = std::max(0, ch0 + nch * W - 1);
        ids.push_back((int)gs.size());
        gs.push_back(g);
    }
}

static size_t tile_bytes(int rows, int cols) { return (size_t)rows * (size_t)(cols | 1) * 16; }

std::vector<int> ring_width_candidates(int n)
{
    const int d = ring_width(n);
    std::vector<int> c{d};
    for (int w : {8, 12, 4})
        if (w < d && (w >= 8 || n <= 8)) c.push_back(w);
    return c;
}

// Finalize items (every unique combination, eq. 3.3, in lag-index order,
// dr-major, so that neighbouring items read neighbouring partial sums), the
// finalize variant, the workspace size and the product counts.
template <class BulkRange>
static void finish_plan(ShapePlan &sp, BulkRange bulk_range)
{
    const int N = sp.N, M = sp.M, P = sp.P, Q = sp.Q;
    for (int dr = -(P - 1); dr < P; ++dr) {
        for (int dc = (dr < 0 ? 1 : 0); dc < Q; ++dc) {
            FinItem it{};
            it.inst = 0;
            it.dr = dr;
            it.dc = dc;
            it.bulk0 = it.bulk1 = 0;
            bulk_range(dr, dc, it);
            sp.items.push_back(it);
        }
    }
    const size_t table = (size_t)(1 + sp.n_ir) * (sp.n_ic | 1) * 16;
    const bool fin_table = table <= kFinTableMax && sp.n_ir <= kFinMaxRows;
    sp.fin_variant = !fin_table ? kFinLean : sp.n_ir * sp.n_ic <= kFinSmallCorners ? kFinTableSmall : kFinTable;
    sp.lds_fin = fin_table ? table : (size_t)(1 + sp.n_ir) * Q * 16;
    // wave prefix sums: an individual column per lane in the row pass, an
    // individual row per lane in the column pass; LDS holds the classes'
    // sums per column offset.  Its cost per combination only pays for large
    // corner tables (measured: 55 -> 50 us at 1024^2 / 32 x 32, 62 x 62
    // corners; tables of up to ~45 x 45, as in a batch of 4..16 windows, run
    // slower than with the table variants)
    if (sp.n_ic <= 63 && sp.n_ir <= 63 && sp.n_ir * sp.n_ic > 2 * kFinSmallCorners) {
        sp.fin_variant = kFinScan;
        sp.lds_fin = (size_t)Q * ((1 + sp.n_ir) | 1) * 16;
    }
    if (sp.n_ic <= 63 && sp.n_ir <= 31) {
        sp.fin_variant = kFinScanSmall;
        sp.lds_fin = (size_t)Q * ((1 + sp.n_ir) | 1) * 16;
    }

    sp.ws_bytes = (size_t)16 * sp.lag_stride *
                  ((size_t)sp.n_bulk + (size_t)sp.zpieces * ((size_t)sp.n_ir + (size_t)sp.n_ic));

    // Product counts (for throughput figures): the finalize computes the
    // corner products (individual row and individual column) of every lag, the
    // main kernel all the others.
    const Counts cnt = method_counts(N, M, P, Q);
    int64_t corner = 0;
    for (int dc = 0; dc < Q; ++dc) {
        for (int dr = (dc == 0 ? 0 : -(P - 1)); dr < P; ++dr) {
            const int rlo = std::max(0, -dr), rhi = N - std::max(0, dr);
            const int chi = M - dc;
            int64_t rows = 0, cols = 0;
            for (int r = rlo; r < rhi; ++r) rows += (r < sp.Rm0 || r >= sp.Rm1) ? 1 : 0;
            for (int c = 0; c < chi; ++c) cols += (c < sp.Cm0 || c >= sp.Cm1) ? 1 : 0;
            corner += rows * cols;
        }
    }
    sp.fin_products = corner;
    sp.main_products = cnt.um - corner;
}

ShapePlan make_shape_plan(int N, int M, int P, int Q, int n_slots, int w0, int w1)
{
    ShapePlan sp;
    sp.N = N;
    sp.M = M;
    sp.P = P;
    sp.Q = Q;
    sp.W0 = w0 > 0 ? w0 : ring_width(Q);
    sp.W1 = w1 > 0 ? w1 : ring_width(P);
    sp.lag_stride = (2 * P - 1) * Q;
    sp.bandw = kWaves * sp.W0;

    // Middle rows: walked by column strips in blocks of W1.
    sp.Rm0 = P - 1;
    const int lenR = N - 2 * P + 2;
    sp.Rm1 = sp.Rm0 + (lenR >= sp.W1 ? (lenR / sp.W1) * sp.W1 : 0);
    // Middle columns: bulk bands of kWaves * W0.
    sp.Cm0 = Q - 1;
    const int lenC = M - 2 * Q + 2;
    sp.Cm1 = sp.Cm0 + (lenC >= sp.bandw ? (lenC / sp.bandw) * sp.bandw : 0);
    const int nMr = sp.Rm1 - sp.Rm0, nMc = sp.Cm1 - sp.Cm0;
    sp.n_ir = N - nMr;
    sp.n_ic = M - nMc;

    // Lag groups.  Orientation 0 walks A's columns (ring over dc); orientation 1
    // walks A's rows on the transposed tile (ring over dr).
    std::vector<int> g0, g1;
    add_groups(sp.groups, 0, sp.W0, 0, P, 0, 0, Q, g0);                  // type A
    if (P > 1 && Q > 1) add_groups(sp.groups, 0, sp.W0, -(P - 1), 0, 1, 1, Q, g0);  // type B
    add_groups(sp.groups, 1, sp.W1, 0, Q, 0, 0, P, g1);                  // type A
    if (P > 1 && Q > 1) add_groups(sp.groups, 1, sp.W1, 1, Q, -(P - 1), -(P - 1), 0, g1);  // type B
    sp.slots0 = sp.groups.empty() ? 1 : sp.groups[g0.front()].slots;

    // --- job costs in wave-steps (one ring column of W complex MACs) -------
    struct Strip { int group, x0, x1, c0, c1, out; double cost; };
    std::vector<Strip> strips;
    auto add_strips = [&](int gid, int lo, int hi, int out_base, int c0, int c1) {
        const LagGroup &g = sp.groups[gid];
        const int per = kWaves * g.slots;
        for (int x = lo; x < hi; x += per) {
            const int x1 = std::min(hi, x + per);
            strips.push_back({gid, x, x1, c0, c1, out_base + (x - lo), (double)(c1 - c0) * g.W});
        }
    };
    if (nMc > 0) {   // row strips: individual rows x middle columns
        for (int gid : g0) {
            add_strips(gid, 0, sp.Rm0, 0, sp.Cm0, sp.Cm1);
            add_strips(gid, sp.Rm1, N, sp.Rm0, sp.Cm0, sp.Cm1);
        }
    }
    if (nMr > 0) {   // column strips: individual columns x middle rows (B rows = A cols)
        for (int gid : g1) {
            add_strips(gid, 0, sp.Cm0, 0, sp.Rm0, sp.Rm1);
            add_strips(gid, sp.Cm1, M, sp.Cm0, sp.Rm0, sp.Rm1);
        }
    }
    double strip_total = 0.0, strip_max = 0.0;
    for (const Strip &s : strips) {
        strip_total += s.cost;
        strip_max = std::max(strip_max, s.cost);
    }

    // Bulk units per orientation-0 group.
    std::vector<int64_t> units(g0.size(), 0);
    int64_t units_total = 0;
    if (nMr > 0 && nMc > 0) {
        for (size_t k = 0; k < g0.size(); ++k) {
            const int S = sp.groups[g0[k]].slots;
            units[k] = (int64_t)((nMr + S - 1) / S) * (nMc / sp.bandw);
            units_total += units[k];
        }
    }
    const double unit_cost = (double)sp.W0 * sp.W0;
    const double bulk_total = (double)units_total * unit_cost;

    int n_bulk = 0;
    if (units_total > 0) {
        const int n_strips = (int)strips.size();
        const double ideal = (bulk_total + strip_total) / std::max(1, n_slots);
        const double min_job = 32.0 * unit_cost;   // keep tiny problems to few jobs
        double target;
        if (strip_max <= ideal && n_strips < n_slots) {
            n_bulk = n_slots - n_strips;
            target = bulk_total / n_bulk;
        } else {
            target = std::max(strip_max, ideal);
            n_bulk = (int)std::ceil(bulk_total / target);
        }
        if (target < min_job) n_bulk = (int)std::ceil(bulk_total / min_job);
        n_bulk = (int)std::max<int64_t>(1, std::min<int64_t>(n_bulk, units_total));
    }

    // Split n_bulk over the groups in proportion to their units.
    std::vector<int> njob(g0.size(), 0);
    if (n_bulk > 0) {
        int assigned = 0;
        for (size_t k = 0; k < g0.size(); ++k) {
            if (units[k] == 0) continue;
            njob[k] = std::max<int>(1, (int)std::llround((double)n_bulk * units[k] / units_total));
            njob[k] = (int)std::min<int64_t>(njob[k], units[k]);
            assigned += njob[k];
        }
        (void)assigned;
    }

    // Bulk jobs, groups interleaved so that neighbouring jobs cover the same
    // region of A.
    std::vector<int> out_base(g0.size(), 0);
    int outs = 0;
    for (size_t k = 0; k < g0.size(); ++k) {
        out_base[k] = outs;
        outs += njob[k];
    }
    sp.n_bulk = outs;
    int max_njob = 0;
    for (int v : njob) max_njob = std::max(max_njob, v);
    for (int j = 0; j < max_njob; ++j) {
        for (size_t k = 0; k < g0.size(); ++k) {
            if (j >= njob[k]) continue;
            const LagGroup &g = sp.groups[g0[k]];
            Job jb{};
            jb.mode = kJobBulk;
            jb.inst = 0;
            jb.group = g0[k];
            jb.out = out_base[k] + j;
            jb.u0 = (int)((int64_t)j * units[k] / njob[k]);
            jb.u1 = (int)((int64_t)(j + 1) * units[k] / njob[k]);
            // rows per LDS sub-tile: a multiple of the slot count
            const int S = g.slots;
            const int cols = sp.bandw + g.hc_hi - g.hc_lo;
            const int halo = g.hr_hi - g.hr_lo;
            int tr = S;
            while (tr + S <= std::max(S, 64) && tile_bytes(tr + S + halo, cols) <= kLdsBudget) tr += S;
            jb.tile_rows = tr;
            sp.jobs.push_back(jb);
            sp.job_cost.push_back((double)(jb.u1 - jb.u0) * unit_cost);
            sp.lds_main = std::max(sp.lds_main, tile_bytes(tr + halo, cols));
            sp.lds_main = std::max(sp.lds_main, (size_t)kThreads * g.W * 16);
        }
    }
    for (const Strip &s : strips) {
        const LagGroup &g = sp.groups[s.group];
        Job jb{};
        jb.mode = kJobStrip;
        jb.inst = 0;
        jb.group = s.group;
        jb.out = s.out;
        jb.x0 = s.x0;
        jb.x1 = s.x1;
        jb.c0 = s.c0;
        jb.c1 = s.c1;
        const int rows = (s.x1 - s.x0) + g.hr_hi - g.hr_lo;
        const int halo_c = g.hc_hi - g.hc_lo;
        int tc = g.W;
        while (tc + g.W <= (s.c1 - s.c0) && tile_bytes(rows, tc + g.W + halo_c) <= kLdsBudget) tc += g.W;
        jb.tile_cols = tc;
        sp.jobs.push_back(jb);
        sp.job_cost.push_back(s.cost);
        sp.lds_main = std::max(sp.lds_main, tile_bytes(rows, tc + halo_c));
    }

    finish_plan(sp, [&](int dr, int dc, FinItem &it) {
        for (size_t k = 0; k < g0.size(); ++k) {
            const LagGroup &g = sp.groups[g0[k]];
            const bool in_type = (dr >= 0) == (g.d1lo >= 0);
            if (in_type && dr >= g.d1lo && dr < g.d1hi && njob[k] > 0) {
                it.bulk0 = out_base[k];
                it.bulk1 = out_base[k] + njob[k];
            }
        }
    });
    return sp;
}


bool mfma_fits(int N, int M, int P, int Q, double min_fill)
{
    if (N - 2 * P + 2 < 1 || M - 2 * Q + 2 < 1 || Q < 4) return false;
    const int mt = (2 * P - 1 + 15) / 16, nt = (Q + 15) / 16;
    if (mt * nt > 8) return false;
    return (double)(2 * P - 1) * Q >= min_fill * 256.0 * mt * nt;
}

bool mfma_preferred(int N, int M, int P, int Q, bool batch)
{
    if (!mfma_fits(N, M, P, Q)) return false;
    const int tiles = ((2 * P - 1 + 15) / 16) * ((Q + 15) / 16);
    const double fill = (double)(2 * P - 1) * Q / (256.0 * tiles);
    if (batch) return fill >= 0.7;
    return !(fill < 0.3 && tiles >= 7);
}

// K-groups of 4 positions, the first at k0, that lie wholly inside a line of
// npos positions (at most nkg).  Written with a guard, not as one truncating
// division: for npos - k0 < 4 the count is 0, not 1.
static int kgroups_inside(int npos, int k0, int nkg)
{
    if (npos - k0 < 4) return 0;
    return std::min(nkg, (npos - k0 - 4) / 4 + 1);
}

ShapePlan make_mfma_plan(int N, int M, int P, int Q, int n_cu, double job_units)
{
    ShapePlan sp;
    sp.engine = 2;
    sp.N = N;
    sp.M = M;
    sp.P = P;
    sp.Q = Q;
    sp.mt = (2 * P - 1 + 15) / 16;
    sp.nt = (Q + 15) / 16;
    sp.lag_stride = (2 * P - 1) * Q;
    sp.Rm0 = P - 1;
    sp.Rm1 = N - P + 1;
    sp.Cm0 = Q - 1;
    sp.Cm1 = M - Q + 1;
    sp.n_ir = N - (sp.Rm1 - sp.Rm0);
    sp.n_ic = M - (sp.Cm1 - sp.Cm0);
    n_cu = std::max(1, n_cu);

    // Positions a line walks: orientation 0 (rows) has first-factor columns
    // [Cm0, Cm1) and lags dc in [0, Q); orientation 1 (columns) has first-factor
    // rows [Rm0, Rm1) and lags dr in (-P, P).
    const int nkg[2] = {(sp.Cm1 - sp.Cm0 + Q - 1 + 3) / 4, (sp.Rm1 - sp.Rm0 + 2 * (P - 1) + 3) / 4};
    const int plo[2] = {sp.Cm0, sp.Rm0}, phi[2] = {sp.Cm1, sp.Rm1};
    // Orientation 0 ends its k-groups at the last column of A (it reads its
    // first operand unchecked), starting up to 3 positions before Cm0: those
    // positions only meet first factors outside [Cm0, Cm1), which are zero.
    const int k0[2] = {sp.Cm1 + Q - 1 - 4 * nkg[0], sp.Rm0 - (P - 1)};

    struct StripBlock { int orient, line0, line_end, zrow0; };
    std::vector<StripBlock> sbs;
    auto add_side = [&](int orient, int lo, int hi, int zbase) {
        for (int l = lo; l < hi; l += kMWaves) sbs.push_back({orient, l, std::min(hi, l + kMWaves), zbase + (l - lo)});
    };
    add_side(0, 0, sp.Rm0, 0);
    add_side(0, sp.Rm1, N, sp.Rm0);
    add_side(1, 0, sp.Cm0, 0);
    add_side(1, sp.Cm1, M, sp.Cm0);

    const int nblk = (sp.Rm1 - sp.Rm0 + kMWaves - 1) / kMWaves;
    const int64_t U = (int64_t)nblk * nkg[0];
    double strip_total = 0.0;
    int strip_len = 0, strip_min = 1 << 30;
    for (const StripBlock &b : sbs) {
        strip_total += nkg[b.orient];
        strip_len = std::max(strip_len, nkg[b.orient]);
        strip_min = std::min(strip_min, nkg[b.orient]);
    }
    const double ideal = job_units > 0.0 ? job_units : ((double)U + strip_total) / n_cu;
    // pieces per strip line: a piece no longer than a balanced share, and no
    // piece empty (the finalize adds every piece's row, so each is written)
    sp.zpieces = 1;
    if (strip_len > 0) {
        const double want = std::ceil(strip_len / ideal - 1e-9);
        sp.zpieces = (int)std::max(1.0, std::min({8.0, want, (double)strip_min}));
    }

    int smax = 0;
    std::vector<MJob> strips;
    for (const StripBlock &b : sbs) {
        const int o = b.orient, nk = nkg[o];
        for (int p = 0; p < sp.zpieces; ++p) {
            MJob j{};
            j.orient = o;
            j.kind = kMStrip;
            j.out = p * (o ? sp.n_ic : sp.n_ir) + b.zrow0;
            j.line0 = b.line0;
            j.line_end = b.line_end;
            j.b0 = j.b1 = 0;
            j.kg0 = (int)((int64_t)nk * p / sp.zpieces);
            j.kg1 = (int)((int64_t)nk * (p + 1) / sp.zpieces);
            j.n_kg = nk;
            j.pos_lo = plo[o];
            j.pos_hi = phi[o];
            j.k0 = k0[o];
            j.kin = kgroups_inside(o ? N : M, k0[o], nk);
            strips.push_back(j);
            smax = std::max(smax, j.kg1 - j.kg0);
        }
    }

    const int n_strip = (int)strips.size();
    int n_bulk;
    if (job_units > 0.0) n_bulk = (int)std::ceil((double)U / ideal);
    else if (n_strip < n_cu && smax <= 1.1 * ideal) n_bulk = n_cu - n_strip;
    else n_bulk = (int)std::ceil((double)U / std::max((double)smax, ideal));
    n_bulk = (int)std::max<int64_t>(1, std::min<int64_t>(n_bulk, std::max<int64_t>(1, U / 4)));
    sp.n_bulk = n_bulk;
    for (int j = 0; j < n_bulk; ++j) {
        const int64_t u0 = U * j / n_bulk, u1 = U * (j + 1) / n_bulk;
        MJob b{};
        b.orient = 0;
        b.kind = kMBulk;
        b.out = j;
        b.line0 = sp.Rm0;
        b.line_end = sp.Rm1;
        b.b0 = (int)(u0 / nkg[0]);
        b.kg0 = (int)(u0 % nkg[0]);
        b.b1 = (int)(u1 / nkg[0]);
        b.kg1 = (int)(u1 % nkg[0]);
        b.n_kg = nkg[0];
        b.pos_lo = plo[0];
        b.pos_hi = phi[0];
        b.k0 = k0[0];
        b.kin = kgroups_inside(M, k0[0], nkg[0]);
        sp.mjobs.push_back(b);
        sp.job_cost.push_back((double)(u1 - u0));
    }
    for (const MJob &j : strips) {
        sp.mjobs.push_back(j);
        sp.job_cost.push_back((double)(j.kg1 - j.kg0));
    }
    sp.lds_main = std::max((size_t)4 * 8 * sp.mt * sp.nt * 64 * sizeof(double),
                           (size_t)kMWaves * kMXCap * 8);
    finish_plan(sp, [&](int, int, FinItem &it) {
        it.bulk0 = 0;
        it.bulk1 = sp.n_bulk;
    });
    return sp;
}

}  // namespace covest

namespace covest {

static int planes_of(int prec)
{
    switch (prec) {
    case kPrecF32: return 3;
    case kPrecBF16: case kPrecF16: return 2;
    default: return 4;
    }
}

// Row stride of an LDS window: at least w, and 1 (mod 32) 4-byte elements.
// The kernel reads its operands 4 bytes at a time (a lane's window column can
// start at any element), and the 32 lanes of a half-wave take 32 different
// rows: with an odd stride their words fall in 32 different banks.  (A stride
// of 4 (mod 32) put them in 8 banks, a 4-way conflict that halved the speed
// of the 16-bit forms.)
static int pad_stride(int w) { return w + ((1 - w) % 32 + 32) % 32; }

// LDS row stride of a staged rectangle read by 32 lanes at once: at least w,
// and, among the next 32 values, the one that spreads the lanes of every
// 32-row fragment of the tile rows [k_lo, k_lo + rows) over the most banks
// (lane m reads row k % P, column k / P of the rectangle, k = k_lo + 32f + m).
static int bank_stride(int w, int P, int PQ, int k_lo_step, int rows)
{
    int best = w, best_cost = 1 << 30;
    for (int s = w; s < w + 32; ++s) {
        int cost = 0;
        for (int k0 = 0; k0 < PQ; k0 += 32) {
            const int lo = (k0 / k_lo_step) * k_lo_step;   // first row of the tile holding k0
            int hits[32] = {0};
            int worst = 0;
            for (int m = 0; m < 32 && k0 + m < PQ && k0 + m < lo + rows; ++m) {
                const int k = k0 + m;
                const int b = ((k % P) * s + (k / P - lo / P)) & 31;
                worst = std::max(worst, ++hits[b]);
            }
            cost += worst;
        }
        if (cost < best_cost) {
            best_cost = cost;
            best = s;
        }
    }
    return best;
}

// 16-bit forms (B1-B3): A is split once into packed planes, workgroups own
// 128 x 128 tiles (128 x 64 for FP16x3, whose cross terms keep accumulators of
// their own), each item sums at most item_positions16(prec) positions in FP32.
static HankelPlan make_hankel_plan16(int N, int M, int P, int Q, int prec, int n_cu)
{
    HankelPlan hp;
    hp.N = N; hp.M = M; hp.P = P; hp.Q = Q; hp.prec = prec;
    const int PQ = P * Q, Kr = N - P + 1, Kc = M - Q + 1;
    const bool split = prec == kPrecBF16x3 || prec == kPrecF16x3;
    hp.npl16 = split ? 2 : 1;
    hp.tm = 128;
    hp.tn = prec == kPrecF16x3 ? 64 : 128;
    // output tiles meeting the upper triangle
    std::vector<std::pair<int, int>> tiles;
    for (int tr = 0; tr < PQ; tr += hp.tm)
        for (int tc = 0; tc < PQ; tc += hp.tn)
            if (tc + hp.tn - 1 >= tr) tiles.push_back({tr, tc});
    // widest column window of a tile's rows, per side
    auto span_of = [&](int rows) {
        int span = 0;
        for (int lo = 0; lo < PQ; lo += rows)
            span = std::max(span, std::min(Q - 1, std::min(PQ - 1, lo + rows - 1) / P) - lo / P);
        return span;
    };
    const int span_a = span_of(hp.tm), span_b = span_of(hp.tn);
    // item geometry: rows of positions x a column range, at most
    // item_positions16(prec) positions, and at least ~4 items per workgroup slot
    int rows_item, cols_item;
    const int item_pos = item_positions16(prec);
    if (Kc <= item_pos) {
        // Items of equal rows, one workgroup each, two resident per CU.  The
        // split count S (items per tile) minimises rounds of workgroups times
        // the rows of one item plus a halo allowance (the P - 1 extra rows every
        // staged sub-block reads, worth ~4 rows of compute), so that the last
        // round is not left half empty.
        cols_item = Kc;
        const int rows_max = std::max(1, std::min(Kr, item_pos / Kc));
        const int64_t slots = 2LL * std::max(1, n_cu);
        const int64_t nt = (int64_t)tiles.size();
        const int s_lo = (Kr + rows_max - 1) / rows_max;
        const int s_hi = std::min<int64_t>(Kr, std::max<int64_t>(s_lo, 16 * slots / nt + 1));
        double best_t = 1e300;
        rows_item = rows_max;
        for (int S = s_lo; S <= s_hi; ++S) {
            const int r = (Kr + S - 1) / S;
            const int64_t n = nt * ((Kr + r - 1) / r);
            const double t = (double)((n + slots - 1) / slots) * (r + 4.0);
            if (t < best_t - 1e-9) {
                best_t = t;
                rows_item = r;
            }
        }
    } else {
        rows_item = 1;
        cols_item = item_pos;
    }
    // sub-tile: the most positions per staged word within the LDS budget
    const size_t budget = 76 * 1024;
    double best = -1.0;
    for (int qb : {32, 64, 96, 128, 192, 256}) {
        if (qb > ((cols_item + 7) / 8) * 8 && qb != 32) continue;
        // a row holds the sub-block's columns plus the 16 words that the last
        // step and the next step's early reads may touch past them
        const int s_a = bank_stride(qb + span_a + 16, P, PQ, hp.tm, hp.tm);
        const int s_b = bank_stride(qb + span_b + 16, P, PQ, hp.tn, hp.tn);
        for (int pb = 1; pb <= rows_item; ++pb) {
            const size_t bytes = (size_t)hp.npl16 * (pb + P) * (s_a + s_b) * 4;
            if (bytes > budget) break;
            const double eff = (double)pb * std::min(qb, cols_item) / ((double)(pb + P) * (s_a + s_b));
            if (eff > best) {
                best = eff;
                hp.pb = pb;
                hp.qb = qb;
                hp.stride_a = s_a;
                hp.stride_b = s_b;
                hp.lds = bytes;
            }
        }
    }
    if (hp.pb == 0) {
        hp.pb = 1;
        hp.qb = 32;
        hp.stride_a = bank_stride(32 + span_a + 16, P, PQ, hp.tm, hp.tm);
        hp.stride_b = bank_stride(32 + span_b + 16, P, PQ, hp.tn, hp.tn);
        hp.lds = (size_t)hp.npl16 * (1 + P) * (hp.stride_a + hp.stride_b) * 4;
    }
    // items ordered by position range, then tile: neighbouring items read the
    // same rows of A (the kernel gives each XCD a contiguous range of items)
    std::vector<std::vector<int>> of_tile(tiles.size());
    for (int p0 = 0; p0 < Kr; p0 += rows_item) {
        const int p1 = std::min(Kr, p0 + rows_item);
        for (int q0 = 0; q0 < Kc; q0 += cols_item) {
            const int q1 = std::min(Kc, q0 + cols_item);
            for (size_t t = 0; t < tiles.size(); ++t) {
                of_tile[t].push_back((int)hp.items.size());
                hp.items.push_back({tiles[t].first, tiles[t].second, p0, p1, q0, q1});
            }
        }
    }
    // the reduction reads each tile's items through an index list (item0 .. item1
    // of `order`); items stay in position order, so the FP64 sum order is fixed
    for (size_t t = 0; t < tiles.size(); ++t) {
        HTile ht{tiles[t].first, tiles[t].second, (int)hp.item_index.size(), 0};
        hp.item_index.insert(hp.item_index.end(), of_tile[t].begin(), of_tile[t].end());
        ht.item1 = (int)hp.item_index.size();
        hp.tiles.push_back(ht);
    }
    // staging reads whole 64-column chunks of a row: pad the planes' rows so
    // that every chunk stays inside them
    hp.ldp = M + 64 * ((hp.qb + std::max(span_a, span_b) + 63) / 64) + 64;
    const size_t plane_bytes = (size_t)hp.npl16 * N * hp.ldp * 4;
    hp.planes_bytes = (plane_bytes + 255) / 256 * 256;
    hp.ws_bytes = hp.planes_bytes + hp.items.size() * (size_t)hp.tm * hp.tn * 8;
    return hp;
}

HankelPlan make_hankel_plan(int N, int M, int P, int Q, int prec, int n_cu)
{
    if (prec != kPrecF32) return make_hankel_plan16(N, M, P, Q, prec, n_cu);
    HankelPlan hp;
    hp.N = N; hp.M = M; hp.P = P; hp.Q = Q; hp.prec = prec;
    const int PQ = P * Q, Kr = N - P + 1, Kc = M - Q + 1;
    const int nt = (PQ + 63) / 64;
    const int npl = planes_of(prec);
    // widest column window of a 64-row tile
    int span = 0;
    for (int t = 0; t < nt; ++t) {
        const int lo = (64 * t) / P, hi = std::min(Q - 1, std::min(PQ - 1, 64 * t + 63) / P);
        span = std::max(span, hi - lo);
    }
    // sub-tile: the most positions per staged byte within the LDS budget
    const size_t budget = 76 * 1024;
    double best = -1.0;
    for (int qb : {32, 64, 128}) {
        const int s = pad_stride(qb + span);
        for (int pb = 1; pb <= std::max(1, Kr); ++pb) {
            const size_t bytes = (size_t)npl * (pb + P) * (2 * s) * 4;
            if (bytes > budget) break;
            const double eff = (double)pb * qb / ((double)(pb + P) * s);
            if (eff > best) {
                best = eff;
                hp.pb = pb;
                hp.qb = qb;
                hp.stride_a = hp.stride_b = s;
                hp.lds = bytes;
            }
        }
    }
    if (hp.pb == 0) {   // very large windows: one row of positions, one workgroup per CU
        hp.qb = 32;
        hp.pb = 1;
        hp.stride_a = hp.stride_b = pad_stride(32 + span);
        hp.lds = (size_t)npl * (1 + P) * (2 * hp.stride_a) * 4;
    }
    // split the position rows of every upper tile so that there are ~8 items per CU
    const int n_tiles = nt * (nt + 1) / 2;
    const int target = 8 * std::max(1, n_cu);
    int splits = std::max(1, std::min(Kr, (target + n_tiles - 1) / n_tiles));
    for (int a = 0; a < nt; ++a) {
        for (int b = a; b < nt; ++b) {
            HTile t{64 * a, 64 * b, (int)hp.items.size(), 0};
            for (int s = 0; s < splits; ++s) {
                const int p0 = (int)((int64_t)s * Kr / splits), p1 = (int)((int64_t)(s + 1) * Kr / splits);
                if (p1 > p0) hp.items.push_back({64 * a, 64 * b, p0, p1, 0, Kc});
            }
            t.item1 = (int)hp.items.size();
            hp.tiles.push_back(t);
        }
    }
    hp.ws_bytes = hp.items.size() * (size_t)64 * 64 * 16;
    return hp;
}

}  // namespace covest
