// rec_kernels.hip -- the diagonal-segment recurrence (kernel family a) for
// gfx950.
//
// The paper's combination-parallel method (Sec. 3.3, Algorithm 1) computes each
// product A[r][c] * conj(A[r+dr][c+dc]) once and adds it to every output entry
// of its combination; those entries lie on one diagonal of R, in Q-|dc|
// segments of P-|dr| entries (Sec. 3.3, eq. 3.8).  Here the additions are not
// repeated either: entry (i1, j1) of combination (dr, dc) is the sum of the
// product grid over a Kr x Kc box, every box contains a common middle region,
// and neighbouring entries of a segment differ by one row (or column) of
// products entering the box and one leaving it (the shift rule of Sec. 3.3).
//
// rec_main      one launch for all products: bulk jobs (middle x middle, one sum
//               per lag), row-strip jobs (middle columns, one sum per
//               individual row) and column-strip jobs (middle rows, one sum per
//               individual column; walked on the transposed tile).
// rec_finalize  the finalize, one unique combination at a time: adds the
//               corner products, slides the box along the segment (FP64
//               carries), divides by K and writes the segment entries (upper
//               triangle and mirror).  Variants: rec_finalize (one wave per
//               combination, any size), rec_finalize_tab (a workgroup with the
//               corner table in LDS) and rec_finalize_scan (a workgroup, wave
//               prefix sums instead of slides, for large corner tables).
//
// Arithmetic: complex64 inputs are widened to FP64 once, when a tile is staged
// in LDS.  A product of two floats is exact in FP64, so every sum is an FP64
// sum of exact products; on small-integer inputs every intermediate is an
// integer below 2^53 and the result is bit-exact.
#include <hip/hip_runtime.h>

#include "covest_internal.hpp"
#include "device_util.hpp"

namespace covest {

// acc += x * conj(y)
__device__ __forceinline__ void cmac(double2 &acc, const double2 x, const double2 y)
{
    acc.x = fma(x.x, y.x, acc.x);
    acc.x = fma(x.y, y.y, acc.x);
    acc.y = fma(x.y, y.x, acc.y);
    acc.y = fma(-x.x, y.y, acc.y);
}

__device__ __forceinline__ double2 cprod(const double2 x, const double2 y)
{
    double2 r = make_double2(0.0, 0.0);
    cmac(r, x, y);
    return r;
}

__device__ __forceinline__ double2 cadd(double2 a, double2 b) { return make_double2(a.x + b.x, a.y + b.y); }
__device__ __forceinline__ double2 csub(double2 a, double2 b) { return make_double2(a.x - b.x, a.y - b.y); }

// Strip sum of individual row (or column) idx for one lag: the pieces of the
// strip, added in piece order.
__device__ __forceinline__ double2 zsum(const double2 *z, int idx, int nrows, int pieces, int64_t ls2, int lag)
{
    double2 s = z[(int64_t)idx * ls2 + lag];
    for (int p = 1; p < pieces; ++p) s = cadd(s, z[((int64_t)p * nrows + idx) * ls2 + lag]);
    return s;
}

__device__ __forceinline__ double2 ld_a(const Inst &in, int r, int c)
{
    const float2 v = static_cast<const float2 *>(in.A)[(int64_t)r * in.lda + c];
    return make_double2((double)v.x, (double)v.y);
}

// Ring walk along one tile row.  xs[c] is the first factor at walk column c,
// ys[c + w] the second factor of lag w.  Per column: one LDS read of the new
// second factor, one (broadcast) read of the first factor, W complex MACs.
template <int W>
__device__ __forceinline__ void ring_walk(const double2 *__restrict__ xs,
                                          const double2 *__restrict__ ys, int nblocks,
                                          double2 (&acc)[W])
{
    double2 ring[W];
#pragma unroll
    for (int k = 0; k < W - 1; ++k) ring[k] = ys[k];
    for (int b = 0; b < nblocks; ++b) {
        const double2 *xb = xs + b * W;
        const double2 *yb = ys + b * W;
#pragma unroll
        for (int u = 0; u < W; ++u) {
            ring[(u + W - 1) % W] = yb[u + W - 1];
            const double2 x = xb[u];
#pragma unroll
            for (int w = 0; w < W; ++w) cmac(acc[w], x, ring[(u + w) % W]);
        }
    }
}

// Stage B[tr0 + i][tc0 + j] (i < nr, j < nc) as FP64 into lds[i * stride + j];
// B = A (orient 0) or A^T (orient 1); entries outside A are zero.  The global
// loads are issued in batches of kFillBatch per thread before any of them is
// used, so their latencies overlap.
constexpr int kFillBatch = 8;

__device__ __forceinline__ void fill_tile(double2 *lds, int stride, const Inst &in, int orient,
                                          int tr0, int nr, int tc0, int nc)
{
    const float2 *A = static_cast<const float2 *>(in.A);
    const int total = nr * nc;
    // orient 0: j (A column) runs fastest; orient 1: i (A column) runs fastest
    const int fast = orient ? nr : nc;
    for (int e0 = threadIdx.x; e0 < total; e0 += kFillBatch * kThreads) {
        float2 v[kFillBatch];
        int dst[kFillBatch];
#pragma unroll
        for (int k = 0; k < kFillBatch; ++k) {
            const int e = e0 + k * kThreads;
            const int s = e / fast, f = e - s * fast;
            const int i = orient ? f : s, j = orient ? s : f;
            const int ar = orient ? tc0 + j : tr0 + i;
            const int ac = orient ? tr0 + i : tc0 + j;
            const bool ok = e < total && ar >= 0 && ar < in.N && ac >= 0 && ac < in.M;
            v[k] = ok ? A[(int64_t)ar * in.lda + ac] : make_float2(0.f, 0.f);
            dst[k] = e < total ? i * stride + j : -1;
        }
#pragma unroll
        for (int k = 0; k < kFillBatch; ++k)
            if (dst[k] >= 0) lds[dst[k]] = make_double2((double)v[k].x, (double)v[k].y);
    }
}

__device__ __forceinline__ int lag_index(const Inst &in, int orient, int d1, int d2)
{
    const int dr = orient ? d2 : d1;
    const int dc = orient ? d1 : d2;
    return (dr + in.P - 1) * in.Q + dc;
}

template <int W>
__device__ void run_bulk(const Job &job, const Inst &in, const LagGroup &g, double2 *lds)
{
    const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
    const int L = g.lanes, S = g.slots;
    const int slot = lane / L, li = lane - slot * L;
    const bool active = slot < S;
    const int d1 = g.d1lo + li / g.nch;
    const int d2 = g.ch0 + (li % g.nch) * W;

    double2 acc[W];
#pragma unroll
    for (int w = 0; w < W; ++w) acc[w] = make_double2(0.0, 0.0);

    const int nrg = (in.Rm1 - in.Rm0 + S - 1) / S;
    const int bandw = kWaves * W;
    int u = job.u0;
    while (u < job.u1) {
        const int band = u / nrg, rg = u - band * nrg;
        const int rg_end = min(nrg, rg + (job.u1 - u));
        const int xr_a = in.Rm0 + rg * S;
        const int xr_b = min(in.Rm1, in.Rm0 + rg_end * S);
        const int xc = in.Cm0 + band * bandw;
        for (int r = xr_a; r < xr_b; r += job.tile_rows) {
            const int r_end = min(xr_b, r + job.tile_rows);
            const int tr0 = r + g.hr_lo, nr = r_end + g.hr_hi - tr0;
            const int tc0 = xc + g.hc_lo, nc = xc + bandw + g.hc_hi - tc0;
            const int stride = nc | 1;
            __syncthreads();
            fill_tile(lds, stride, in, 0, tr0, nr, tc0, nc);
            __syncthreads();
            if (active) {
                const int xcw = xc + wave * W;
                for (int t = r + slot; t < r_end; t += S) {
                    const double2 *xs = lds + (t - tr0) * stride + (xcw - tc0);
                    const double2 *ys = lds + (t + d1 - tr0) * stride + (xcw + d2 - tc0);
                    ring_walk<W>(xs, ys, 1, acc);
                }
            }
        }
        u += rg_end - rg;
    }

    // Sum the lanes that hold the same lags (every wave and slot), fixed order.
    __syncthreads();
#pragma unroll
    for (int w = 0; w < W; ++w) lds[(wave * 64 + lane) * W + w] = acc[w];
    __syncthreads();
    double *out = in.partial + (int64_t)job.out * in.lag_stride * 2;
    for (int e = threadIdx.x; e < L * W; e += kThreads) {
        const int l2 = e / W, w = e - l2 * W;
        const int e1 = g.d1lo + l2 / g.nch;
        const int e2 = g.ch0 + (l2 % g.nch) * W + w;
        if (e2 < g.v2lo || e2 >= g.v2hi) continue;
        double2 s = make_double2(0.0, 0.0);
        for (int wv = 0; wv < kWaves; ++wv)
            for (int sl = 0; sl < S; ++sl) s = cadd(s, lds[(wv * 64 + sl * L + l2) * W + w]);
        const int idx = lag_index(in, 0, e1, e2);
        reinterpret_cast<double2 *>(out)[idx] = s;
    }
}

template <int W>
__device__ void run_strip(const Job &job, const Inst &in, const LagGroup &g, double2 *lds)
{
    const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
    const int L = g.lanes, S = g.slots;
    const int slot = lane / L, li = lane - slot * L;
    const int d1 = g.d1lo + li / g.nch;
    const int d2 = g.ch0 + (li % g.nch) * W;
    const int t = job.x0 + wave * S + slot;
    const bool mine = slot < S && t < job.x1;

    double2 acc[W];
#pragma unroll
    for (int w = 0; w < W; ++w) acc[w] = make_double2(0.0, 0.0);

    const int tr0 = job.x0 + g.hr_lo, nr = job.x1 + g.hr_hi - tr0;
    for (int c = job.c0; c < job.c1; c += job.tile_cols) {
        const int c_end = min(job.c1, c + job.tile_cols);
        const int tc0 = c + g.hc_lo, nc = c_end + g.hc_hi - tc0;
        const int stride = nc | 1;
        __syncthreads();
        fill_tile(lds, stride, in, g.orient, tr0, nr, tc0, nc);
        __syncthreads();
        if (mine) {
            const double2 *xs = lds + (t - tr0) * stride + (c - tc0);
            const double2 *ys = lds + (t + d1 - tr0) * stride + (c + d2 - tc0);
            ring_walk<W>(xs, ys, (c_end - c) / W, acc);
        }
    }
    if (!mine) return;
    double *base = g.orient ? in.zc : in.zr;
    double2 *row = reinterpret_cast<double2 *>(base + (int64_t)(job.out + (t - job.x0)) * in.lag_stride * 2);
#pragma unroll
    for (int w = 0; w < W; ++w) {
        const int e2 = d2 + w;
        if (e2 >= g.v2lo && e2 < g.v2hi) row[lag_index(in, g.orient, d1, e2)] = acc[w];
    }
}

__device__ __forceinline__ void run_job(const MainArgs &ma, int b, double2 *lds)
{
    const Job job = ma.jobs[b];
    const Inst in = ma.use_inline ? ma.inst_inline : ma.insts[job.inst];
    const LagGroup g = ma.groups[job.group];
    if (job.mode == kJobBulk) {
        switch (g.W) {
        case 16: run_bulk<16>(job, in, g, lds); break;
        case 12: run_bulk<12>(job, in, g, lds); break;
        case 8: run_bulk<8>(job, in, g, lds); break;
        default: run_bulk<4>(job, in, g, lds); break;
        }
    } else {
        switch (g.W) {
        case 16: run_strip<16>(job, in, g, lds); break;
        case 12: run_strip<12>(job, in, g, lds); break;
        case 8: run_strip<8>(job, in, g, lds); break;
        default: run_strip<4>(job, in, g, lds); break;
        }
    }
}

// One workgroup per job (single problems).
__global__ void __launch_bounds__(kThreads, 2) rec_main(MainArgs ma)
{
    extern __shared__ double2 lds[];
    int b = blockIdx.x;
    if (ma.xcd_remap) b = xcd_block(b, ma.n_jobs);
    run_job(ma, b, lds);
}

// Persistent form for batches: every resident workgroup claims the next job
// of the (longest-first) work list from a device counter until the list is
// exhausted (Sec. 3.4: a free core simply takes the next combination).  Each
// job writes its own outputs, so results do not depend on which workgroup ran
// which job.
__global__ void __launch_bounds__(kThreads, 2) rec_main_persistent(MainArgs ma, unsigned int *counter)
{
    extern __shared__ double2 lds[];
    __shared__ int s_job;
    for (;;) {
        if (threadIdx.x == 0) s_job = (int)atomicAdd(counter, 1u);
        __syncthreads();
        const int j = s_job;
        __syncthreads();
        if (j >= ma.n_jobs) break;
        run_job(ma, j, lds);
    }
}

__global__ void reset_counter(unsigned int *counter) { *counter = 0u; }

// ---------------------------------------------------------------------------
// Finalize: one wave per unique combination.
// ---------------------------------------------------------------------------

__device__ __forceinline__ double2 wave_sum(double2 v)
{
#pragma unroll
    for (int off = 32; off >= 1; off >>= 1) {
        v.x += __shfl_xor(v.x, off, 64);
        v.y += __shfl_xor(v.y, off, 64);
    }
    return v;
}

__device__ __forceinline__ void store_r(const Inst &in, int k1, int k2, double2 s, bool diag)
{
    double2 v = s;
    if (in.normalize) {
        const double K = (double)in.Kr * (double)in.Kc;
        v.x = s.x / K;
        v.y = s.y / K;
    }
    if (diag) v.y = 0.0;
    if (in.out_fp64) {
        double2 *R = static_cast<double2 *>(in.R);
        R[(int64_t)k1 * in.ldr + k2] = v;
        if (in.fill_full && !diag) R[(int64_t)k2 * in.ldr + k1] = make_double2(v.x, -v.y);
    } else {
        float2 *R = static_cast<float2 *>(in.R);
        const float2 f = make_float2((float)v.x, (float)v.y);
        R[(int64_t)k1 * in.ldr + k2] = f;
        if (in.fill_full && !diag) R[(int64_t)k2 * in.ldr + k1] = make_float2(f.x, -f.y);
    }
}

// Per-item timing of a measurement run (fa.stamps non-null): the constant
// 100 MHz wall clock when the item's workgroup starts and when all its threads
// are done, written by thread 0.  A null fa.stamps (every ordinary call)
// skips both.
struct ItemStamp {
    unsigned long long t0;
    __device__ explicit ItemStamp(const FinArgs &fa) : t0(fa.stamps ? wall_clock64() : 0ull) {}
    __device__ void done(const FinArgs &fa, int idx) const
    {
        if (fa.stamps) {
            __syncthreads();
            if (threadIdx.x == 0) {
                fa.stamps[2 * idx] = t0;
                fa.stamps[2 * idx + 1] = wall_clock64();
            }
        }
    }
};

__global__ void __launch_bounds__(64) rec_finalize(FinArgs fa)
{
    const ItemStamp stamp(fa);
    extern __shared__ double2 cs[];
    const FinItem it = fa.items[xcd_block(blockIdx.x, fa.n_items)];
    const Inst in = fa.use_inline ? fa.inst_inline : fa.insts[it.inst];
    const int P = in.P, N = in.N, Kr = in.Kr, Kc = in.Kc;
    const int dr = it.dr, dc = it.dc;
    const int lag = (dr + P - 1) * in.Q + dc;
    const int64_t ls2 = (int64_t)in.lag_stride;
    const int lane = threadIdx.x;
    const int rlo = max(0, -dr), rhi = N - max(0, dr);
    const int nr = P - abs(dr);
    const int nc = in.Q - dc;
    const int Rm0 = in.Rm0, Rm1 = in.Rm1, Cm0 = in.Cm0, Cm1 = in.Cm1;
    const double2 *partial = reinterpret_cast<const double2 *>(in.partial);
    const double2 *zr = reinterpret_cast<const double2 *>(in.zr);
    const double2 *zc = reinterpret_cast<const double2 *>(in.zc);
#define ZR(i) zsum(zr, (i), in.n_ir, in.zpieces, ls2, lag)
#define ZC(i) zsum(zc, (i), in.n_ic, in.zpieces, ls2, lag)
    const bool has_mr = Rm1 > Rm0;   // column strips exist (they walk the middle rows)
    const bool has_mc = Cm1 > Cm0;   // row strips exist (they walk the middle columns)

    // Middle sum of this lag: fixed-order sum of the bulk partials.
    double2 zm = make_double2(0.0, 0.0);
    for (int j = it.bulk0 + lane; j < it.bulk1; j += 64) zm = cadd(zm, partial[j * ls2 + lag]);
    zm = wave_sum(zm);

    // Step 1: for every row class (the middle rows as one class, then each
    // individual row that some box of this lag contains), the sums over the
    // column range of every column offset b, by sliding along b.
    const int ncls = 1 + in.n_ir;
    for (int e = lane; e < ncls; e += 64) {
        double2 *out = cs + e * nc;
        if (e == 0) {
            if (!has_mr) {
                for (int b = 0; b < nc; ++b) out[b] = make_double2(0.0, 0.0);
                continue;
            }
            double2 s = zm;
            for (int c = 0; c < min(Cm0, Kc); ++c) s = cadd(s, ZC(c));
            for (int c = Cm1; c < Kc; ++c) s = cadd(s, ZC(Cm0 + c - Cm1));
            out[0] = s;
            for (int b = 0; b + 1 < nc; ++b) {
                const int cin = b + Kc;   // enters: an individual column >= Cm1
                s = csub(s, ZC(b));
                s = cadd(s, ZC(Cm0 + cin - Cm1));
                out[b + 1] = s;
            }
        } else {
            const int rho = e - 1;
            const int r = rho < Rm0 ? rho : Rm1 + (rho - Rm0);
            if (r < rlo || r >= rhi) continue;
            double2 s = has_mc ? ZR(rho) : make_double2(0.0, 0.0);
            for (int c = 0; c < min(Cm0, Kc); ++c) s = cadd(s, cprod(ld_a(in, r, c), ld_a(in, r + dr, c + dc)));
            for (int c = Cm1; c < Kc; ++c) s = cadd(s, cprod(ld_a(in, r, c), ld_a(in, r + dr, c + dc)));
            out[0] = s;
            for (int b = 0; b + 1 < nc; ++b) {
                const int cin = b + Kc;
                s = csub(s, cprod(ld_a(in, r, b), ld_a(in, r + dr, b + dc)));
                s = cadd(s, cprod(ld_a(in, r, cin), ld_a(in, r + dr, cin + dc)));
                out[b + 1] = s;
            }
        }
    }
    __syncthreads();

    // Step 2: for each column offset b, slide the box down the segment.
    for (int b = lane; b < nc; b += 64) {
        double2 s = cs[b];
        for (int r = rlo; r < min(Rm0, rlo + Kr); ++r) s = cadd(s, cs[(1 + r) * nc + b]);
        for (int r = max(Rm1, rlo); r < rlo + Kr; ++r) s = cadd(s, cs[(1 + Rm0 + r - Rm1) * nc + b]);
        for (int a = 0; a < nr; ++a) {
            const int i1 = rlo + a;
            const int k1 = i1 + P * b;
            const int k2 = (i1 + dr) + P * (b + dc);
            store_r(in, k1, k2, s, dr == 0 && dc == 0);
            if (a + 1 < nr) {
                const int rout = i1;          // an individual row < Rm0
                const int rin = i1 + Kr;      // an individual row >= Rm1
                s = csub(s, cs[(1 + rout) * nc + b]);
                s = cadd(s, cs[(1 + Rm0 + rin - Rm1) * nc + b]);
            }
        }
    }
    stamp.done(fa, xcd_block(blockIdx.x, fa.n_items));
}

// s + t[lo·st] + t[(lo+1)·st] + ... + t[(hi−1)·st], added in index order.  The
// LDS reads of each group of kChainGroup terms are issued together, so the
// chain waits for one read latency per group instead of one per term.
constexpr int kChainGroup = 8;
__device__ __forceinline__ double2 lds_chain(double2 s, const double2 *t, int lo, int hi, int st)
{
    for (int g = lo; g < hi; g += kChainGroup) {
        double2 v[kChainGroup];
#pragma unroll
        for (int k = 0; k < kChainGroup; ++k) v[k] = t[min(g + k, hi - 1) * st];
#pragma unroll
        for (int k = 0; k < kChainGroup; ++k)
            if (g + k < hi) s = cadd(s, v[k]);
    }
    return s;
}

// Table variant of the finalize (256 threads, one unique combination): every
// product the sliding needs is computed at once into an LDS table (rows:
// the middle class and each individual row; columns: the individual columns),
// so the loads overlap instead of forming one long dependent chain per lane.
// The sums run in the same order as rec_finalize.  kFinBatch: corner loads
// per thread in flight; kFinChunk: offsets per thread in the two slides.
// Small tables take <4, 4>, which needs fewer registers, so that more
// workgroups share a CU.
template <int kFinBatch, int kFinChunk>
__global__ void __launch_bounds__(256) rec_finalize_tab(FinArgs fa)
{
    const ItemStamp stamp(fa);
    extern __shared__ double2 V[];
    __shared__ double2 red[256];
    __shared__ double2 zrs[kFinMaxRows];   // row-strip sums of the individual rows
    const FinItem it = fa.items[xcd_block(blockIdx.x, fa.n_items)];
    const Inst in = fa.use_inline ? fa.inst_inline : fa.insts[it.inst];
    const int P = in.P, N = in.N, M = in.M, Kr = in.Kr, Kc = in.Kc;
    const int dr = it.dr, dc = it.dc;
    const int lag = (dr + P - 1) * in.Q + dc;
    const int64_t ls2 = (int64_t)in.lag_stride;
    const int tid = threadIdx.x;
    const int rlo = max(0, -dr), rhi = N - max(0, dr);
    const int nr = P - abs(dr);
    const int nc = in.Q - dc;
    const int Rm0 = in.Rm0, Rm1 = in.Rm1, Cm0 = in.Cm0, Cm1 = in.Cm1;
    const bool has_mr = Rm1 > Rm0, has_mc = Cm1 > Cm0;
    const double2 *partial = reinterpret_cast<const double2 *>(in.partial);
    const double2 *zr = reinterpret_cast<const double2 *>(in.zr);
    const double2 *zc = reinterpret_cast<const double2 *>(in.zc);
#define ZR(i) zsum(zr, (i), in.n_ir, in.zpieces, ls2, lag)
#define ZC(i) zsum(zc, (i), in.n_ic, in.zpieces, ls2, lag)
    const float2 *A = static_cast<const float2 *>(in.A);
    const int nV = in.n_ic;
    const int nVs = nV | 1;   // odd row stride: no LDS bank conflicts across rows
    const int ncls = 1 + in.n_ir;

    // Every global load of the item goes out before any result is used: the
    // lag's bulk partials (two per thread, more in a loop if there are
    // more), its column- and row-strip sums and the first kFinBatch corner
    // products of each thread; so the item waits for about one load latency.
    const int ncorner = (ncls - 1) * nV;
    // corner e -> (individual row rho, individual column gi): floor((e + 1/2) / nV)
    // in float is exact for every used e (a quotient below n_ir <= 160 carries
    // an error below 161 * 2^-23 < 2^-15; its distance to an integer is at
    // least 1/(2 nV) >= 2^-14, as the table holds at most 6144 entries), and
    // much cheaper than an integer division by a run-time value
    const float rcp_nV = 1.0f / (float)nV;
    auto corner_rho = [&](int e) { return (int)fmaf((float)e, rcp_nV, 0.5f * rcp_nV); };
    float2 xs[kFinBatch], ys[kFinBatch];
    bool ok[kFinBatch];
    const int64_t lag_off = (int64_t)dr * in.lda + dc;
    auto corner_loads = [&](int e0) {
#pragma unroll
        for (int k = 0; k < kFinBatch; ++k) {
            const int e = e0 + k * 256;
            const int rho = corner_rho(e), gi = e - rho * nV;
            const int c = gi < Cm0 ? gi : Cm1 + (gi - Cm0);
            const int r = rho < Rm0 ? rho : Rm1 + (rho - Rm0);
            ok[k] = e < ncorner && c + dc < M && r >= rlo && r < rhi;
            const int rr = ok[k] ? r : rlo, cc = ok[k] ? c : 0;
            const int64_t off = (int64_t)rr * in.lda + cc;
            xs[k] = A[off];
            ys[k] = A[off + lag_off];
        }
    };
    auto corner_store = [&](int e0) {
#pragma unroll
        for (int k = 0; k < kFinBatch; ++k) {
            const int e = e0 + k * 256;
            const int rho = corner_rho(e);
            if (e < ncorner)
                V[(1 + rho) * nVs + (e - rho * nV)] =
                    ok[k] ? cprod(make_double2(xs[k].x, xs[k].y), make_double2(ys[k].x, ys[k].y))
                          : make_double2(0.0, 0.0);
        }
    };
    const int j0 = it.bulk0 + tid, j1 = j0 + 256;
    const double2 p0 = j0 < it.bulk1 ? partial[j0 * ls2 + lag] : make_double2(0.0, 0.0);
    const double2 p1 = j1 < it.bulk1 ? partial[j1 * ls2 + lag] : make_double2(0.0, 0.0);
    const int cz = tid < Cm0 ? tid : Cm1 + (tid - Cm0);
    const bool zc_ok = tid < nV && has_mr && cz + dc < M;
    const double2 zc_v = zc_ok ? ZC(tid) : make_double2(0.0, 0.0);
    for (int i = tid; i < in.n_ir; i += 256) zrs[i] = has_mc ? ZR(i) : make_double2(0.0, 0.0);
    corner_loads(tid);

    // Middle sum: fixed-order tree over the bulk partials.
    double2 z = cadd(make_double2(0.0, 0.0), p0);
    if (j1 < it.bulk1) z = cadd(z, p1);
    for (int j = j1 + 256; j < it.bulk1; j += 256) z = cadd(z, partial[j * ls2 + lag]);
    red[tid] = z;
    __syncthreads();
    for (int s = 128; s > 0; s >>= 1) {
        if (tid < s) red[tid] = cadd(red[tid], red[tid + s]);
        __syncthreads();
    }
    const double2 zm = red[0];

    // Phase A: the table of individual-column terms of every row class: the
    // column-strip sums (class 0), then the corner products.
    for (int gi = tid; gi < nV; gi += 256) {
        const int c = gi < Cm0 ? gi : Cm1 + (gi - Cm0);
        V[gi] = gi == tid ? zc_v : ((has_mr && c + dc < M) ? ZC(gi) : make_double2(0.0, 0.0));
    }
    corner_store(tid);
    for (int e0 = tid + kFinBatch * 256; e0 < ncorner; e0 += kFinBatch * 256) {
        corner_loads(e0);
        corner_store(e0);
    }
    __syncthreads();

    // Phase B: per class, the sums over the column range of every offset b.
    // Thread (class, chunk of kFinChunk offsets) seeds its first offset with a
    // direct sum and slides across the chunk (one column leaves, one enters);
    // results are written in place over the consumed left-column terms after
    // a barrier.
    const int nchunk_b = (nc + kFinChunk - 1) / kFinChunk;
    const int cls_per = 256 / nchunk_b;   // whole classes per pass: a class is never split
    for (int cbase = 0; cbase < ncls; cbase += cls_per) {
        // neighbouring threads take neighbouring classes: rows nVs apart,
        // which fall in different LDS banks
        const int cls = cbase + tid % cls_per, ch = tid / cls_per;
        double2 res[kFinChunk];
        bool live = tid < cls_per * nchunk_b && cls < ncls;
        if (live && cls > 0) {
            const int rho = cls - 1;
            const int r = rho < Rm0 ? rho : Rm1 + (rho - Rm0);
            live = r >= rlo && r < rhi;
        }
        const int b0 = ch * kFinChunk, b1 = min(nc, b0 + kFinChunk);
        if (live) {
            const double2 *row = V + cls * nVs;
            double2 s;
            if (cls == 0) s = has_mr ? zm : make_double2(0.0, 0.0);
            else s = zrs[cls - 1];
            // columns [b0, b0 + Kc) of the individual set: left part, right part
            s = lds_chain(s, row, b0, min(Cm0, b0 + Kc), 1);
            s = lds_chain(s, row, Cm0 + max(Cm1, b0) - Cm1, Cm0 + b0 + Kc - Cm1, 1);
#pragma unroll
            for (int k = 0; k < kFinChunk; ++k) {
                const int b = b0 + k;
                res[k] = s;
                if (b + 1 < b1) s = cadd(csub(s, row[b]), row[Cm0 + (b + Kc) - Cm1]);
            }
        }
        __syncthreads();
        if (live) {
            double2 *row = V + cls * nVs;
#pragma unroll
            for (int k = 0; k < kFinChunk; ++k)
                if (b0 + k < b1) row[b0 + k] = res[k];
        }
        __syncthreads();
    }

    // Phase C: thread (b, chunk of kFinChunk row offsets) seeds the box at its
    // first offset with a direct sum over the row classes and slides it down
    // the segment (one row leaves, one enters), writing each entry.
    const int nchunk_a = (nr + kFinChunk - 1) / kFinChunk;
    for (int t = tid; t < nc * nchunk_a; t += 256) {
        const int b = t % nc, ch = t / nc;
        const int a0 = ch * kFinChunk, a1 = min(nr, a0 + kFinChunk);
        const int i0 = rlo + a0;
        double2 s = V[b];
        s = lds_chain(s, V + nVs + b, i0, min(Rm0, i0 + Kr), nVs);
        s = lds_chain(s, V + nVs + b, Rm0 + max(Rm1, i0) - Rm1, Rm0 + i0 + Kr - Rm1, nVs);
        // the rows leaving and entering at each step, read up front (a step
        // that does not slide reads entry b of class 0 instead, and drops it)
        double2 vout[kFinChunk - 1], vin[kFinChunk - 1];
#pragma unroll
        for (int k = 0; k + 1 < kFinChunk; ++k) {
            const int i1 = rlo + a0 + k;
            const bool sl = a0 + k + 1 < a1;
            vout[k] = V[sl ? (1 + i1) * nVs + b : b];
            vin[k] = V[sl ? (1 + Rm0 + i1 + Kr - Rm1) * nVs + b : b];
        }
#pragma unroll
        for (int k = 0; k < kFinChunk; ++k) {
            const int a = a0 + k;
            if (a < a1) {
                const int i1 = rlo + a;
                const int k1 = i1 + P * b;
                const int k2 = (i1 + dr) + P * (b + dc);
                store_r(in, k1, k2, s, dr == 0 && dc == 0);
                if (k + 1 < kFinChunk && a + 1 < a1) s = cadd(csub(s, vout[k]), vin[k]);
            }
        }
    }
    stamp.done(fa, xcd_block(blockIdx.x, fa.n_items));
}

// Inclusive prefix sum over the 64 lanes of a wave, in a fixed order: three
// shifts inside each row of 16 lanes give sums of 4, shifts by 4 and 8 (which
// lanes near the start of a row read as zero) complete the rows, two row
// broadcasts carry the row totals.  Lanes a step does not reach add zero.
template <int CTRL, int RMASK, int BMASK>
__device__ __forceinline__ double dpp_f64(double v)
{
    const int lo = __builtin_amdgcn_update_dpp(0, __double2loint(v), CTRL, RMASK, BMASK, true);
    const int hi = __builtin_amdgcn_update_dpp(0, __double2hiint(v), CTRL, RMASK, BMASK, true);
    return __hiloint2double(hi, lo);
}

__device__ __forceinline__ double wave_scan(double v)
{
    double s = v + dpp_f64<0x111, 0xf, 0xf>(v);   // row_shr:1
    s += dpp_f64<0x112, 0xf, 0xf>(v);             // row_shr:2
    s += dpp_f64<0x113, 0xf, 0xf>(v);             // row_shr:3
    s += dpp_f64<0x114, 0xf, 0xf>(s);             // row_shr:4 (lanes 0-3 of a row read zero)
    s += dpp_f64<0x118, 0xf, 0xf>(s);             // row_shr:8 (lanes 0-7 of a row read zero)
    s += dpp_f64<0x142, 0xa, 0xf>(s);             // row_bcast:15 into rows 1 and 3
    s += dpp_f64<0x143, 0xc, 0xf>(s);             // row_bcast:31 into rows 2 and 3
    return s;
}

// exclusive prefix sum over the lanes: the sum of the lanes below this one
__device__ __forceinline__ double2 wave_scan_excl(double2 v)
{
    return make_double2(wave_scan(v.x) - v.x, wave_scan(v.y) - v.y);
}

// E[hi] - E[lo] for this lane, E being the wave's values in its LDS row
// (written just before by the same wave: a wave's LDS operations run in order)
__device__ __forceinline__ double2 range_sum(double2 *row, double2 e, int lo, int hi)
{
    row[threadIdx.x & 63] = e;
    __builtin_amdgcn_fence(__ATOMIC_RELEASE, "wavefront");
    __builtin_amdgcn_wave_barrier();
    __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "wavefront");
    const double2 h = row[hi], l = row[lo];
    __builtin_amdgcn_fence(__ATOMIC_RELEASE, "wavefront");
    __builtin_amdgcn_wave_barrier();
    __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "wavefront");
    return csub(h, l);
}

// Wave-scan variant of the finalize (256 threads, one unique combination;
// at most 63 individual columns and 63 individual rows).  Entry (a, b) of
// the lag's segments is the sum over a box that contains the middle block:
// the middle sum, plus for the middle rows (class 0) and every individual
// row inside the box (classes 1..) the row's strip sum and its terms in the
// individual columns inside the box.  The individual columns inside the box
// for offset b are one contiguous range [glo, ghi) of the individual-column
// order, the rows for offset a likewise [ra, rb) (see span), so
//   row pass:    each wave takes classes in turn, one individual column per
//                lane: an exclusive prefix sum E over the lanes gives, for
//                lane b, the class's sum over [glo(b), ghi(b)) as
//                E[ghi] - E[glo] (read back through a row of LDS);
//   column pass: each wave takes offsets b in turn, one individual row per
//                lane: likewise the sum over the rows [ra(a), rb(a)).
// Only the classes' sums per offset live in LDS (nc x (1 + n_ir)); the corner
// products never do.  Rows and columns a lag cannot use are zeroed before
// the sums, so the differences of prefix sums cancel exactly what they should.
template <bool INLINE, int KCLS>
__global__ void __launch_bounds__(256) rec_finalize_scan(FinArgs fa)
{
    const ItemStamp stamp(fa);
    // classes per wave at most: 16 (1 + n_ir <= 64) or 8 (1 + n_ir <= 32, fewer
    // registers, so more workgroups per CU hide the loads of small tables)
    constexpr int kCls = KCLS;
    extern __shared__ double2 St[];
    __shared__ double2 red[4];
    __shared__ double2 xch[4][64];   // per wave: the prefix sums, read back at two lanes
    const FinItem it = fa.items[xcd_block(blockIdx.x, fa.n_items)];
    const Inst in = INLINE ? fa.inst_inline : fa.insts[it.inst];
    const int P = in.P, N = in.N, M = in.M, Kr = in.Kr, Kc = in.Kc;
    const int dr = it.dr, dc = it.dc;
    const int lag = (dr + P - 1) * in.Q + dc;
    const int64_t ls2 = (int64_t)in.lag_stride;
    const int tid = threadIdx.x, lane = tid & 63;
    const int wave = __builtin_amdgcn_readfirstlane(tid >> 6);
    const int rlo = max(0, -dr), rhi = N - max(0, dr);
    const int nr = P - abs(dr);
    const int nc = in.Q - dc;
    const int Rm0 = in.Rm0, Rm1 = in.Rm1, Cm0 = in.Cm0, Cm1 = in.Cm1;
    const bool has_mr = Rm1 > Rm0, has_mc = Cm1 > Cm0;
    const int nir = in.n_ir, nic = in.n_ic, ncls = 1 + nir;
    const int sst = ncls | 1;   // row stride of the classes' sums (odd: no bank conflicts)
    const double2 *partial = reinterpret_cast<const double2 *>(in.partial);
    const double2 *zr = reinterpret_cast<const double2 *>(in.zr);
    const double2 *zc = reinterpret_cast<const double2 *>(in.zc);
    const float2 *A = static_cast<const float2 *>(in.A);
    auto span = [](int x0, int n, int m0, int m1, int &lo, int &hi) {
        lo = x0 < m0 ? x0 : m0 + max(0, x0 - m1);
        hi = x0 + n > m1 ? m0 + x0 + n - m1 : min(m0, x0 + n);
    };

    // Every global load goes out first: the bulk partials, this wave's
    // corner pairs (lane = individual column) and, in wave 0, the middle
    // rows' column strips.
    const int g = lane;
    const int c = g < Cm0 ? g : Cm1 + (g - Cm0);
    const bool col_ok = g < nic && c + dc < M;
    double2 z = make_double2(0.0, 0.0);
    {
        const int j0 = it.bulk0 + tid;
        if (j0 < it.bulk1) z = partial[j0 * ls2 + lag];
    }
    float2 xs[kCls], ys[kCls];
    bool ok[kCls];
    const int64_t lag_off = (int64_t)dr * in.lda + dc;
#pragma unroll
    for (int k = 0; k < kCls; ++k) {
        const int cls = wave + 4 * k;
        const int rho = cls - 1;
        const int r = rho < Rm0 ? rho : Rm1 + (rho - Rm0);
        ok[k] = cls >= 1 && cls < ncls && col_ok && r >= rlo && r < rhi;
        const int64_t off = ok[k] ? (int64_t)r * in.lda + c : (int64_t)rlo * in.lda;
        xs[k] = A[off];
        ys[k] = A[off + lag_off];
    }
    const double2 zc_v = wave == 0 && has_mr && col_ok ? ZC(g) : make_double2(0.0, 0.0);
    // the row strips of this wave's classes: lane k holds class wave + 4k's
    double2 zr_l = make_double2(0.0, 0.0);
    {
        const int cls = wave + 4 * lane, rho = cls - 1;
        const int r = rho < Rm0 ? rho : Rm1 + (rho - Rm0);
        if (lane < kCls && cls >= 1 && cls < ncls && has_mc && r >= rlo && r < rhi) zr_l = ZR(rho);
    }
    for (int j = it.bulk0 + tid + 256; j < it.bulk1; j += 256) z = cadd(z, partial[j * ls2 + lag]);
    // middle sum: a fixed-order butterfly in each wave, then the waves in order
    z = wave_sum(z);
    if (lane == 0) red[wave] = z;

    // row pass
    int glo, ghi;
    span(lane, Kc, Cm0, Cm1, glo, ghi);   // lane = offset b
#pragma unroll
    for (int k = 0; k < kCls; ++k) {
        const int cls = wave + 4 * k;
        if (cls >= ncls) break;
        const double2 v = cls == 0 ? zc_v
                          : ok[k] ? cprod(make_double2(xs[k].x, xs[k].y), make_double2(ys[k].x, ys[k].y))
                                  : make_double2(0.0, 0.0);
        // lane k's row strip, read into scalar registers (zero for class 0)
        const double2 base = make_double2(
            __hiloint2double(__builtin_amdgcn_readlane(__double2hiint(zr_l.x), k),
                             __builtin_amdgcn_readlane(__double2loint(zr_l.x), k)),
            __hiloint2double(__builtin_amdgcn_readlane(__double2hiint(zr_l.y), k),
                             __builtin_amdgcn_readlane(__double2loint(zr_l.y), k)));
        const double2 sum = range_sum(xch[wave], wave_scan_excl(v), glo, ghi);
        if (lane < nc) St[lane * sst + cls] = cadd(base, sum);
    }
    __syncthreads();

    // column pass
    const double2 zm = has_mr ? cadd(cadd(red[0], red[1]), cadd(red[2], red[3])) : make_double2(0.0, 0.0);
    int ra, rb;
    span(rlo + lane, Kr, Rm0, Rm1, ra, rb);   // lane = offset a
    const int i1 = rlo + lane;
    for (int b = wave; b < nc; b += 4) {
        const double2 *col = St + b * sst;
        const double2 u = lane < nir ? col[1 + lane] : make_double2(0.0, 0.0);
        const double2 sum = range_sum(xch[wave], wave_scan_excl(u), ra, rb);
        if (lane < nr) {
            const double2 v = cadd(cadd(zm, col[0]), sum);
            store_r(in, i1 + P * b, (i1 + dr) + P * (b + dc), v, dr == 0 && dc == 0);
        }
    }
    stamp.done(fa, xcd_block(blockIdx.x, fa.n_items));
}

#undef ZR
#undef ZC

// ---------------------------------------------------------------------------
// Host launch helpers
// ---------------------------------------------------------------------------

hipError_t prepare_rec_kernels()
{
    static hipError_t status = [] {
        const void *fns[] = {reinterpret_cast<const void *>(&rec_main),
                             reinterpret_cast<const void *>(&rec_main_persistent),
                             reinterpret_cast<const void *>(&rec_finalize),
                             reinterpret_cast<const void *>(&rec_finalize_tab<16, 8>),
                             reinterpret_cast<const void *>(&rec_finalize_tab<4, 4>),
                             reinterpret_cast<const void *>(&rec_finalize_scan<true, 16>),
                             reinterpret_cast<const void *>(&rec_finalize_scan<false, 16>),
                             reinterpret_cast<const void *>(&rec_finalize_scan<true, 8>),
                             reinterpret_cast<const void *>(&rec_finalize_scan<false, 8>)};
        for (const void *f : fns) {
            hipError_t e = hipFuncSetAttribute(f, hipFuncAttributeMaxDynamicSharedMemorySize, 150 * 1024);
            if (e != hipSuccess) return e;
        }
        return hipSuccess;
    }();
    return status;
}

hipError_t launch_rec_main(const MainArgs &ma, int n_blocks, size_t lds_bytes, hipStream_t stream)
{
    hipError_t e = prepare_rec_kernels();
    if (e != hipSuccess) return e;
    hipLaunchKernelGGL(rec_main, dim3(n_blocks), dim3(kThreads), lds_bytes, stream, ma);
    return hipGetLastError();
}

hipError_t launch_rec_persistent(const MainArgs &ma, unsigned int *counter, int n_blocks, size_t lds_bytes,
                                 hipStream_t stream)
{
    hipError_t e = prepare_rec_kernels();
    if (e != hipSuccess) return e;
    hipLaunchKernelGGL(reset_counter, dim3(1), dim3(1), 0, stream, counter);
    e = hipGetLastError();
    if (e != hipSuccess) return e;
    hipLaunchKernelGGL(rec_main_persistent, dim3(n_blocks), dim3(kThreads), lds_bytes, stream, ma, counter);
    return hipGetLastError();
}

hipError_t launch_rec_finalize(const FinArgs &fa, int n_blocks, size_t lds_bytes, int variant,
                               hipStream_t stream)
{
    hipError_t e = prepare_rec_kernels();
    if (e != hipSuccess) return e;
    if (variant == kFinTable)
        hipLaunchKernelGGL((rec_finalize_tab<16, 8>), dim3(n_blocks), dim3(256), lds_bytes, stream, fa);
    else if (variant == kFinTableSmall)
        hipLaunchKernelGGL((rec_finalize_tab<4, 4>), dim3(n_blocks), dim3(256), lds_bytes, stream, fa);
    else if (variant == kFinScan && fa.use_inline)
        hipLaunchKernelGGL((rec_finalize_scan<true, 16>), dim3(n_blocks), dim3(256), lds_bytes, stream, fa);
    else if (variant == kFinScan)
        hipLaunchKernelGGL((rec_finalize_scan<false, 16>), dim3(n_blocks), dim3(256), lds_bytes, stream, fa);
    else if (variant == kFinScanSmall && fa.use_inline)
        hipLaunchKernelGGL((rec_finalize_scan<true, 8>), dim3(n_blocks), dim3(256), lds_bytes, stream, fa);
    else if (variant == kFinScanSmall)
        hipLaunchKernelGGL((rec_finalize_scan<false, 8>), dim3(n_blocks), dim3(256), lds_bytes, stream, fa);
    else
        hipLaunchKernelGGL(rec_finalize, dim3(n_blocks), dim3(64), lds_bytes, stream, fa);
    return hipGetLastError();
}

}  // namespace covest
