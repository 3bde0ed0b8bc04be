// adj_kernels.hip -- adjoint of the covariance map (kernels D1, D2) for gfx950.
//
// For a real loss L with G = dL/dR (PyTorch's convention for complex tensors)
// and H = G + G^H, the gradient with respect to A is
//     dA[r][c] = (1/K) sum_{dr, dc} A[r+dr][c+dc] * h_(dr,dc)(r, c),
//     h_(dr,dc)(r, c) = sum over window offsets (i1, j1) that can hold (r, c)
//                       of H[k(i1, j1)][k(i1+dr, j1+dc)],
// where the offsets range over i1 in [max(0, -dr, r-Kr+1), min(P-1, P-1-dr, r)]
// and likewise for j1 with Q and Kc.  Windows are recomputed from A; nothing
// from the forward call is stored.
//
// adj_tables     one workgroup per lag: T[i1][j1] = H[k(i1,j1)][k(i1+dr,j1+dc)]
//                and its 2-D inclusive prefix sums, FP64; from them the lag's
//                full sum and the weights of the frame's line jobs.
// interior       outputs whose offset ranges are complete (r in [P-1, Kr-1],
//                c in [Q-1, Kc-1]): h is the lag's full sum, so the output is a
//                2-D correlation of A with a (2P-1) x (2Q-1) kernel.  Windows
//                up to 16 x 16: adj_int_mfma on the FP64 matrix cores (below);
//                larger: adj_interior_tile, a ring walk over dc with 8
//                outputs per thread on the vector units.
// frame          the remaining outputs: an output row outside the interior
//                rows, next to interior columns, has weights that depend on
//                its row only, so a line of such outputs is again a
//                correlation with one kernel (row jobs, weights from the
//                tables kernel; column jobs likewise); outputs in a border
//                row and a border column get their own weights, four
//                prefix-sum reads per lag (corner jobs).
// Launches: tables, then either interior and frame together (adj_main) or
// adj_int_mfma followed by the frame and the output rows the matrix-core
// spans share (adj_frame_bnd).
#include <hip/hip_runtime.h>

#include <algorithm>

#include "adj_internal.hpp"

namespace covest {

__device__ __forceinline__ double2 dz() { return make_double2(0.0, 0.0); }

typedef double v4d __attribute__((ext_vector_type(4)));

// v_mfma_f64_16x16x4: lane l supplies A[l%16][l/16] and B[l/16][l%16];
// register r of lane l holds D[l/16 + 4r][l%16]
__device__ __forceinline__ v4d mfma64(double a, double b, v4d c)
{
    return __builtin_amdgcn_mfma_f64_16x16x4f64(a, b, c, 0, 0, 0);
}

// acc += a * w (no conjugate)
__device__ __forceinline__ void cmla(double2 &acc, const double2 a, const double2 w)
{
    acc.x = fma(a.x, w.x, acc.x);
    acc.x = fma(-a.y, w.y, acc.x);
    acc.y = fma(a.x, w.y, acc.y);
    acc.y = fma(a.y, w.x, acc.y);
}

__device__ __forceinline__ double2 g_entry(const AdjArgs &aa, int a, int b)
{
    const int64_t e = (int64_t)a * aa.ldg + b;
    if (aa.g_fp64) return static_cast<const double2 *>(aa.G)[e];
    const float2 g = static_cast<const float2 *>(aa.G)[e];
    return make_double2((double)g.x, (double)g.y);
}

// H[a][b] = G[a][b] + conj(G[b][a]); for an upper-only output the lower
// triangle of R is not a function of A, so only G's entries with column >= row
// count (G[a][b] for b >= a, G[b][a] for a >= b; both on the diagonal)
__device__ __forceinline__ double2 h_entry(const AdjArgs &aa, int a, int b)
{
    double2 h = dz();
    if (!aa.upper || b >= a) h = g_entry(aa, a, b);
    if (!aa.upper || a >= b) {
        const double2 g2 = g_entry(aa, b, a);
        h.x += g2.x;
        h.y -= g2.y;
    }
    return h;
}

// D1: per lag, the prefix-sum table S[i][j] = sum_{i' < i, j' < j} T[i'][j'],
// (P+1) x (Q+1), stored at tables + lag * (P+1)*(Q+1).
__global__ void __launch_bounds__(256) adj_tables(AdjArgs aa)
{
    extern __shared__ double2 tt[];
    const int P = aa.P, Q = aa.Q;
    const int lag = blockIdx.x;
    const int dr = lag / (2 * Q - 1) - (P - 1);
    const int dc = lag % (2 * Q - 1) - (Q - 1);
    const int w = Q + 1;
    for (int e = threadIdx.x; e < (P + 1) * w; e += 256) {
        const int i = e / w, j = e - i * w;
        double2 v = dz();
        if (i > 0 && j > 0) {
            const int i1 = i - 1, j1 = j - 1, i2 = i1 + dr, j2 = j1 + dc;
            if (i2 >= 0 && i2 < P && j2 >= 0 && j2 < Q) v = h_entry(aa, i1 + P * j1, i2 + P * j2);
        }
        tt[e] = v;
    }
    __syncthreads();
    // prefix along j for every row, then along i for every column (fixed order)
    for (int i = threadIdx.x; i <= P; i += 256) {
        double2 s = dz();
        for (int j = 0; j <= Q; ++j) {
            s.x += tt[i * w + j].x;
            s.y += tt[i * w + j].y;
            tt[i * w + j] = s;
        }
    }
    __syncthreads();
    for (int j = threadIdx.x; j <= Q; j += 256) {
        double2 s = dz();
        for (int i = 0; i <= P; ++i) {
            s.x += tt[i * w + j].x;
            s.y += tt[i * w + j].y;
            tt[i * w + j] = s;
        }
    }
    __syncthreads();
    double2 *out = reinterpret_cast<double2 *>(aa.tables) + (int64_t)lag * (P + 1) * w;
    for (int e = threadIdx.x; e < (P + 1) * w; e += 256) out[e] = tt[e];
    const int nl = (2 * P - 1) * (2 * Q - 1);
    if (threadIdx.x == 0) reinterpret_cast<double2 *>(aa.hfull)[lag] = tt[(P + 1) * w - 1];
    if (aa.ir0 >= aa.ir1) return;   // no interior: every output is a corner job on the tables

    // h of this lag for output (r, c), from the table in LDS; false when no
    // window offset holds (r, c)
    auto hlds = [&](int r, int c, double2 &h) {
        const int ilo = max(max(0, -dr), r - aa.Kr + 1), ihi = min(min(P - 1, P - 1 - dr), r);
        const int jlo = max(max(0, -dc), c - aa.Kc + 1), jhi = min(min(Q - 1, Q - 1 - dc), c);
        h = dz();
        if (ilo > ihi || jlo > jhi) return false;
        const double2 a = tt[(ihi + 1) * w + (jhi + 1)], b = tt[ilo * w + (jhi + 1)];
        const double2 c2 = tt[(ihi + 1) * w + jlo], d = tt[ilo * w + jlo];
        h = make_double2(a.x - b.x - c2.x + d.x, a.y - b.y - c2.y + d.y);
        return true;
    };
    const int nbr = aa.N - (aa.ir1 - aa.ir0), nbc = aa.M - (aa.ic1 - aa.ic0);
    auto band_row = [&](int k) { return k < aa.ir0 ? k : aa.ir1 + (k - aa.ir0); };
    auto band_col = [&](int k) { return k < aa.ic0 ? k : aa.ic1 + (k - aa.ic0); };
    // line jobs: a border row next to interior columns (column range full),
    // a border column next to interior rows
    double2 *wr = reinterpret_cast<double2 *>(aa.wrows), *wc = reinterpret_cast<double2 *>(aa.wcols);
    const int lag_t = (dc + Q - 1) * (2 * P - 1) + (dr + P - 1);
    for (int k = threadIdx.x; k < nbr + nbc; k += 256) {
        double2 h;
        if (k < nbr) {
            hlds(band_row(k), aa.ic0, h);
            wr[(int64_t)k * nl + lag] = h;
        } else {
            hlds(aa.ir0, band_col(k - nbr), h);
            wc[(int64_t)(k - nbr) * nl + lag_t] = h;
        }
    }
}

__device__ __forceinline__ void store_da(const AdjArgs &aa, int r, int c, double2 s)
{
    if (aa.normalize) {
        const double K = (double)aa.Kr * (double)aa.Kc;
        s.x = s.x / K;
        s.y = s.y / K;
    }
    const int64_t e = (int64_t)r * aa.ldda + c;
    if (aa.g_fp64) static_cast<double2 *>(aa.dA)[e] = s;
    else static_cast<float2 *>(aa.dA)[e] = make_float2((float)s.x, (float)s.y);
}

// h_(dr,dc)(r, c) from the lag's prefix table, in two steps so that loops can
// issue the reads of several lags before they use any: href names the four
// table entries (ok false when no window offset holds (r, c) for this lag; a
// non-empty offset range implies that A[r+dr][c+dc] lies inside A), hload
// reads them (zeros when not ok), hsum combines them.
struct HRef {
    const double2 *S;
    int e00, e01, e10, e11;
    bool ok;
};

__device__ __forceinline__ HRef href(const AdjArgs &aa, int r, int c, int dr, int dc)
{
    const int P = aa.P, Q = aa.Q, w = Q + 1;
    const int ilo = max(max(0, -dr), r - aa.Kr + 1), ihi = min(min(P - 1, P - 1 - dr), r);
    const int jlo = max(max(0, -dc), c - aa.Kc + 1), jhi = min(min(Q - 1, Q - 1 - dc), c);
    HRef f;
    f.ok = ilo <= ihi && jlo <= jhi;
    const int lag = (dr + P - 1) * (2 * Q - 1) + (dc + Q - 1);
    f.S = reinterpret_cast<const double2 *>(aa.tables) + (int64_t)lag * (P + 1) * w;
    f.e00 = (ihi + 1) * w + (jhi + 1);
    f.e01 = ilo * w + (jhi + 1);
    f.e10 = (ihi + 1) * w + jlo;
    f.e11 = ilo * w + jlo;
    return f;
}

__device__ __forceinline__ void hload(const HRef &f, double2 (&q)[4])
{
    if (f.ok) {
        q[0] = f.S[f.e00];
        q[1] = f.S[f.e01];
        q[2] = f.S[f.e10];
        q[3] = f.S[f.e11];
    } else {
        q[0] = q[1] = q[2] = q[3] = dz();
    }
}

// sum of T over the box from the inclusive-exclusive prefix table
__device__ __forceinline__ double2 hsum(const double2 (&q)[4])
{
    return make_double2(q[0].x - q[1].x - q[2].x + q[3].x, q[0].y - q[1].y - q[2].y + q[3].y);
}

__device__ __forceinline__ double2 block_sum_256(double2 v, double2 *red)
{
    // fixed order: a butterfly inside each wave, then the four waves in order
#pragma unroll
    for (int off = 32; off >= 1; off >>= 1) {
        v.x += __shfl_xor(v.x, off, 64);
        v.y += __shfl_xor(v.y, off, 64);
    }
    if (threadIdx.x % 64 == 0) red[threadIdx.x / 64] = v;
    __syncthreads();
    double2 s = red[0];
    for (int w = 1; w < 4; ++w) s = make_double2(s.x + red[w].x, s.y + red[w].y);
    return s;
}

// D2, frame.  Jobs, in block order: row jobs (border row r, up to kAdjFL
// interior columns), column jobs (border column c, up to kAdjFL interior
// rows), corner jobs (one output in a border row and a border column).
// A line job computes out[u] = sum_{x, y} T[x][u + y] * W[x][y] with
//   row job:    x = dr+P-1, y = dc+Q-1, T[x][j] = A[r+dr][c0-(Q-1)+j]
//   column job: x = dc+Q-1, y = dr+P-1, T[x][j] = A[r0-(P-1)+j][c+dc]
// staged in LDS in slabs of x; wave w takes x = w, w+4, ... of each slab and
// the four waves' sums are added in wave order.
__device__ void adj_frame_job(const AdjArgs &aa, double2 *sm, int64_t job)
{
    const int P = aa.P, Q = aa.Q, N = aa.N, M = aa.M;
    const int tid = threadIdx.x;
    const int nbc = M - (aa.ic1 - aa.ic0);
    const int nlc = (aa.ic1 - aa.ic0 + kAdjFL - 1) / kAdjFL;
    const int nlr = (aa.ir1 - aa.ir0 + kAdjFL - 1) / kAdjFL;
    const int64_t nrow_jobs = (int64_t)(N - (aa.ir1 - aa.ir0)) * nlc;
    const int64_t ncol_jobs = (int64_t)nbc * nlr;
    auto band_row = [&](int k) { return k < aa.ir0 ? k : aa.ir1 + (k - aa.ir0); };
    auto band_col = [&](int k) { return k < aa.ic0 ? k : aa.ic1 + (k - aa.ic0); };

    if (job >= nrow_jobs + ncol_jobs) {
        // corner job: one output with its own weights, lags spread over the block
        const int64_t k = job - nrow_jobs - ncol_jobs;
        const int r = band_row((int)(k / nbc)), c = band_col((int)(k % nbc));
        const int ndc = 2 * Q - 1, nl = (2 * P - 1) * ndc;
        double2 s = dz();
        for (int l0 = tid; l0 < nl; l0 += kAdjBatch * 256) {
            // the reads of kAdjBatch lags go out before any is used
            double2 q[kAdjBatch][4];
            float2 av[kAdjBatch];
            bool ok[kAdjBatch];
#pragma unroll
            for (int u = 0; u < kAdjBatch; ++u) {
                const int l = min(l0 + u * 256, nl - 1);
                const int dr = l / ndc - (P - 1), dc = l % ndc - (Q - 1);
                const HRef f = href(aa, r, c, dr, dc);
                ok[u] = f.ok && l0 + u * 256 < nl;
                // unconditional loads (a branch would wait for each): the
                // output's own element stands in where the lag has no window
                const int ar = f.ok ? r + dr : r, ac = f.ok ? c + dc : c;
                av[u] = aa.A[(int64_t)ar * aa.lda + ac];
                hload(f, q[u]);
            }
#pragma unroll
            for (int u = 0; u < kAdjBatch; ++u)
                if (ok[u]) cmla(s, make_double2(av[u].x, av[u].y), hsum(q[u]));
        }
        s = block_sum_256(s, sm);
        if (tid == 0) store_da(aa, r, c, s);
        return;
    }

    const bool rowjob = job < nrow_jobs;
    int r0, c0, len, band_k;
    if (rowjob) {
        const int k = (int)(job / nlc), ch = (int)(job % nlc);
        band_k = k;
        r0 = band_row(k);
        c0 = aa.ic0 + ch * kAdjFL;
        len = min(kAdjFL, aa.ic1 - c0);
    } else {
        const int64_t j = job - nrow_jobs;
        const int k = (int)(j / nlr), ch = (int)(j % nlr);
        band_k = k;
        c0 = band_col(k);
        r0 = aa.ir0 + ch * kAdjFL;
        len = min(kAdjFL, aa.ir1 - r0);
    }
    // the weights of every output of the line are those of an interior
    // column (row job) or an interior row (column job).  Thread (xl, og)
    // takes weight row x = xs + xl of each slab and the kAdjRing consecutive
    // outputs from kAdjRing og, with a ring of kAdjRing A values along y;
    // the threads' sums are added in x order at the end.
    constexpr int RG = kAdjRing;
    const int X = rowjob ? 2 * P - 1 : 2 * Q - 1, Y = rowjob ? 2 * Q - 1 : 2 * P - 1;
    const int Yp = (Y + RG - 1) / RG * RG;            // weights zero past Y
    const int wst = Yp + 1, span = kAdjFL + Yp, stride = span | 1;
    const int XS = max(1, min(min(X, 256 / (kAdjFL / RG)), aa.frame_lds / (int)adj_line_row_bytes(Y)));
    double2 *Wt = sm;                                               // XS x wst
    float2 *Tt = reinterpret_cast<float2 *>(sm + (size_t)XS * wst);   // XS x stride
    const int xl = tid % 32, og = tid / 32;
    double2 acc[RG];
#pragma unroll
    for (int u = 0; u < RG; ++u) acc[u] = dz();
    for (int xs = 0; xs < X; xs += XS) {
        const int xn = min(XS, X - xs);
        // weights (the tables kernel's, in this job's (x, y) order: the slab
        // is one contiguous run) and A values; the reads of a batch go out
        // before any store
        const double2 *wsrc = reinterpret_cast<const double2 *>(rowjob ? aa.wrows : aa.wcols) +
                              (int64_t)band_k * X * Y + (int64_t)xs * Y;
        for (int e0 = tid; e0 < xn * Yp; e0 += 2 * kAdjBatch * 256) {
            double2 q[2 * kAdjBatch];
#pragma unroll
            for (int u = 0; u < 2 * kAdjBatch; ++u) {
                const int e = min(e0 + u * 256, xn * Yp - 1);
                const int xr = e / Yp, y = e - xr * Yp;
                q[u] = wsrc[xr * Y + min(y, Y - 1)];
                if (y >= Y) q[u] = dz();
            }
#pragma unroll
            for (int u = 0; u < 2 * kAdjBatch; ++u) {
                const int e = e0 + u * 256;
                if (e < xn * Yp) Wt[(e / Yp) * wst + e % Yp] = q[u];
            }
        }
        for (int e0 = tid; e0 < xn * span; e0 += 2 * kAdjBatch * 256) {
            float2 v[2 * kAdjBatch];
            int dst[2 * kAdjBatch];
#pragma unroll
            for (int u = 0; u < 2 * kAdjBatch; ++u) {
                // neighbouring threads read neighbouring columns of A
                const int e = min(e0 + u * 256, xn * span - 1);
                int xr, j, ar, ac;
                if (rowjob) {
                    xr = e / span;
                    j = e - xr * span;
                    ar = r0 + xs + xr - (P - 1);
                    ac = c0 - (Q - 1) + j;
                } else {
                    j = e / xn;
                    xr = e - j * xn;
                    ar = r0 - (P - 1) + j;
                    ac = c0 + xs + xr - (Q - 1);
                }
                dst[u] = e0 + u * 256 < xn * span ? xr * stride + j : -1;
                // unconditional load of a clamped element, zeroed outside A
                // and past the last y (its weights are zero; a non-finite A
                // there must not leak in)
                const bool in = ar >= 0 && ar < N && ac >= 0 && ac < M && j < kAdjFL + Y - 1;
                v[u] = aa.A[(int64_t)min(max(ar, 0), N - 1) * aa.lda + min(max(ac, 0), M - 1)];
                if (!in) v[u] = make_float2(0.f, 0.f);
            }
#pragma unroll
            for (int u = 0; u < 2 * kAdjBatch; ++u)
                if (dst[u] >= 0) Tt[dst[u]] = v[u];
        }
        __syncthreads();
        if (xl < xn) {
            // output RG og + u reads T[xl][RG og + u + y]
            const float2 *trow = Tt + xl * stride + RG * og;
            const double2 *wrow = Wt + xl * wst;
            double2 ring[RG];
#pragma unroll
            for (int k = 0; k < RG - 1; ++k) ring[k] = make_double2(trow[k].x, trow[k].y);
            for (int b = 0; b < Yp; b += RG) {
#pragma unroll
                for (int v = 0; v < RG; ++v) {
                    const float2 an = trow[b + v + RG - 1];
                    ring[(v + RG - 1) % RG] = make_double2(an.x, an.y);
                    const double2 w = wrow[b + v];
#pragma unroll
                    for (int u = 0; u < RG; ++u) cmla(acc[u], ring[(v + u) % RG], w);
                }
            }
        }
        __syncthreads();
    }
    // sums over the x rows, in x order (rows past X hold zeros)
    const int xrows = min(XS, X);
    if (xl < xrows) {
#pragma unroll
        for (int u = 0; u < RG; ++u) sm[xl * kAdjFL + RG * og + u] = acc[u];
    }
    __syncthreads();
    if (tid < len) {
        double2 s = sm[tid];
        for (int x = 1; x < xrows; ++x) s = make_double2(s.x + sm[x * kAdjFL + tid].x, s.y + sm[x * kAdjFL + tid].y);
        if (rowjob) store_da(aa, r0, c0 + tid, s);
        else store_da(aa, r0 + tid, c0, s);
    }
}

// D2, interior: workgroup tile of kAdjTR rows x kAdjTC columns of outputs.
// Thread (row, kAdjRing-column chunk, dr group): ring over dc, kAdjRing FP64
// accumulators; the dr groups are summed through LDS in a fixed order.
__device__ void adj_interior_tile(const AdjArgs &aa, double2 *sm, int tile)
{
    const int P = aa.P, Q = aa.Q;
    const int ndc = aa.ndc;                        // dc steps padded to a multiple of 16
    const int nlag_c = 2 * Q - 1;
    const int tiles_c = (aa.ic1 - aa.ic0 + kAdjTC - 1) / kAdjTC;
    const int r0 = aa.ir0 + (tile / tiles_c) * kAdjTR;
    const int c0 = aa.ic0 + (tile % tiles_c) * kAdjTC;
    const int rows = kAdjTR + 2 * (P - 1);
    const int cols = kAdjTC + ndc;                 // columns c0-(Q-1) .. c0+TC+ndc-(Q-1)
    const int stride = cols | 1;
    // weights (FP64) first, then the A tile kept as complex64 (widened on read)
    double2 *Wt = sm;                              // (2P-1) x ndc, zero padded
    float2 *At = reinterpret_cast<float2 *>(sm + (2 * P - 1) * ndc);   // rows x stride
    for (int e = threadIdx.x; e < rows * cols; e += 256) {
        const int i = e / cols, j = e - i * cols;
        const int ar = r0 - (P - 1) + i, ac = c0 - (Q - 1) + j;
        float2 v = make_float2(0.f, 0.f);
        if (ar >= 0 && ar < aa.N && ac >= 0 && ac < aa.M) v = aa.A[(int64_t)ar * aa.lda + ac];
        At[i * stride + j] = v;
    }
    for (int e = threadIdx.x; e < (2 * P - 1) * ndc; e += 256) {
        const int i = e / ndc, j = e - i * ndc;
        Wt[e] = j < nlag_c ? reinterpret_cast<const double2 *>(aa.hfull)[i * nlag_c + j] : dz();
    }
    __syncthreads();

    const int lr = threadIdx.x % kAdjTR;
    constexpr int RG = kAdjRing;
    const int ch = (threadIdx.x / kAdjTR) % (kAdjTC / RG);
    const int grp = threadIdx.x / (kAdjTR * (kAdjTC / RG));
    constexpr int ngrp = 256 / (kAdjTR * (kAdjTC / RG));
    const int ndr = 2 * P - 1;
    const int dr0 = (int)((int64_t)grp * ndr / ngrp), dr1 = (int)((int64_t)(grp + 1) * ndr / ngrp);

    double2 acc[RG];
#pragma unroll
    for (int u = 0; u < RG; ++u) acc[u] = dz();
    for (int di = dr0; di < dr1; ++di) {           // di = dr + P - 1
        // output (lr, RG*ch + u) reads A[lr + di][RG*ch + u + dj] (tile coordinates)
        const float2 *arow = At + (lr + di) * stride + RG * ch;
        const double2 *wrow = Wt + di * ndc;
        double2 ring[RG];
#pragma unroll
        for (int k = 0; k < RG - 1; ++k) ring[k] = make_double2(arow[k].x, arow[k].y);
        for (int b = 0; b < ndc; b += RG) {
#pragma unroll
            for (int v = 0; v < RG; ++v) {
                // dj = b + v; outputs u need arow[u + dj]
                const float2 an = arow[b + v + RG - 1];
                ring[(v + RG - 1) % RG] = make_double2(an.x, an.y);
                const double2 wv = wrow[b + v];
                // the padding lags dj >= 2Q-1 (zero weights) add nothing, and
                // a non-finite A value there must not reach a product
                if (b + v < nlag_c) {
#pragma unroll
                    for (int u = 0; u < RG; ++u) cmla(acc[u], ring[(v + u) % RG], wv);
                }
            }
        }
    }
    __syncthreads();
    // fixed-order sum over the dr groups
    double2 *red = sm;
#pragma unroll
    for (int u = 0; u < RG; ++u) red[threadIdx.x * RG + u] = acc[u];
    __syncthreads();
    constexpr int per_grp = kAdjTR * (kAdjTC / RG);
    for (int e = threadIdx.x; e < kAdjTR * kAdjTC; e += 256) {
        const int row = e / kAdjTC, col = e - row * kAdjTC;
        const int r = r0 + row, c = c0 + col;
        if (r >= aa.ir1 || c >= aa.ic1) continue;
        const int tid0 = row + kAdjTR * (col / RG);
        double2 s = dz();
        for (int g = 0; g < ngrp; ++g) {
            const double2 v = red[(tid0 + g * per_grp) * RG + (col % RG)];
            s.x += v.x;
            s.y += v.y;
        }
        store_da(aa, r, c, s);
    }
}

// D2, interior, on the FP64 matrix cores.  With y = r - (P-1), x = c - (Q-1)
// and the lag's full sum W[a][b] (a = dr + P-1, b = dc + Q-1), an interior
// output is
//     out(y, x) = sum_a Y_{y+a}[a][x],   Y_rho[a][x] = sum_b W[a][b] * A[rho][x + b]:
// each input row rho gives the product of the weights (2P-1 rows a by 2Q-1
// columns b) with a Hankel block of its own values (b by x), which is a dense
// 16 x 16 x 4 tile product with no padding but the last k-step and tile row.
// Row rho's product feeds outputs y = rho - a; a wave sums them into a ring
// of output rows in LDS.  The weights stay in registers for the whole launch
// (first operand: lane l holds W[16 mt + l%16][4 ks + l/16]); the second
// operand comes straight from A (lane l reads A[rho][x0 + l%16 + 4 ks + l/16]).
// Complex products take three real products (the three-multiplication form):
//     K1 += (Wr + Wi) * Xr,  K2 += Wr * (Xi - Xr),  K3 += Wi * (Xr + Xi),
//     Re Y = K1 - K3,  Im Y = K1 + K2.
// A workgroup walks kAdjMSpan input rows of one 16-column tile, one
// kAdjMRows slice per wave; the waves' rings are added in wave order.  Output
// rows whose 2P-1 input rows all lie in the workgroup's span are stored; the
// 2P-2 rows on each side that a neighbouring span shares go to `bnd`, and
// adj_frame_bnd adds the two halves (one addition: the same bits in either
// order).
template <int MT, int KS>
__device__ void adj_int_block(const AdjArgs &aa, double2 *ring, int blk)
{
    constexpr int NT = kAdjMWaves * 64;
    const int P = aa.P, N = aa.N, M = aa.M;
    const int H = 2 * P - 2;                        // output rows an input row reaches below it
    const int nlr = 2 * P - 1, nlc = 2 * aa.Q - 1;
    const int lane = threadIdx.x & 63;
    const int wave = __builtin_amdgcn_readfirstlane(threadIdx.x >> 6);
    const int n = lane & 15, g = lane >> 4;
    const int tile = blk % aa.mtiles, range = blk / aa.mtiles;
    const int x0 = 16 * tile;
    const int rho0 = kAdjMSpan * range;
    const int rw = rho0 + kAdjMRows * wave;         // this wave's first input row
    const int brows = kAdjMRows + H;                // ring rows: outputs rw - H .. rw + kAdjMRows - 1
    // plus one row that takes the padding rows a >= 2P-1 of the tiles
    double2 *buf = ring + (size_t)wave * (brows + 1) * 16;
    // the wave's input rows, staged once: kAdjMRows rows of the columns
    // x0 .. x0 + 4 KS + 15 (clamped to M - 1; those feed only dropped outputs)
    constexpr int XW = 4 * KS + 16;
    float2 *xs = reinterpret_cast<float2 *>(ring + (size_t)kAdjMWaves * (brows + 1) * 16) + (size_t)wave * kAdjMRows * XW;

    double w1[MT][KS], w2[MT][KS], w3[MT][KS];
    const double2 *hf = reinterpret_cast<const double2 *>(aa.hfull);
#pragma unroll
    for (int mt = 0; mt < MT; ++mt)
#pragma unroll
        for (int ks = 0; ks < KS; ++ks) {
            const int a = 16 * mt + n, b = 4 * ks + g;
            double2 w = dz();
            if (a < nlr && b < nlc) w = hf[a * nlc + b];
            w1[mt][ks] = w.x + w.y;
            w2[mt][ks] = w.x;
            w3[mt][ks] = w.y;
        }
    for (int e = lane; e < (brows + 1) * 16; e += 64) buf[e] = dz();

    // ring row of register r of tile mt (a = 16 mt + g + 4 r) at step t:
    // t - a + H, or the padding row
    int rrow[MT][4];
#pragma unroll
    for (int mt = 0; mt < MT; ++mt)
#pragma unroll
        for (int r = 0; r < 4; ++r) {
            const int a = 16 * mt + g + 4 * r;
            rrow[mt][r] = a < nlr ? (H - a) * 16 + n : brows * 16 + n - (1 << 20);
        }

    const int rows_here = min(kAdjMRows, N - rw);
    {
        // all loads of the staging go out before any store
        constexpr int NL = (kAdjMRows * XW + 63) / 64;
        float2 v[NL];
#pragma unroll
        for (int k = 0; k < NL; ++k) {
            const int e = min(lane + 64 * k, kAdjMRows * XW - 1);
            const int rr = min(e / XW, max(rows_here - 1, 0)), cc = min(x0 + e % XW, M - 1);
            v[k] = aa.A[(int64_t)min(rw + rr, N - 1) * aa.lda + cc];
        }
#pragma unroll
        for (int k = 0; k < NL; ++k)
            if (lane + 64 * k < kAdjMRows * XW) xs[lane + 64 * k] = v[k];
    }
    __builtin_amdgcn_fence(__ATOMIC_RELEASE, "wavefront");
    __builtin_amdgcn_wave_barrier();
    __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "wavefront");

    // second operand of k-step ks: staged column n + 4 ks + g; past the last
    // column b the value is zeroed (its weights are zero, and a non-finite A
    // must not leak in)
    bool pad[KS];
#pragma unroll
    for (int ks = 0; ks < KS; ++ks) pad[ks] = 4 * ks + g >= nlc;
    const float2 *xl = xs + n + g;
    float2 xv[KS];
#pragma unroll
    for (int ks = 0; ks < KS; ++ks) xv[ks] = xl[4 * ks];
    for (int t = 0; t < rows_here; ++t) {
        float2 xn[KS];
        const float2 *xrow = xl + min(t + 1, kAdjMRows - 1) * XW;   // the last row rereads a staged row
#pragma unroll
        for (int ks = 0; ks < KS; ++ks) xn[ks] = xrow[4 * ks];
        v4d acc[MT][3];
#pragma unroll
        for (int mt = 0; mt < MT; ++mt)
#pragma unroll
            for (int c = 0; c < 3; ++c) acc[mt][c] = (v4d){0.0, 0.0, 0.0, 0.0};
#pragma unroll
        for (int ks = 0; ks < KS; ++ks) {
            const double xr = pad[ks] ? 0.0 : (double)xv[ks].x;
            const double xi = pad[ks] ? 0.0 : (double)xv[ks].y;
            const double x2 = xi - xr, x3 = xr + xi;
#pragma unroll
            for (int mt = 0; mt < MT; ++mt) {
                acc[mt][0] = mfma64(w1[mt][ks], xr, acc[mt][0]);
                acc[mt][1] = mfma64(w2[mt][ks], x2, acc[mt][1]);
                acc[mt][2] = mfma64(w3[mt][ks], x3, acc[mt][2]);
            }
        }
        // output y = rw + t - a sits in ring row t - a + H: all ring reads of
        // the step first (one wait), then the writes
        double2 *dst[MT][4];
        double2 cur[MT][4];
#pragma unroll
        for (int mt = 0; mt < MT; ++mt)
#pragma unroll
            for (int r = 0; r < 4; ++r) {
                const int ro = rrow[mt][r];
                dst[mt][r] = buf + (ro >= 0 ? ro + t * 16 : ro + (1 << 20));
                cur[mt][r] = *dst[mt][r];
            }
#pragma unroll
        for (int mt = 0; mt < MT; ++mt)
#pragma unroll
            for (int r = 0; r < 4; ++r) {
                double2 v = cur[mt][r];
                v.x += acc[mt][0][r] - acc[mt][2][r];
                v.y += acc[mt][0][r] + acc[mt][1][r];
                *dst[mt][r] = v;
            }
#pragma unroll
        for (int ks = 0; ks < KS; ++ks) xv[ks] = xn[ks];
    }
    __syncthreads();

    // the workgroup's outputs y in [rho0 - H, rho0 + kAdjMSpan)
    const int xpad = 16 * aa.mtiles;
    for (int e = threadIdx.x; e < (kAdjMSpan + H) * 16; e += NT) {
        const int row = e >> 4, nn = e & 15;
        const int y = rho0 - H + row, x = x0 + nn;
        if (y < 0 || y >= aa.ny || x >= aa.nx) continue;
        double2 s = dz();
        for (int w = 0; w < kAdjMWaves; ++w) {
            const int br = y - (rho0 + kAdjMRows * w - H);
            if (br >= 0 && br < brows) {
                const double2 v = ring[((size_t)w * (brows + 1) + br) * 16 + nn];
                s.x += v.x;
                s.y += v.y;
            }
        }
        if (range > 0 && y < rho0) {
            // shared with the span above: its side 1 of boundary range - 1
            const int br = y - (rho0 - H);
            reinterpret_cast<double2 *>(aa.bnd)[((int64_t)((range - 1) * 2 + 1) * H + br) * xpad + x] = s;
        } else if (y + H >= rho0 + kAdjMSpan) {
            // shared with the span below: side 0 of boundary range
            const int br = y - (rho0 + kAdjMSpan - H);
            reinterpret_cast<double2 *>(aa.bnd)[((int64_t)(range * 2) * H + br) * xpad + x] = s;
        } else {
            store_da(aa, y + P - 1, x + aa.Q - 1, s);
        }
    }
}

// The output rows two neighbouring spans share: boundary b holds rows
// y in [kAdjMSpan (b+1) - H, kAdjMSpan (b+1)).
__device__ void adj_bnd_rows(const AdjArgs &aa, int blk, int nblk)
{
    const int H = 2 * aa.P - 2;
    const int xpad = 16 * aa.mtiles;
    // one thread per output of the boundary rows (the planner keeps the
    // count below 2^31)
    const int total = (aa.mranges - 1) * H * aa.nx;
    const double2 *bd = reinterpret_cast<const double2 *>(aa.bnd);
    for (int e = blk * 256 + threadIdx.x; e < total; e += nblk * 256) {
        const int x = e % aa.nx;
        const int q = e / aa.nx;
        const int br = q % H, b = q / H;
        const int y = kAdjMSpan * (b + 1) - H + br;
        if (y >= aa.ny) continue;
        const double2 u = bd[((int64_t)(b * 2) * H + br) * xpad + x];
        const double2 v = bd[((int64_t)(b * 2 + 1) * H + br) * xpad + x];
        store_da(aa, y + aa.P - 1, x + aa.Q - 1, make_double2(u.x + v.x, u.y + v.y));
    }
}

// D2, matrix-core interior: one workgroup per span of one output tile.
template <int MT, int KS>
__global__ void __launch_bounds__(kAdjMWaves * 64) adj_int_mfma(AdjArgs aa)
{
    extern __shared__ double2 sm[];
    adj_int_block<MT, KS>(aa, sm, blockIdx.x);
}

// After the matrix-core interior: blocks [0, n_frame) take the frame's jobs,
// the rest add up the output rows two spans share.
__global__ void __launch_bounds__(256) adj_frame_bnd(AdjArgs aa, int n_frame)
{
    extern __shared__ double2 sm[];
    if ((int)blockIdx.x < n_frame) adj_frame_job(aa, sm, (int64_t)blockIdx.x);
    else adj_bnd_rows(aa, (int)blockIdx.x - n_frame, (int)gridDim.x - n_frame);
}

// D2 in one launch: blocks [0, n_interior) take the interior tiles, the rest
// the frame's jobs, so that the frame's many short jobs run beside the
// interior's long ones instead of after them.
__global__ void __launch_bounds__(256) adj_main(AdjArgs aa, int n_interior)
{
    extern __shared__ double2 sm[];
    if ((int)blockIdx.x < n_interior) adj_interior_tile(aa, sm, blockIdx.x);
    else adj_frame_job(aa, sm, (int64_t)blockIdx.x - n_interior);
}

hipError_t launch_adjoint(const AdjArgs &aa_in, int n_lags, size_t lds_tables, int n_interior_blocks,
                          size_t lds_interior, int64_t n_frame_jobs, hipStream_t s)
{
    // One launch holds both kinds of blocks, so they share its LDS size: the
    // interior's when there are interior tiles (the frame's slabs adapt to it;
    // one slab of weights and A columns and the final 256-entry sum must fit),
    // else the frame's own.
    AdjArgs aa = aa_in;
    const int P = aa.P, Q = aa.Q;
    const size_t slab_max = std::max(adj_line_row_bytes(2 * Q - 1), adj_line_row_bytes(2 * P - 1));
    const size_t frame_min = std::max<size_t>(256 * 16, slab_max);
    size_t lds = n_interior_blocks > 0 ? lds_interior : 0;
    if (n_frame_jobs > 0) lds = n_interior_blocks > 0 ? std::max(lds, frame_min) : (size_t)kAdjFrameLds;
    aa.frame_lds = (int)lds;
    static const hipError_t attr = [] {
        hipError_t e = hipFuncSetAttribute(reinterpret_cast<const void *>(&adj_main),
                                           hipFuncAttributeMaxDynamicSharedMemorySize, 160 * 1024);
        if (e == hipSuccess)
            e = hipFuncSetAttribute(reinterpret_cast<const void *>(&adj_tables),
                                    hipFuncAttributeMaxDynamicSharedMemorySize, 160 * 1024);
        return e;
    }();
    if (attr != hipSuccess) return attr;
    hipLaunchKernelGGL(adj_tables, dim3(n_lags), dim3(256), lds_tables, s, aa);
    hipError_t e = hipGetLastError();
    if (e != hipSuccess) return e;
    const int64_t n = n_interior_blocks + n_frame_jobs;
    if (n > 0) {
        hipLaunchKernelGGL(adj_main, dim3((unsigned)n), dim3(256), lds, s, aa, n_interior_blocks);
        e = hipGetLastError();
    }
    return e;
}

template <int MT, int KS>
static hipError_t launch_int_mt_ks(const AdjArgs &aa, size_t lds, hipStream_t s)
{
    static const hipError_t attr = hipFuncSetAttribute(reinterpret_cast<const void *>(&adj_int_mfma<MT, KS>),
                                                       hipFuncAttributeMaxDynamicSharedMemorySize, 160 * 1024);
    if (attr != hipSuccess) return attr;
    hipLaunchKernelGGL((adj_int_mfma<MT, KS>), dim3((unsigned)(aa.mtiles * aa.mranges)), dim3(kAdjMWaves * 64), lds,
                       s, aa);
    return hipGetLastError();
}

template <int MT>
static hipError_t launch_int_mt(const AdjArgs &aa, size_t lds, hipStream_t s)
{
    switch ((2 * aa.Q - 1 + 3) / 4) {
    case 1: return launch_int_mt_ks<MT, 1>(aa, lds, s);
    case 2: return launch_int_mt_ks<MT, 2>(aa, lds, s);
    case 3: return launch_int_mt_ks<MT, 3>(aa, lds, s);
    case 4: return launch_int_mt_ks<MT, 4>(aa, lds, s);
    case 5: return launch_int_mt_ks<MT, 5>(aa, lds, s);
    case 6: return launch_int_mt_ks<MT, 6>(aa, lds, s);
    case 7: return launch_int_mt_ks<MT, 7>(aa, lds, s);
    case 8: return launch_int_mt_ks<MT, 8>(aa, lds, s);
    default: return hipErrorInvalidValue;
    }
}

hipError_t launch_adjoint_mfma(const AdjArgs &aa_in, int n_lags, size_t lds_tables, int64_t n_frame_jobs,
                               size_t lds_frame, hipStream_t s)
{
    AdjArgs aa = aa_in;
    aa.frame_lds = (int)lds_frame;
    // set once (a function-local static: thread-safe initialisation)
    static const hipError_t attr = [] {
        const void *fns[] = {reinterpret_cast<const void *>(&adj_tables), reinterpret_cast<const void *>(&adj_frame_bnd)};
        for (const void *f : fns) {
            const hipError_t e = hipFuncSetAttribute(f, hipFuncAttributeMaxDynamicSharedMemorySize, 160 * 1024);
            if (e != hipSuccess) return e;
        }
        return hipSuccess;
    }();
    if (attr != hipSuccess) return attr;
    hipLaunchKernelGGL(adj_tables, dim3(n_lags), dim3(256), lds_tables, s, aa);
    hipError_t e = hipGetLastError();
    if (e != hipSuccess) return e;
    // tile rows MT = ceil((2P-1)/16), k-steps KS = ceil((2Q-1)/4)
    const size_t lds_int = adj_mfma_lds(aa.P, aa.Q);
    if (2 * aa.P - 1 <= 16) e = launch_int_mt<1>(aa, lds_int, s);
    else if (2 * aa.P - 1 <= 32) e = launch_int_mt<2>(aa, lds_int, s);
    else e = hipErrorInvalidValue;
    if (e != hipSuccess) return e;
    const int64_t nbnd = (int64_t)(aa.mranges - 1) * (2 * aa.P - 2) * aa.nx;
    const int64_t nb = n_frame_jobs + std::min<int64_t>((nbnd + 255) / 256, 1024);
    if (nb > 0) {
        hipLaunchKernelGGL(adj_frame_bnd, dim3((unsigned)nb), dim3(256), lds_frame, s, aa, (int)n_frame_jobs);
        e = hipGetLastError();
    }
    return e;
}

}  // namespace covest
