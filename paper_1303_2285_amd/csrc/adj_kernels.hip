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
//                and its 2-D inclusive prefix sums, FP64.
// adj_interior   outputs whose offset ranges are complete (r in [P-1, Kr-1],
//                c in [Q-1, Kc-1]): h is the lag's full sum, so the output is a
//                2-D correlation of A with a (2P-1) x (2Q-1) kernel; ring walk
//                over dc with 16 outputs per thread, FP64 accumulators.
// adj_frame      the remaining outputs, h taken from the prefix sums (4 reads):
//                an output row outside the interior rows, next to interior
//                columns, has weights that depend on its row only, so a line
//                of such outputs is again a correlation with one kernel (row
//                jobs; column jobs likewise); outputs in a border row and a
//                border column get their own weights (corner jobs).
#include <hip/hip_runtime.h>

#include <algorithm>

#include "adj_internal.hpp"

namespace covest {

__device__ __forceinline__ double2 dz() { return make_double2(0.0, 0.0); }

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
    if (threadIdx.x == 0) reinterpret_cast<double2 *>(aa.hfull)[lag] = tt[(P + 1) * w - 1];
}

__device__ __forceinline__ double2 box(const double2 *S, int w, int ilo, int ihi, int jlo, int jhi)
{
    // sum of T over [ilo, ihi] x [jlo, jhi] from the inclusive-exclusive prefix table
    const double2 a = S[(ihi + 1) * w + (jhi + 1)];
    const double2 b = S[ilo * w + (jhi + 1)];
    const double2 c = S[(ihi + 1) * w + jlo];
    const double2 d = S[ilo * w + jlo];
    return make_double2(a.x - b.x - c.x + d.x, a.y - b.y - c.y + d.y);
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

// h_(dr,dc)(r, c) from the lag's prefix table; false (and zero) when no
// window offset holds (r, c) for this lag.  A non-empty offset range implies
// that A[r+dr][c+dc] lies inside A.
__device__ __forceinline__ bool hbox(const AdjArgs &aa, int r, int c, int dr, int dc, double2 &h)
{
    const int P = aa.P, Q = aa.Q;
    const int ilo = max(max(0, -dr), r - aa.Kr + 1), ihi = min(min(P - 1, P - 1 - dr), r);
    const int jlo = max(max(0, -dc), c - aa.Kc + 1), jhi = min(min(Q - 1, Q - 1 - dc), c);
    h = dz();
    if (ilo > ihi || jlo > jhi) return false;
    const int lag = (dr + P - 1) * (2 * Q - 1) + (dc + Q - 1);
    const double2 *S = reinterpret_cast<const double2 *>(aa.tables) + (int64_t)lag * (P + 1) * (Q + 1);
    h = box(S, Q + 1, ilo, ihi, jlo, jhi);
    return true;
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
        for (int l = tid; l < nl; l += 256) {
            const int dr = l / ndc - (P - 1), dc = l % ndc - (Q - 1);
            double2 h;
            if (hbox(aa, r, c, dr, dc, h)) {
                const float2 av = aa.A[(int64_t)(r + dr) * aa.lda + (c + dc)];
                cmla(s, make_double2(av.x, av.y), h);
            }
        }
        s = block_sum_256(s, sm);
        if (tid == 0) store_da(aa, r, c, s);
        return;
    }

    const bool rowjob = job < nrow_jobs;
    int r0, c0, len;
    if (rowjob) {
        const int k = (int)(job / nlc), ch = (int)(job % nlc);
        r0 = band_row(k);
        c0 = aa.ic0 + ch * kAdjFL;
        len = min(kAdjFL, aa.ic1 - c0);
    } else {
        const int64_t j = job - nrow_jobs;
        const int k = (int)(j / nlr), ch = (int)(j % nlr);
        c0 = band_col(k);
        r0 = aa.ir0 + ch * kAdjFL;
        len = min(kAdjFL, aa.ir1 - r0);
    }
    // the weights of every output of the line: those of an interior column
    // (row job) or an interior row (column job)
    const int wr = rowjob ? r0 : aa.ir0, wc = rowjob ? aa.ic0 : c0;
    const int X = rowjob ? 2 * P - 1 : 2 * Q - 1, Y = rowjob ? 2 * Q - 1 : 2 * P - 1;
    const int span = kAdjFL + Y - 1;
    const int stride = span | 1;
    const int XS = max(1, min(X, aa.frame_lds / (Y * 16 + stride * 8)));
    double2 *Wt = sm;                                               // XS x Y
    float2 *Tt = reinterpret_cast<float2 *>(sm + (size_t)XS * Y);   // XS x stride
    const int u = tid % 64, wv = tid / 64;
    double2 acc0 = dz(), acc1 = dz();
    for (int xs = 0; xs < X; xs += XS) {
        const int xn = min(XS, X - xs);
        for (int e = tid; e < xn * Y; e += 256) {
            const int x = xs + e / Y, y = e % Y;
            const int dr = (rowjob ? x : y) - (P - 1), dc = (rowjob ? y : x) - (Q - 1);
            double2 h;
            hbox(aa, wr, wc, dr, dc, h);
            Wt[e] = h;
        }
        for (int e = tid; e < xn * span; e += 256) {
            // neighbouring threads read neighbouring columns of A
            int xl, j, ar, ac;
            if (rowjob) {
                xl = e / span;
                j = e - xl * span;
                ar = r0 + xs + xl - (P - 1);
                ac = c0 - (Q - 1) + j;
            } else {
                j = e / xn;
                xl = e - j * xn;
                ar = r0 - (P - 1) + j;
                ac = c0 + xs + xl - (Q - 1);
            }
            float2 v = make_float2(0.f, 0.f);
            if (ar >= 0 && ar < N && ac >= 0 && ac < M) v = aa.A[(int64_t)ar * aa.lda + ac];
            Tt[xl * stride + j] = v;
        }
        __syncthreads();
        for (int xl = wv; xl < xn; xl += 4) {
            const float2 *trow = Tt + xl * stride + u;
            const double2 *wrow = Wt + xl * Y;
            int y = 0;
            for (; y + 1 < Y; y += 2) {
                const float2 t0 = trow[y], t1 = trow[y + 1];
                cmla(acc0, make_double2(t0.x, t0.y), wrow[y]);
                cmla(acc1, make_double2(t1.x, t1.y), wrow[y + 1]);
            }
            if (y < Y) {
                const float2 t0 = trow[y];
                cmla(acc0, make_double2(t0.x, t0.y), wrow[y]);
            }
        }
        __syncthreads();
    }
    sm[tid] = make_double2(acc0.x + acc1.x, acc0.y + acc1.y);
    __syncthreads();
    if (tid < len) {
        double2 s = sm[tid];
        for (int w = 1; w < 4; ++w) s = make_double2(s.x + sm[w * 64 + tid].x, s.y + sm[w * 64 + tid].y);
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
#pragma unroll
                for (int u = 0; u < RG; ++u) cmla(acc[u], ring[(v + u) % RG], wv);
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
    const int slab_max = std::max((2 * Q - 1) * 16 + ((kAdjFL + 2 * P - 2) | 1) * 8,
                                  (2 * P - 1) * 16 + ((kAdjFL + 2 * Q - 2) | 1) * 8);
    const size_t frame_min = std::max<size_t>(256 * 16, slab_max);
    size_t lds = n_interior_blocks > 0 ? lds_interior : 0;
    if (n_frame_jobs > 0) lds = n_interior_blocks > 0 ? std::max(lds, frame_min) : (size_t)kAdjFrameLds;
    aa.frame_lds = (int)lds;
    static bool attr = false;
    if (!attr) {
        hipError_t e = hipFuncSetAttribute(reinterpret_cast<const void *>(&adj_main),
                                           hipFuncAttributeMaxDynamicSharedMemorySize, 160 * 1024);
        if (e != hipSuccess) return e;
        e = hipFuncSetAttribute(reinterpret_cast<const void *>(&adj_tables),
                                hipFuncAttributeMaxDynamicSharedMemorySize, 160 * 1024);
        if (e != hipSuccess) return e;
        attr = true;
    }
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

}  // namespace covest
