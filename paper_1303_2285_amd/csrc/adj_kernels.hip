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
// adj_frame      the remaining outputs: h read from the prefix sums (4 reads).
#include <hip/hip_runtime.h>

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

// H[a][b] = G[a][b] + conj(G[b][a]) from the complex64 gradient
__device__ __forceinline__ double2 h_entry(const AdjArgs &aa, int a, int b)
{
    const float2 g1 = aa.G[(int64_t)a * aa.ldg + b];
    const float2 g2 = aa.G[(int64_t)b * aa.ldg + a];
    return make_double2((double)g1.x + (double)g2.x, (double)g1.y - (double)g2.y);
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
    aa.dA[(int64_t)r * aa.ldda + c] = make_float2((float)s.x, (float)s.y);
}

// D2, frame: one thread per output outside the interior.
__global__ void __launch_bounds__(256) adj_frame(AdjArgs aa)
{
    const int P = aa.P, Q = aa.Q, N = aa.N, M = aa.M, Kr = aa.Kr, Kc = aa.Kc;
    const int64_t t = (int64_t)blockIdx.x * 256 + threadIdx.x;
    if (t >= aa.n_frame) return;
    // frame outputs enumerated row by row: rows outside [ir0, ir1) are whole,
    // rows inside contribute their columns outside [ic0, ic1)
    int r, c;
    {
        const int ir0 = aa.ir0, ir1 = aa.ir1, ic0 = aa.ic0, ic1 = aa.ic1;
        const int64_t top = (int64_t)ir0 * M;
        const int per_mid = M - (ic1 - ic0);
        const int64_t mid = (int64_t)(ir1 - ir0) * per_mid;
        if (t < top) {
            r = (int)(t / M);
            c = (int)(t % M);
        } else if (t < top + mid) {
            const int64_t u = t - top;
            r = ir0 + (int)(u / per_mid);
            const int k = (int)(u % per_mid);
            c = k < ic0 ? k : ic1 + (k - ic0);
        } else {
            const int64_t u = t - top - mid;
            r = ir1 + (int)(u / M);
            c = (int)(u % M);
        }
    }
    const int w = Q + 1;
    double2 s = dz();
    for (int dr = -(P - 1); dr < P; ++dr) {
        const int ilo = max(max(0, -dr), r - Kr + 1), ihi = min(min(P - 1, P - 1 - dr), r);
        if (ilo > ihi || r + dr < 0 || r + dr >= N) continue;
        for (int dc = -(Q - 1); dc < Q; ++dc) {
            const int jlo = max(max(0, -dc), c - Kc + 1), jhi = min(min(Q - 1, Q - 1 - dc), c);
            if (jlo > jhi || c + dc < 0 || c + dc >= M) continue;
            const int lag = (dr + P - 1) * (2 * Q - 1) + (dc + Q - 1);
            const double2 *S = reinterpret_cast<const double2 *>(aa.tables) + (int64_t)lag * (P + 1) * w;
            const double2 h = box(S, w, ilo, ihi, jlo, jhi);
            const float2 av = aa.A[(int64_t)(r + dr) * aa.lda + (c + dc)];
            cmla(s, make_double2(av.x, av.y), h);
        }
    }
    store_da(aa, r, c, s);
}

// D2, interior: workgroup tile of kAdjTR rows x kAdjTC columns of outputs.
// Thread (row, 16-column chunk, dr group): ring over dc, 16 FP64 accumulators;
// the dr groups are summed through LDS in a fixed order.
__global__ void __launch_bounds__(256) adj_interior(AdjArgs aa)
{
    extern __shared__ double2 sm[];
    const int P = aa.P, Q = aa.Q;
    const int ndc = aa.ndc;                        // dc steps padded to a multiple of 16
    const int nlag_c = 2 * Q - 1;
    const int tiles_c = (aa.ic1 - aa.ic0 + kAdjTC - 1) / kAdjTC;
    const int r0 = aa.ir0 + (blockIdx.x / tiles_c) * kAdjTR;
    const int c0 = aa.ic0 + (blockIdx.x % tiles_c) * kAdjTC;
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
    const int ch = (threadIdx.x / kAdjTR) % (kAdjTC / 16);
    const int grp = threadIdx.x / (kAdjTR * (kAdjTC / 16));
    constexpr int ngrp = 256 / (kAdjTR * (kAdjTC / 16));
    const int ndr = 2 * P - 1;
    const int dr0 = (int)((int64_t)grp * ndr / ngrp), dr1 = (int)((int64_t)(grp + 1) * ndr / ngrp);

    double2 acc[16];
#pragma unroll
    for (int u = 0; u < 16; ++u) acc[u] = dz();
    for (int di = dr0; di < dr1; ++di) {           // di = dr + P - 1
        // output (lr, 16*ch + u) reads A[lr + di][16*ch + u + dj] (tile coordinates)
        const float2 *arow = At + (lr + di) * stride + 16 * ch;
        const double2 *wrow = Wt + di * ndc;
        double2 ring[16];
#pragma unroll
        for (int k = 0; k < 15; ++k) ring[k] = make_double2(arow[k].x, arow[k].y);
        for (int b = 0; b < ndc; b += 16) {
#pragma unroll
            for (int v = 0; v < 16; ++v) {
                // dj = b + v; outputs u need arow[u + dj]
                const float2 an = arow[b + v + 15];
                ring[(v + 15) % 16] = make_double2(an.x, an.y);
                const double2 wv = wrow[b + v];
#pragma unroll
                for (int u = 0; u < 16; ++u) cmla(acc[u], ring[(v + u) % 16], wv);
            }
        }
    }
    __syncthreads();
    // fixed-order sum over the dr groups
    double2 *red = sm;
#pragma unroll
    for (int u = 0; u < 16; ++u) red[threadIdx.x * 16 + u] = acc[u];
    __syncthreads();
    constexpr int per_grp = kAdjTR * (kAdjTC / 16);
    for (int e = threadIdx.x; e < kAdjTR * kAdjTC; e += 256) {
        const int row = e / kAdjTC, col = e - row * kAdjTC;
        const int r = r0 + row, c = c0 + col;
        if (r >= aa.ir1 || c >= aa.ic1) continue;
        const int tid0 = row + kAdjTR * (col / 16);
        double2 s = dz();
        for (int g = 0; g < ngrp; ++g) {
            const double2 v = red[(tid0 + g * per_grp) * 16 + (col % 16)];
            s.x += v.x;
            s.y += v.y;
        }
        store_da(aa, r, c, s);
    }
}

hipError_t launch_adjoint(const AdjArgs &aa, int n_lags, size_t lds_tables, int n_interior_blocks,
                          size_t lds_interior, int64_t n_frame, hipStream_t s)
{
    static bool attr = false;
    if (!attr) {
        hipError_t e = hipFuncSetAttribute(reinterpret_cast<const void *>(&adj_interior),
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
    if (n_interior_blocks > 0) {
        hipLaunchKernelGGL(adj_interior, dim3(n_interior_blocks), dim3(256), lds_interior, s, aa);
        e = hipGetLastError();
        if (e != hipSuccess) return e;
    }
    if (n_frame > 0) {
        hipLaunchKernelGGL(adj_frame, dim3((unsigned)((n_frame + 255) / 256)), dim3(256), 0, s, aa);
        e = hipGetLastError();
    }
    return e;
}

}  // namespace covest
