// capon_kernels.hip -- minimum-variance (Capon) spectrum of estimated
// covariance matrices, the estimator the paper names as the consumer of R
// (Sec. 2.3: MVM imaging, Capon's method).
//
// For a PQ x PQ Hermitian positive definite R and the steering vector
// a[i + P*j] = exp(i (w1 i + w2 j)) (the window's index map, eq. 2.1):
//     a^H R^{-1} a = sum_{k1,k2} R^{-1}[k1][k2] exp(-i (w1 (i1-i2) + w2 (j1-j2))),
// so the quadratic form depends on R^{-1} only through its sums along the
// lags (di, dj) = (i1 - i2, j1 - j2) -- the same combinations as in R itself
// (Sec. 3.1) -- and the spectrum over a grid of (w1, w2) is a separable 2-D
// DFT of (2P-1) x (2Q-1) lag sums.
//
// One workgroup per matrix (n = PQ <= 256); for n <= 128 everything but the
// DFT lives in LDS, above that the packed factor lives in the workspace:
//   1. the lower triangle of R into LDS (packed, row i at i(i+1)/2), read as
//      the conjugate of the upper triangle (the part every fill writes);
//   2. Cholesky R = L L^H in place (right-looking, FP64, one barrier per
//      column: the column's scaling is deferred to one pass at the end);
//   3. W = L^{-1} in place, columns from n-1 down to 0, two per step: with
//      the trailing block already inverted, W[i][j] = -(1/L[j][j]) sum_{m=j+1..i}
//      W[i][m] L[m][j] (the columns of L are copied aside first);
//   4. the lag sums of R^{-1} = W^H W, whose entry (k1, k2) is
//      sum_{r >= max(k1,k2)} conj(W[r][k1]) W[r][k2] (half of the lags: the
//      others are their conjugates);
//   5. T[f1][dj] = sum_di lag[di][dj] e^{-i w1 di} (workspace), then
//      S[f1][f2] = 1 / Re(sum_dj T[f1][dj] e^{-i w2 dj}), the twiddles of each
//      sum by a recurrence from its first (two sincos per output).
// A matrix that is not numerically positive definite (a pivot <= 0 or NaN)
// gets an all-NaN spectrum.
#include "capon_internal.hpp"

#include <cmath>

namespace covest {

namespace {

constexpr int kCT = 512;   // threads per workgroup (the LDS allows one workgroup per CU)

__device__ __forceinline__ int tri(int i) { return i * (i + 1) / 2; }

// Sum of v over the 4 lanes of a quad, in a fixed order (every lane gets it).
__device__ __forceinline__ double quad_sum(double v)
{
    v += __shfl_xor(v, 1);
    return v + __shfl_xor(v, 2);
}

// GF: the packed factor lives in the workspace (global memory, L2-resident)
// instead of LDS, for PQ above what one CU's LDS holds; the code is the same.
template <bool GF>
__global__ void __launch_bounds__(kCT) capon_kernel(CaponArgs ca)
{
    extern __shared__ double2 sh[];
    __shared__ int s_bad;
    const int n = ca.n, P = ca.P, Q = ca.Q, F1 = ca.F1, F2 = ca.F2;
    const int tid = threadIdx.x;
    const size_t mat = blockIdx.x;
    const double2 *R = ca.R + mat * n * n;
    double2 *T = ca.T + mat * (size_t)F1 * (2 * Q - 1);
    double *S = ca.S + mat * (size_t)F1 * F2;
    double2 *Lp = GF ? ca.F + mat * (size_t)tri(n) : sh;
    double2 *const colbuf = GF ? sh : sh + tri(n);   // n entries, then the lag sums

    // 1. lower triangle of R, taken from the upper one (R[i][k] = conj(R[k][i])):
    // both output fills of the forward write the upper triangle, so R from a
    // FILL_UPPER call works too.  Reads follow R's memory order.
    for (int e = tid; e < n * n; e += kCT) {
        const int k = e / n, i = e - k * n;
        if (k <= i) {
            const double2 v = R[e];
            Lp[tri(i) + k] = make_double2(v.x, -v.y);
        }
    }
    if (tid == 0) s_bad = 0;
    __syncthreads();

    // 2. Cholesky, column j at a time, the column's scaling deferred: column j
    // keeps a[i][j] = L[i][j] * L[j][j] and the update divides by the pivot
    // d = L[j][j]^2, so a step needs one barrier; the pivots' square roots go
    // to piv and the factor is rescaled once at the end.
    double *piv = reinterpret_cast<double *>(colbuf);   // n doubles, in the column buffer
    for (int j = 0; j < n; ++j) {
        const double d = Lp[tri(j) + j].x;   // final since the previous step's barrier
        if (tid == 0) {
            piv[j] = sqrt(d);
            if (!(d > 0.0)) s_bad = 1;
        }
        const double invd = 1.0 / d;
        // trailing update: A[i][k] -= a[i][j] conj(a[k][j]) / d for j < k <= i
        const int m = n - j - 1;
        for (int ii = tid >> 4; ii < m; ii += kCT >> 4) {
            const int i = j + 1 + ii;
            const double2 a = Lp[tri(i) + j];
            for (int kk = tid & 15; kk <= ii; kk += 16) {
                const int k = j + 1 + kk;
                const double2 b = Lp[tri(k) + j];
                double2 t = Lp[tri(i) + k];
                t.x -= (a.x * b.x + a.y * b.y) * invd;
                t.y -= (a.y * b.x - a.x * b.y) * invd;
                Lp[tri(i) + k] = t;
            }
        }
        __syncthreads();
    }
    const bool bad = s_bad != 0;
    // rescale: L[i][j] = a[i][j] / piv[j], L[j][j] = piv[j]
    for (int i = tid >> 4; i < n; i += kCT >> 4)
        for (int j = tid & 15; j <= i; j += 16) {
            const double sj = piv[j];
            double2 v = Lp[tri(i) + j];
            v = j == i ? make_double2(sj, 0.0) : make_double2(v.x / sj, v.y / sj);
            Lp[tri(i) + j] = v;
        }
    __syncthreads();

    // 3. W = L^{-1} in place, two columns (j, j-1) per step: for i > j
    //      W[i][j]   = -(1/L[j][j])     sum_{m=j+1..i} W[i][m] L[m][j]
    //      W[i][j-1] = -(1/L[j-1][j-1]) (W[i][j] L[j][j-1] + sum_{m=j+1..i} W[i][m] L[m][j-1])
    // from one pass over row i of the inverted trailing block; W[j][j-1] =
    // -(1/L[j-1][j-1]) W[j][j] L[j][j-1]; an odd n leaves column 0 alone.
    const int nq = 2 * Q - 1, nl = (2 * P - 1) * nq;
    double2 *col = colbuf;           // column j of L
    double2 *col2 = colbuf + n;      // column j-1 of L
    double2 *lag = colbuf + 2 * n;   // the lag sums
    if (!bad) {
        const int q = tid & 3;
        int j = n - 1;
        for (; j >= 1; j -= 2) {
            const int j1 = j - 1;
            for (int i = j + 1 + tid; i < n; i += kCT) col[i] = Lp[tri(i) + j];
            for (int i = j + tid; i < n; i += kCT) col2[i] = Lp[tri(i) + j1];
            __syncthreads();   // also orders the previous step's diagonal writes
            const double wjj = 1.0 / Lp[tri(j) + j].x, w11 = 1.0 / Lp[tri(j1) + j1].x;
            const double2 ljj1 = col2[j];   // L[j][j-1]
            for (int i = j + 1 + (tid >> 2); i < n; i += kCT / 4) {
                const double2 *wrow = Lp + tri(i);
                double ax = 0.0, ay = 0.0, bx = 0.0, by = 0.0;
#pragma unroll 4
                for (int m = j + 1 + q; m <= i; m += 4) {
                    const double2 w = wrow[m], l = col[m], l2 = col2[m];
                    ax += w.x * l.x - w.y * l.y;
                    ay += w.x * l.y + w.y * l.x;
                    bx += w.x * l2.x - w.y * l2.y;
                    by += w.x * l2.y + w.y * l2.x;
                }
                ax = quad_sum(ax);
                ay = quad_sum(ay);
                bx = quad_sum(bx);
                by = quad_sum(by);
                if (q == 0) {
                    const double wx = -wjj * ax, wy = -wjj * ay;   // W[i][j]
                    const double cx = wx * ljj1.x - wy * ljj1.y + bx;
                    const double cy = wx * ljj1.y + wy * ljj1.x + by;
                    Lp[tri(i) + j] = make_double2(wx, wy);
                    Lp[tri(i) + j1] = make_double2(-w11 * cx, -w11 * cy);
                }
            }
            __syncthreads();
            if (tid == 0) {
                Lp[tri(j) + j] = make_double2(wjj, 0.0);
                Lp[tri(j) + j1] = make_double2(-w11 * wjj * ljj1.x, -w11 * wjj * ljj1.y);
                Lp[tri(j1) + j1] = make_double2(w11, 0.0);
            }
        }
        if (j == 0) {   // n odd: column 0
            for (int i = 1 + tid; i < n; i += kCT) col[i] = Lp[tri(i)];
            __syncthreads();
            const double w00 = 1.0 / Lp[0].x;
            for (int i = 1 + (tid >> 2); i < n; i += kCT / 4) {
                const double2 *wrow = Lp + tri(i);
                double sx = 0.0, sy = 0.0;
#pragma unroll 4
                for (int m = 1 + q; m <= i; m += 4) {
                    const double2 w = wrow[m], l = col[m];
                    sx += w.x * l.x - w.y * l.y;
                    sy += w.x * l.y + w.y * l.x;
                }
                sx = quad_sum(sx);
                sy = quad_sum(sy);
                if (q == 0) Lp[tri(i)] = make_double2(-w00 * sx, -w00 * sy);
            }
            __syncthreads();
            if (tid == 0) Lp[0] = make_double2(w00, 0.0);
        }
    }
    __syncthreads();

    // 4. lag sums of R^{-1} = W^H W: lag l = (di + P-1) * (2Q-1) + (dj + Q-1)
    if (!bad) {
        // R^{-1} is Hermitian, so the sum along -(di, dj) is the conjugate of
        // the sum along (di, dj): only lags from the centre lc = (P-1)(2Q-1) +
        // (Q-1) up are summed, each also written conjugated to 2 lc - l.
        // A quad per lag: lane q of the quad takes rows r = r0+q, r0+4+q, ...
        const int q = tid & 3, lc = (P - 1) * nq + (Q - 1);
        for (int l = lc + (tid >> 2); l < nl; l += kCT / 4) {
            const int di = l / nq - (P - 1), dj = l - (l / nq) * nq - (Q - 1);
            double sx = 0.0, sy = 0.0;
            for (int j2 = max(0, -dj); j2 < Q - max(0, dj); ++j2)
                for (int i2 = max(0, -di); i2 < P - max(0, di); ++i2) {
                    const int k2 = i2 + P * j2, k1 = (i2 + di) + P * (j2 + dj);
                    int r = max(k1, k2) + q, base = tri(r);
#pragma unroll 4
                    for (; r < n; r += 4) {   // tri(r + 4) = tri(r) + 4r + 10
                        const double2 a = Lp[base + k1], b = Lp[base + k2];   // conj(a) * b
                        sx += a.x * b.x + a.y * b.y;
                        sy += a.x * b.y - a.y * b.x;
                        base += 4 * r + 10;
                    }
                }
            sx = quad_sum(sx);
            sy = quad_sum(sy);
            if (q == 0) {
                lag[l] = make_double2(sx, sy);
                if (l != lc) lag[2 * lc - l] = make_double2(sx, -sy);
            }
        }
    }
    __syncthreads();

    // 5. separable DFT over the grid w = -pi + 2 pi f / F
    const double two_pi = 6.283185307179586476925286766559;
    const double pi = 3.14159265358979323846264338328;
    if (!bad) {
        for (int e = tid; e < F1 * nq; e += kCT) {
            const int f1 = e / nq, q = e - f1 * nq;
            const double w1 = -pi + two_pi * f1 / F1;
            // twiddles e^{-i w1 (p - (P-1))} by a recurrence from p = 0
            double tr, ti, sr, si;
            sincos(w1 * (P - 1), &ti, &tr);
            sincos(-w1, &si, &sr);
            double sx = 0.0, sy = 0.0;
            for (int p = 0; p < 2 * P - 1; ++p) {
                const double2 v = lag[p * nq + q];
                sx += v.x * tr - v.y * ti;
                sy += v.x * ti + v.y * tr;
                const double nr = tr * sr - ti * si;
                ti = tr * si + ti * sr;
                tr = nr;
            }
            T[e] = make_double2(sx, sy);
        }
    }
    __syncthreads();
    for (int e = tid; e < F1 * F2; e += kCT) {
        if (bad) {
            S[e] = __builtin_nan("");
            continue;
        }
        const int f1 = e / F2, f2 = e - f1 * F2;
        const double w2 = -pi + two_pi * f2 / F2;
        double tr, ti, sr, si;   // e^{-i w2 (q - (Q-1))} by a recurrence from q = 0
        sincos(w2 * (Q - 1), &ti, &tr);
        sincos(-w2, &si, &sr);
        double re = 0.0;
        for (int q = 0; q < nq; ++q) {
            const double2 t = T[f1 * nq + q];
            re += t.x * tr - t.y * ti;
            const double nr = tr * sr - ti * si;
            ti = tr * si + ti * sr;
            tr = nr;
        }
        S[e] = 1.0 / re;
    }
}

}  // namespace

hipError_t launch_capon(const CaponArgs &ca, int count, hipStream_t stream)
{
    static const hipError_t attr = hipFuncSetAttribute(reinterpret_cast<const void *>(&capon_kernel<false>),
                                                       hipFuncAttributeMaxDynamicSharedMemorySize, 150 * 1024);
    if (attr != hipSuccess) return attr;
    if (count <= 0) return hipSuccess;
    if (capon_factor_in_lds(ca.n))
        hipLaunchKernelGGL(capon_kernel<false>, dim3(count), dim3(kCT), capon_lds_bytes(ca.n, ca.P, ca.Q), stream,
                           ca);
    else
        hipLaunchKernelGGL(capon_kernel<true>, dim3(count), dim3(kCT), capon_lds_bytes(ca.n, ca.P, ca.Q), stream,
                           ca);
    return hipGetLastError();
}

}  // namespace covest
