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
// One workgroup per matrix (n = PQ <= 128):
//   1. the lower triangle of R into LDS (packed, row i at i(i+1)/2);
//   2. Cholesky R = L L^H in place (right-looking, FP64);
//   3. R^{-1} = L^{-H} L^{-1}: thread c solves L x = e_c, then L^H y = x, for
//      column c, in the workspace; every thread walks the same rows, so the
//      workspace reads coalesce and the LDS reads of L are broadcasts;
//   4. the lag sums of R^{-1} into LDS (over the factor's space);
//   5. T[f1][dj] = sum_di lag[di][dj] e^{-i w1 di}, then
//      S[f1][f2] = 1 / Re(sum_dj T[f1][dj] e^{-i w2 dj}).
// A matrix that is not numerically positive definite (a pivot <= 0 or NaN)
// gets an all-NaN spectrum.
#include "capon_internal.hpp"

#include <cmath>

namespace covest {

namespace {

__device__ __forceinline__ int tri(int i) { return i * (i + 1) / 2; }

__global__ void __launch_bounds__(256) capon_kernel(CaponArgs ca)
{
    extern __shared__ double2 Lp[];
    __shared__ int s_bad;
    const int n = ca.n, P = ca.P, Q = ca.Q, F1 = ca.F1, F2 = ca.F2;
    const int tid = threadIdx.x;
    const size_t mat = blockIdx.x;
    const double2 *R = ca.R + mat * n * n;
    double2 *X = ca.X + mat * n * n;
    double2 *T = ca.T + mat * (size_t)F1 * (2 * Q - 1);
    double *S = ca.S + mat * (size_t)F1 * F2;

    // 1. lower triangle of R
    for (int e = tid; e < n * n; e += 256) {
        const int i = e / n, k = e - i * n;
        if (k <= i) Lp[tri(i) + k] = R[e];
    }
    if (tid == 0) s_bad = 0;
    __syncthreads();

    // 2. Cholesky, column j at a time
    for (int j = 0; j < n; ++j) {
        const double d = Lp[tri(j) + j].x;
        const double s = sqrt(d);
        __syncthreads();   // every thread has read the pivot
        if (tid == 0) {
            Lp[tri(j) + j] = make_double2(s, 0.0);
            if (!(d > 0.0)) s_bad = 1;
        }
        const double inv = 1.0 / s;
        for (int i = j + 1 + tid; i < n; i += 256) {
            double2 v = Lp[tri(i) + j];
            v.x *= inv;
            v.y *= inv;
            Lp[tri(i) + j] = v;
        }
        __syncthreads();
        // trailing update: L[i][k] -= L[i][j] conj(L[k][j]) for j < k <= i
        const int m = n - j - 1;
        for (int e = tid; e < m * m; e += 256) {
            const int ii = e / m, kk = e - ii * m;
            if (kk <= ii) {
                const int i = j + 1 + ii, k = j + 1 + kk;
                const double2 a = Lp[tri(i) + j], b = Lp[tri(k) + j];
                double2 t = Lp[tri(i) + k];
                t.x -= a.x * b.x + a.y * b.y;
                t.y -= a.y * b.x - a.x * b.y;
                Lp[tri(i) + k] = t;
            }
        }
        __syncthreads();
    }
    const bool bad = s_bad != 0;

    // 3. R^{-1}, column c per thread
    if (!bad) {
        for (int c = tid; c < n; c += 256) {
            for (int k = 0; k < n; ++k) {   // L x = e_c
                double sx = k == c ? 1.0 : 0.0, sy = 0.0;
                const double2 *row = Lp + tri(k);
                for (int m = 0; m < k; ++m) {
                    const double2 l = row[m], x = X[(size_t)m * n + c];
                    sx -= l.x * x.x - l.y * x.y;
                    sy -= l.x * x.y + l.y * x.x;
                }
                const double dinv = 1.0 / row[k].x;
                X[(size_t)k * n + c] = make_double2(sx * dinv, sy * dinv);
            }
            for (int k = n - 1; k >= 0; --k) {   // L^H y = x
                const double2 xk = X[(size_t)k * n + c];
                double sx = xk.x, sy = xk.y;
                for (int m = k + 1; m < n; ++m) {
                    const double2 l = Lp[tri(m) + k], y = X[(size_t)m * n + c];   // conj(l) * y
                    sx -= l.x * y.x + l.y * y.y;
                    sy -= l.x * y.y - l.y * y.x;
                }
                const double dinv = 1.0 / Lp[tri(k) + k].x;
                X[(size_t)k * n + c] = make_double2(sx * dinv, sy * dinv);
            }
        }
    }
    __syncthreads();   // the solves' writes are visible to the workgroup; L is no longer needed

    // 4. lag sums of R^{-1}: lag l = (di + P-1) * (2Q-1) + (dj + Q-1)
    const int nq = 2 * Q - 1, nl = (2 * P - 1) * nq;
    double2 *lag = Lp;
    if (!bad) {
        for (int l = tid; l < nl; l += 256) {
            const int di = l / nq - (P - 1), dj = l - (l / nq) * nq - (Q - 1);
            double sx = 0.0, sy = 0.0;
            for (int j2 = max(0, -dj); j2 < Q - max(0, dj); ++j2)
                for (int i2 = max(0, -di); i2 < P - max(0, di); ++i2) {
                    const int k2 = i2 + P * j2, k1 = (i2 + di) + P * (j2 + dj);
                    const double2 v = X[(size_t)k1 * n + k2];
                    sx += v.x;
                    sy += v.y;
                }
            lag[l] = make_double2(sx, sy);
        }
    }
    __syncthreads();

    // 5. separable DFT over the grid w = -pi + 2 pi f / F
    const double two_pi = 6.283185307179586476925286766559;
    const double pi = 3.14159265358979323846264338328;
    if (!bad) {
        for (int e = tid; e < F1 * nq; e += 256) {
            const int f1 = e / nq, q = e - f1 * nq;
            const double w1 = -pi + two_pi * f1 / F1;
            double sx = 0.0, sy = 0.0;
            for (int p = 0; p < 2 * P - 1; ++p) {
                double sn, cs;
                sincos(-w1 * (p - (P - 1)), &sn, &cs);
                const double2 v = lag[p * nq + q];
                sx += v.x * cs - v.y * sn;
                sy += v.x * sn + v.y * cs;
            }
            T[e] = make_double2(sx, sy);
        }
    }
    __syncthreads();
    for (int e = tid; e < F1 * F2; e += 256) {
        if (bad) {
            S[e] = __builtin_nan("");
            continue;
        }
        const int f1 = e / F2, f2 = e - f1 * F2;
        const double w2 = -pi + two_pi * f2 / F2;
        double re = 0.0;
        for (int q = 0; q < nq; ++q) {
            double sn, cs;
            sincos(-w2 * (q - (Q - 1)), &sn, &cs);
            const double2 t = T[f1 * nq + q];
            re += t.x * cs - t.y * sn;
        }
        S[e] = 1.0 / re;
    }
}

}  // namespace

hipError_t launch_capon(const CaponArgs &ca, int count, hipStream_t stream)
{
    static const hipError_t attr = hipFuncSetAttribute(reinterpret_cast<const void *>(&capon_kernel),
                                                       hipFuncAttributeMaxDynamicSharedMemorySize, 150 * 1024);
    if (attr != hipSuccess) return attr;
    if (count <= 0) return hipSuccess;
    hipLaunchKernelGGL(capon_kernel, dim3(count), dim3(256), capon_lds_bytes(ca.n, ca.P, ca.Q), stream, ca);
    return hipGetLastError();
}

}  // namespace covest
