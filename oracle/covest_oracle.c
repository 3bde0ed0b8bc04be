/*
 * covest_oracle.c -- CPU reference ("oracle") for the sliding-window estimated
 * covariance matrix.  TEST INFRASTRUCTURE ONLY: the tests, the smoke check and
 * the benchmark's CPU-baseline leg may call it; the library never does.
 *
 * Plain, slow and obviously correct.  Everything is FP64, compiled without
 * FMA contraction (-ffp-contract=off) and without fast-math.  It shares no code
 * with the GPU library.
 *
 * Definitions (Green, David, Galperin, Birk, "Efficient Parallel Computation of
 * the Estimated Covariance Matrix", Sec. 2.2):
 *   - A is N x M complex, row-major, A[n*M+m] = (re, im) interleaved, n the row.
 *   - S^{p,q} is the P x Q window whose upper-left corner is at (p, q); the
 *     column stack V^{p,q} takes window element (i, j) to index k = i + P*j
 *     (eq. 2.1, 0-based here).
 *   - C = sum over window positions of V V^H (eq. 2.2): entry (k1, k2) is the
 *     sum of A[p+i1][q+j1] * conj(A[p+i2][q+j2]).
 *   Readings taken where the text is ambiguous:
 *   - every window that fits is a position: p in [0, N-P], q in [0, M-Q], so
 *     K = (N-P+1)(M-Q+1) positions (the printed bounds drop the last row and
 *     column of positions);
 *   - R = C / K when normalize != 0 (one IEEE division per part), C otherwise;
 *   - the lower triangle is the exact conjugate of the upper one (C is
 *     Hermitian, Sec. 2.2).
 */
#include <stddef.h>
#include <stdint.h>
#include <string.h>
#include <stdlib.h>

#ifdef _OPENMP
#include <omp.h>
#endif

#define RE(p, idx) (p)[2 * (size_t)(idx)]
#define IM(p, idx) (p)[2 * (size_t)(idx) + 1]

static int shape_ok(int64_t N, int64_t M, int64_t P, int64_t Q)
{
    return N >= 1 && M >= 1 && P >= 1 && Q >= 1 && P <= N && Q <= M;
}

/* One entry (k1, k2) of C (eq. 2.2), summed over positions p-major. */
static void entry_sum(const double *A, int64_t N, int64_t M, int64_t P, int64_t Q,
                      int64_t k1, int64_t k2, double *sre, double *sim)
{
    (void)N;
    const int64_t i1 = k1 % P, j1 = k1 / P;
    const int64_t i2 = k2 % P, j2 = k2 / P;
    const int64_t Kr = N - P + 1, Kc = M - Q + 1;
    double re = 0.0, im = 0.0;
    for (int64_t p = 0; p < Kr; ++p) {
        for (int64_t q = 0; q < Kc; ++q) {
            const int64_t a = (p + i1) * M + (q + j1);  /* V^{p,q}[k1] */
            const int64_t b = (p + i2) * M + (q + j2);  /* V^{p,q}[k2] */
            const double xr = RE(A, a), xi = IM(A, a);
            const double yr = RE(A, b), yi = IM(A, b);
            /* x * conj(y) */
            const double tr = xr * yr + xi * yi;
            const double ti = xi * yr - xr * yi;
            re += tr;
            im += ti;
        }
    }
    *sre = re;
    *sim = im;
}

/* Full R (PQ x PQ, row-major, complex interleaved).  nthreads <= 1 runs the
 * plain serial loop; larger values split the k1 loop over OpenMP threads with
 * the loop body unchanged.  Returns 0 on success, -2 on a bad shape. */
int covest_oracle_fwd(const double *A, int64_t N, int64_t M, int64_t P, int64_t Q,
                      int normalize, double *R, int nthreads)
{
    if (!shape_ok(N, M, P, Q)) return -2;
    const int64_t PQ = P * Q;
    const double K = (double)((N - P + 1) * (M - Q + 1));
#ifdef _OPENMP
    if (nthreads < 1) nthreads = 1;
#pragma omp parallel for schedule(dynamic, 1) num_threads(nthreads)
#endif
    for (int64_t k1 = 0; k1 < PQ; ++k1) {
        for (int64_t k2 = k1; k2 < PQ; ++k2) {
            double sre, sim;
            entry_sum(A, N, M, P, Q, k1, k2, &sre, &sim);
            if (normalize) {
                sre = sre / K;
                sim = sim / K;
            }
            RE(R, k1 * PQ + k2) = sre;
            IM(R, k1 * PQ + k2) = sim;
            RE(R, k2 * PQ + k1) = sre;   /* Hermitian mirror */
            IM(R, k2 * PQ + k1) = -sim;
        }
    }
    return 0;
}

/* Selected entries: out[2*t] = R[k1[t], k2[t]].  Any (k1, k2) pair is allowed;
 * lower-triangle requests are answered as the conjugate of the upper entry. */
int covest_oracle_entries(const double *A, int64_t N, int64_t M, int64_t P, int64_t Q,
                          int normalize, const int64_t *k1, const int64_t *k2,
                          int64_t count, double *out, int nthreads)
{
    if (!shape_ok(N, M, P, Q)) return -2;
    const int64_t PQ = P * Q;
    for (int64_t t = 0; t < count; ++t)
        if (k1[t] < 0 || k2[t] < 0 || k1[t] >= PQ || k2[t] >= PQ) return -1;
    const double K = (double)((N - P + 1) * (M - Q + 1));
#ifdef _OPENMP
    if (nthreads < 1) nthreads = 1;
#pragma omp parallel for schedule(dynamic, 1) num_threads(nthreads)
#endif
    for (int64_t t = 0; t < count; ++t) {
        int64_t a = k1[t], b = k2[t];
        int flip = 0;
        if (b < a) { int64_t s = a; a = b; b = s; flip = 1; }
        double sre, sim;
        entry_sum(A, N, M, P, Q, a, b, &sre, &sim);
        if (normalize) {
            sre = sre / K;
            sim = sim / K;
        }
        out[2 * t] = sre;
        out[2 * t + 1] = flip ? -sim : sim;
    }
    return 0;
}

/*
 * Adjoint (not in the paper; PyTorch's convention for a real loss L of complex
 * variables, grad = dL/dRe + i dL/dIm).  With G the gradient of L with respect
 * to every entry of R and H = G + G^H, the gradient with respect to the window
 * vector V^{p,q} is H V^{p,q} / K, and each window element scatters back to the
 * input element it was taken from.  Direct definition, one position at a time.
 * dA is overwritten.
 */
int covest_oracle_adj(const double *A, const double *G, int64_t N, int64_t M,
                      int64_t P, int64_t Q, int normalize, double *dA)
{
    if (!shape_ok(N, M, P, Q)) return -2;
    const int64_t PQ = P * Q;
    const int64_t Kr = N - P + 1, Kc = M - Q + 1;
    const double K = normalize ? (double)(Kr * Kc) : 1.0;
    double *H = (double *)malloc(sizeof(double) * 2 * (size_t)PQ * (size_t)PQ);
    double *v = (double *)malloc(sizeof(double) * 2 * (size_t)PQ);
    if (!H || !v) { free(H); free(v); return -4; }
    for (int64_t a = 0; a < PQ; ++a)
        for (int64_t b = 0; b < PQ; ++b) {
            /* H[a][b] = G[a][b] + conj(G[b][a]) */
            RE(H, a * PQ + b) = RE(G, a * PQ + b) + RE(G, b * PQ + a);
            IM(H, a * PQ + b) = IM(G, a * PQ + b) - IM(G, b * PQ + a);
        }
    memset(dA, 0, sizeof(double) * 2 * (size_t)N * (size_t)M);
    for (int64_t p = 0; p < Kr; ++p) {
        for (int64_t q = 0; q < Kc; ++q) {
            for (int64_t k = 0; k < PQ; ++k) {            /* V^{p,q} (eq. 2.1) */
                const int64_t i = k % P, j = k / P;
                RE(v, k) = RE(A, (p + i) * M + (q + j));
                IM(v, k) = IM(A, (p + i) * M + (q + j));
            }
            for (int64_t k1 = 0; k1 < PQ; ++k1) {
                double ur = 0.0, ui = 0.0;                  /* (H v)[k1] */
                for (int64_t k2 = 0; k2 < PQ; ++k2) {
                    const double hr = RE(H, k1 * PQ + k2), hi = IM(H, k1 * PQ + k2);
                    const double xr = RE(v, k2), xi = IM(v, k2);
                    ur += hr * xr - hi * xi;
                    ui += hr * xi + hi * xr;
                }
                const int64_t i = k1 % P, j = k1 / P;
                RE(dA, (p + i) * M + (q + j)) += ur / K;
                IM(dA, (p + i) * M + (q + j)) += ui / K;
            }
        }
    }
    free(H);
    free(v);
    return 0;
}

int covest_oracle_max_threads(void)
{
#ifdef _OPENMP
    return omp_get_max_threads();
#else
    return 1;
#endif
}
