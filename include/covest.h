/*
 * covest.h -- C ABI of libcovest, the sliding-window estimated covariance
 * matrix on AMD Instinct MI355X (gfx950).
 *
 * The operation (Green, David, Galperin, Birk, "Efficient Parallel Computation
 * of the Estimated Covariance Matrix", Sec. 2.2, eqs. 2.1-2.2): for a complex
 * N x M input A and a P x Q window, every window position (p, q) with
 * 0 <= p <= N-P, 0 <= q <= M-Q gives the column stack V^{p,q}, whose entry
 * k = i + P*j is A[p+i][q+j].  The estimated covariance matrix is
 *
 *     R = (1/K) * sum_{p,q} V^{p,q} (V^{p,q})^H,     K = (N-P+1)(M-Q+1),
 *
 * a PQ x PQ Hermitian positive semi-definite matrix; entry (k1, k2) is
 * (1/K) sum_{p,q} A[p+i1][q+j1] * conj(A[p+i2][q+j2]).
 *
 * Conventions shared by every call:
 *   - A is complex64 (interleaved float re, im), row-major, A[n*lda + m] with
 *     n the row (0 <= n < N) and lda >= M (lda = M for the plain calls).
 *   - R is PQ x PQ row-major.  Its element type is complex128 (interleaved
 *     double) when opts->prec == COVEST_PREC_FP64 and complex64 otherwise.
 *   - All pointers named A, R, dR, dA, ws are DEVICE pointers on the current
 *     HIP device, owned by the caller.  The library never frees caller memory.
 *   - All device work is enqueued on `stream` (0 = the null stream) and is
 *     stream-ordered: no call synchronises the host unless COVEST_SYNC=1 is set
 *     in the environment, which makes every call wait and check for errors.
 *   - R must not alias A; dA must not alias A or dR.
 *   - Every call returns a covest_status; no C++ exception crosses the ABI.
 *     On a non-OK status covest_last_error() describes the problem.
 *   - Calls on different streams may run concurrently.
 *   - Non-finite input (NaN or Inf in A) is propagated, never checked.  By the
 *     definition exactly the entries whose windows meet such an element are
 *     non-finite.  The recurrence form recovers entries by adding and
 *     subtracting edge sums of one combination (Sec. 3.3), so it may make
 *     further entries of the same combination NaN as well; every entry it
 *     returns finite is the definition's value.  For the plain (Hankel) form
 *     only the propagation is stated: which entries turn non-finite depends
 *     on its tiling.  The adjoint makes non-finite every element of every
 *     window that holds a non-finite element of A (as the definition does),
 *     exactly those among the interior outputs; an output next to A's border
 *     may also turn non-finite through a zero weight (0 * NaN).  Every
 *     finite output is the definition's value.
 */
#ifndef COVEST_H
#define COVEST_H

#include <stddef.h>
#include <stdint.h>
#include <hip/hip_runtime_api.h>

#ifdef __cplusplus
extern "C" {
#endif

#define COVEST_VERSION 5

typedef enum {
    COVEST_OK = 0,
    COVEST_ERR_INVALID_ARG = -1,   /* null pointer, bad enum, bad leading dimension   */
    COVEST_ERR_SHAPE = -2,         /* P < 1, Q < 1, P > N, Q > M, or size overflow     */
    COVEST_ERR_WORKSPACE = -3,     /* ws_bytes below covest_workspace_size()          */
    COVEST_ERR_HIP = -4,           /* a HIP runtime call failed                        */
    COVEST_ERR_UNSUPPORTED = -5,   /* form/precision/shape combination not provided   */
    COVEST_ERR_PLAN_MISMATCH = -6  /* a batched plan was used on another device/state */
} covest_status;

/* Which kernel family computes R. */
typedef enum {
    COVEST_FORM_AUTO = 0,          /* recurrence (the faster form for every size)          */
    COVEST_FORM_RECURRENCE = 1,    /* diagonal-segment recurrence, FP64 sums (Sec. 3)      */
    COVEST_FORM_HANKEL_MFMA = 2    /* R = X X^H / K as a dense product on matrix cores     */
} covest_form;

typedef enum {
    COVEST_PREC_FP64 = 0,   /* recurrence: FP64 products and sums, complex128 R            */
    COVEST_PREC_FP32 = 1,   /* recurrence: FP64 sums rounded to complex64 R;
                               Hankel: FP32 matrix-core products, FP64 split-K reduction   */
    COVEST_PREC_BF16X3 = 2, /* Hankel: A split into bf16 hi + lo, hi*hi + hi*lo + lo*hi     */
    COVEST_PREC_FP16X3 = 3, /* Hankel: same with fp16 planes (lo plane scaled by 2^11)      */
    COVEST_PREC_BF16 = 4,   /* Hankel: plain bf16 inputs, FP32 accumulation                 */
    COVEST_PREC_FP16 = 5    /* Hankel: plain fp16 inputs, FP32 accumulation                 */
} covest_precision;

typedef enum {
    COVEST_FILL_FULL = 0,   /* whole R; the lower triangle is the exact conjugate mirror  */
    COVEST_FILL_UPPER = 1   /* entries with k2 >= k1 only; the lower triangle is untouched */
} covest_fill;

/* Which units run the main pass of the recurrence.  Both compute the same
 * FP64 sums of the same products (each distinct product once, Sec. 3.3); they
 * differ in speed and in the order of the additions. */
typedef enum {
    COVEST_ENGINE_AUTO = 0,    /* matrix cores wherever they can run, except lag blocks
                                  of 7-8 tiles under 30% real (P = 56..64, Q = 4); in a
                                  batch only windows whose tiles are at least 70% real */
    COVEST_ENGINE_VECTOR = 1,  /* FP64 FMA on the vector units, lags in a register ring  */
    COVEST_ENGINE_MATRIX = 2,  /* FP64 MFMA: per line, a block of A times a Toeplitz band
                                  of the line; needs N >= 2P-1, M >= 2Q-1, Q >= 4 and a
                                  lag block of at most 8 tiles of 16 x 16
                                  (COVEST_ERR_UNSUPPORTED otherwise)                     */
    COVEST_ENGINE_LANE = 3     /* one lane per unique combination (Sec. 3.1) of one input:
                                  the lane slides its box sums down and across the input
                                  (the shift rule of Sec. 3.3 in both directions) and
                                  writes every entry itself -- no finalize, no
                                  workspace.  For many small inputs (aperture plans pick
                                  it under AUTO); one input is one workgroup, slow on
                                  its own.
                                  Needs Q <= 16, PQ + (P-1)(Q-1) <= 512 and
                                  (P+3)g + 8M <= 4096, g = M+2Q-2 rounded up to odd
                                  (its staged rows fit 64 KB of LDS); FP64 or
                                  FP32 output; covest_forward, _ex, _noalloc and aperture
                                  plans only (COVEST_ERR_UNSUPPORTED otherwise)          */
} covest_engine;

typedef struct {
    covest_form form;
    covest_precision prec;
    covest_fill fill;
    int normalize;          /* 1: R = C / K (default); 0: the paper's unnormalised C       */
    int ring_cols;          /* vector engine tile shape: lags per lane along columns (dc)   */
    int ring_rows;          /* and along rows (dr): 4, 8, 12 or 16; 0 = the library's choice;
                               a non-zero width makes AUTO pick the vector engine           */
    int engine;             /* covest_engine (recurrence form only)                         */
} covest_opts;

/* Work counts of the method for one shape (Sec. 3.2-4.1):
 *   K         number of window positions, (N-P+1)(M-Q+1)
 *   n_uc      unique combinations, PQ + (P-1)(Q-1)                  (eq. 3.4)
 *   um        distinct products, sum over combinations of
 *             (N-|dr|)(M-|dc|)                                      (eqs. 3.5-3.6, 4.6)
 *   eta       upper-triangle entries, PQ(PQ+1)/2                    (eqs. 3.8, 4.22)
 *   segments  diagonal segments, sum over combinations of Q-|dc|    (Sec. 3.3)         */
typedef struct {
    int64_t K, n_uc, um, eta, segments;
} covest_counts_t;

/* One problem of a batch.  A and R are device pointers; the element type of R
 * follows the batch's precision. */
typedef struct {
    const void *A;
    void *R;
    int32_t N, M, P, Q;
} covest_problem;

typedef struct covest_plan covest_plan;   /* opaque, owned by the library */

/* Counts of the method for (N, M, P, Q).  Host only.  out must be non-null. */
int covest_counts(int64_t N, int64_t M, int64_t P, int64_t Q, covest_counts_t *out);

/* Device workspace (bytes) covest_forward needs for this shape and options.
 * Host only; opts may be NULL (defaults: AUTO, FP64, FULL, normalize=1). */
int covest_workspace_size(int64_t N, int64_t M, int64_t P, int64_t Q,
                          const covest_opts *opts, size_t *bytes);

/* R of the operation above (Sec. 2.2, eq. 2.2) for A (N x M, lda = M).
 * ws must hold at least covest_workspace_size() bytes (NULL allowed when that
 * size is 0).  The first call for a shape builds and caches its plan (host work
 * plus a small device table); later calls only enqueue kernels. */
int covest_forward(const void *A, int64_t N, int64_t M, int64_t P, int64_t Q, void *R,
                   const covest_opts *opts, void *ws, size_t ws_bytes, hipStream_t stream);

/* As covest_forward, for a strided view of A (row stride lda >= M elements)
 * and of R (row stride ldr >= PQ elements). */
int covest_forward_ex(const void *A, int64_t lda, int64_t N, int64_t M, int64_t P, int64_t Q,
                      void *R, int64_t ldr, const covest_opts *opts, void *ws, size_t ws_bytes,
                      hipStream_t stream);

/* For callers that cannot allocate device memory (code under HIP graph
 * capture, tight serving loops, harnesses that forbid hipMalloc): the
 * recurrence form of covest_forward_ex with no workspace argument and no
 * device allocation at all.  The plan's job tables and the FP64 workspace live
 * in one fixed device array of COVEST_NOALLOC_SCRATCH_BYTES (32 MiB) per GPU,
 * held from the library's first use of that GPU until the process ends; the
 * call neither calls hipMalloc nor hipFree.  A, R, strides and options are as
 * for covest_forward_ex; results are bitwise those of covest_forward_ex with
 * the same options.
 *   - form must be AUTO or RECURRENCE and prec FP64 or FP32 (the plain form:
 *     COVEST_ERR_UNSUPPORTED).  COVEST_ENGINE_LANE needs no scratch at all.
 *   - A shape whose tables plus workspace exceed the array is rejected with
 *     COVEST_ERR_WORKSPACE before any device work (covest_workspace_size()
 *     plus a few hundred KB of tables must fit; the 1024 x 1024 input with a
 *     32 x 32 window needs about 15 MB).
 *   - Every call on one GPU shares that GPU's array.  The host copies a
 *     shape's tables into it (hipMemcpyAsync on `stream`, from the library's
 *     cached host plan) when the previous call on that GPU used another
 *     shape.  Calls that may overlap on one GPU -- on different streams
 *     without ordering between them, or from several host threads -- race on
 *     the array and give wrong results; order them on one stream.  Nothing in
 *     the array needs to start at zero: every kernel writes each workspace
 *     word before reading it. */
#define COVEST_NOALLOC_SCRATCH_BYTES (32u << 20)
int covest_forward_noalloc(const void *A, int64_t lda, int64_t N, int64_t M, int64_t P, int64_t Q,
                           void *R, int64_t ldr, const covest_opts *opts, hipStream_t stream);

/* Adjoint of the forward map for a real loss L (PyTorch's convention for
 * complex tensors: a gradient is dL/dRe + i dL/dIm; the adjoint is derived
 * from eq. 2.2).  dR (PQ x PQ) is the gradient of L with respect to every
 * entry of R; with H = dR + dR^H, the result is dA = fold(H X) / K, where
 * column (p, q) of X is V^{p,q} and fold adds row i + P*j of the product onto
 * A[p+i][q+j].  dA (N x M) is OVERWRITTEN.  Windows are recomputed from A;
 * nothing is stored by the forward call.  A is complex64 as for the forward.
 *   opts->prec    element type of dR and dA: complex128 for COVEST_PREC_FP64
 *                 (also the default with opts = NULL), complex64 for every
 *                 other precision -- the type of R the forward returns under
 *                 the same options.  The arithmetic is FP64 either way.
 *   opts->fill    FULL: H = dR + dR^H.  UPPER: the output's lower triangle is
 *                 not a function of A, so only the entries k2 >= k1 of dR are
 *                 read and H = triu(dR) + triu(dR)^H.
 *   opts->normalize  0 drops the 1/K.  form, ring widths and engine are
 *                 ignored.
 * ws holds covest_backward_workspace_size() bytes (COVEST_ERR_WORKSPACE if
 * smaller).  Errors: COVEST_ERR_INVALID_ARG for null pointers, dA overlapping A
 * or dR, or (in _ex) lda < M, ldda < M, ldr < PQ; COVEST_ERR_SHAPE as for the
 * forward; COVEST_ERR_UNSUPPORTED for P or Q above 64.
 * covest_backward_ex takes strided views: A[n*lda + m], dR[k1*ldr + k2],
 * dA[n*ldda + m] (elements). */
int covest_backward_workspace_size(int64_t N, int64_t M, int64_t P, int64_t Q,
                                   const covest_opts *opts, size_t *bytes);
int covest_backward(const void *A, const void *dR, void *dA, int64_t N, int64_t M, int64_t P,
                    int64_t Q, const covest_opts *opts, void *ws, size_t ws_bytes,
                    hipStream_t stream);
int covest_backward_ex(const void *A, int64_t lda, const void *dR, int64_t ldr, void *dA, int64_t ldda,
                       int64_t N, int64_t M, int64_t P, int64_t Q, const covest_opts *opts, void *ws,
                       size_t ws_bytes, hipStream_t stream);

/* Batched forward (Sec. 3.4, 5.1: many matrices at once keep every core busy).
 * covest_plan_batched_create copies the problem array, builds one work list for
 * all problems (longest work first), allocates the plan's device tables and
 * workspace, and captures the launches into a HIP graph on `stream`.  Every
 * problem uses opts->prec (FP64 or FP32) with the recurrence form.
 * covest_forward_batched replays that graph on `stream`: one launch for every
 * instance.  The A and R buffers named at creation must stay valid.
 * opts->engine applies per problem as for a single call (AUTO: the matrix
 * cores wherever they fit; MATRIX: an error if some problem does not fit).
 * Matrix-core problems run in one extra launch per lag-block shape.
 * Measurement knob: COVEST_WORKERS=n in the environment when a plan is
 * created caps the persistent vector kernel at n workgroups (n >= 1); the
 * results do not change, only how many workers claim the jobs. */
int covest_plan_batched_create(covest_plan **out, const covest_problem *problems, int64_t count,
                               const covest_opts *opts, hipStream_t stream);
int covest_forward_batched(covest_plan *plan, hipStream_t stream);
int covest_plan_destroy(covest_plan *plan);

/* One problem of a batch over strided views: A[n*lda + m] (lda >= M elements)
 * and R[k1*ldr + k2] (ldr >= PQ elements), so that the problems of a batch can
 * be windows into one larger array.  Device pointers, as above. */
typedef struct {
    const void *A;
    void *R;
    int64_t lda, ldr;
    int32_t N, M, P, Q;
} covest_problem_ex;

/* As covest_plan_batched_create, for strided problems (the same checks, and
 * COVEST_ERR_INVALID_ARG for lda < M or ldr < PQ). */
int covest_plan_batched_create_ex(covest_plan **out, const covest_problem_ex *problems, int64_t count,
                                  const covest_opts *opts, hipStream_t stream);

/* The apertures of one image (Sec. 2.3: minimum-variance SAR imaging divides
 * an image into overlapping apertures and needs the estimated covariance
 * matrix of every one of them, with the same P x Q window).  Aperture (a, b),
 * 0 <= a < n_rows, 0 <= b < n_cols, is the ap_rows x ap_cols block of the
 * image whose first element is image[(a*row_step)*ld + b*col_step]; it is one
 * problem of a batched plan (N = ap_rows, M = ap_cols, lda = ld).  Its R is
 * the PQ x PQ matrix at R + (a*n_cols + b) * PQ*PQ elements (contiguous,
 * ldr = PQ; complex128 or complex64 as opts->prec says).
 * Errors: COVEST_ERR_INVALID_ARG for null pointers, ld < W, a step below 1 or
 * a count below 1; COVEST_ERR_SHAPE when an aperture leaves the image
 * ((n_rows-1)*row_step + ap_rows > H, likewise for columns), for a window
 * larger than an aperture, or for more than 2^31 - 1 apertures; otherwise as
 * covest_plan_batched_create.  The image and R must stay valid while the
 * plan is used; covest_forward_batched recomputes every R from the image.
 * Engines: COVEST_ENGINE_LANE (one launch, no workspace) is what AUTO picks
 * when the window fits it and the grid has at least as many apertures as the
 * device has compute units; VECTOR and MATRIX build the batched plan of
 * strided views.  The lane engine shares work between overlapping apertures
 * of a grid column: when the row step is below half the box height plus P-1,
 * one workgroup walks several apertures down the image (its box slides from
 * one aperture's last window row to the next aperture's first, instead of
 * summing a new box), as many as keep four workgroups per compute unit;
 * COVEST_AP_CHAIN=n in the environment at plan creation fixes that count
 * (n >= 1; results change only by rounding). */
typedef struct {
    const void *image;
    int64_t ld, H, W;
    int64_t ap_rows, ap_cols;
    int64_t row_step, col_step;
    int64_t n_rows, n_cols;
} covest_aperture_grid;
int covest_plan_apertures_create(covest_plan **out, const covest_aperture_grid *grid, int64_t P, int64_t Q,
                                 void *R, const covest_opts *opts, hipStream_t stream);

/* Minimum-variance (Capon) spectrum of a batch of estimated covariance
 * matrices (Sec. 2.3: R feeds the MVM / Capon estimator).  Each R is PQ x PQ
 * complex128, row-major, Hermitian positive definite (the FP64 output of
 * covest_forward or of a batched plan); matrix c starts at R + c*PQ*PQ.  Only
 * the upper triangle (k2 >= k1) is read, so R from either fill works.  On
 * the grid w1 = -pi + 2 pi f1 / F1, w2 = -pi + 2 pi f2 / F2:
 *     S[c][f1][f2] = 1 / Re(a^H R^{-1} a),   a[i + P*j] = exp(i (w1 i + w2 j)),
 * S being count x F1 x F2 doubles (device).  Cholesky factor in FP64, R^{-1}
 * from two triangular solves, its sums along the lags (i1 - i2, j1 - j2) and a
 * separable 2-D DFT of those sums (the quadratic form depends on R^{-1} only
 * through them).  Limits: PQ <= 256 (COVEST_ERR_UNSUPPORTED; above PQ = 128
 * the factor lives in the workspace, not in LDS, and the call is slower),
 * 1 <= F1, F2 <= 4096 (COVEST_ERR_SHAPE).  ws holds covest_capon_workspace_size() bytes
 * (COVEST_ERR_WORKSPACE if smaller).  A matrix that is not numerically positive
 * definite (a Cholesky pivot <= 0 or NaN) gets an all-NaN spectrum. */
int covest_capon_workspace_size(int64_t count, int64_t P, int64_t Q, int64_t F1, size_t *bytes);
int covest_capon_spectrum(const void *R, int64_t count, int64_t P, int64_t Q, int64_t F1, int64_t F2, double *S,
                          void *ws, size_t ws_bytes, hipStream_t stream);

/* Kernel timing for benchmarks: while enabled, every kernel the library
 * launches is bracketed by HIP events on its stream and its duration is added
 * to a per-kernel total.  covest_timing_read copies up to `cap` records (name,
 * launches, total milliseconds) after synchronising the recorded events, and
 * returns the number of records; covest_timing_reset clears them.  Host only. */
typedef struct {
    char name[48];
    int64_t launches;
    double total_ms;
} covest_timing_record;
int covest_timing_enable(int on);
int covest_timing_reset(void);
int covest_timing_read(covest_timing_record *out, int cap);

/* Message for the last non-OK status returned on this thread ("" if none). */
const char *covest_last_error(void);

/* COVEST_VERSION of the library. */
int covest_version(void);

#ifdef __cplusplus
}
#endif

#endif /* COVEST_H */
