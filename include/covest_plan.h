/*
 * covest_plan.h -- introspection of libcovest's plans for tests and tools
 * (host only, no device needed), and one measurement call
 * (covest_forward_stamped) that times every finalize item on the device.
 *
 * The recurrence (Sec. 3.3 of the paper: each product is computed once and
 * every output entry has a single writer) splits the products of every unique
 * combination (eq. 3.3) into a middle block shared by all window offsets,
 * strips of individual rows and columns, and corner products.  These calls
 * expose that split so a test can check that every product is owned by exactly
 * one job and every upper-triangle entry by exactly one finalize item
 * (Sec. 4.2-4.3).
 *
 * n_slots is the number of workgroups the plan assumes resident at once (two
 * per compute unit: 512 on MI355X).  w0 and w1 choose the ring widths (lags
 * per lane along columns and along rows: 4, 8, 12 or 16; 0 = the default the
 * library uses without tuning).  All arrays are caller-owned host memory.
 */
#ifndef COVEST_PLAN_H
#define COVEST_PLAN_H

#include <stddef.h>
#include <stdint.h>
#include <hip/hip_runtime_api.h>

#include "covest.h"

#ifdef __cplusplus
extern "C" {
#endif

typedef struct {
    int32_t W0, W1;             /* ring widths: along columns (dc), along rows (dr)   */
    int32_t Rm0, Rm1, Cm0, Cm1; /* middle rows [Rm0, Rm1) and columns [Cm0, Cm1)      */
    int32_t n_ir, n_ic;         /* individual rows / columns                           */
    int32_t lag_stride;         /* (2P-1)Q; lag (dr, dc) has index (dr+P-1)Q + dc       */
    int32_t bandw;              /* columns per bulk unit                                */
    int32_t n_bulk;             /* partial-sum rows                                     */
    int32_t n_jobs, n_groups, n_items;
    int64_t ws_bytes;           /* forward workspace                                    */
    int64_t lds_main, lds_fin;  /* dynamic LDS bytes of the two kernels                 */
    int64_t main_products;      /* distinct products kept by the main kernel            */
    int64_t fin_products;       /* corner products computed by the finalize kernel      */
} covest_plan_info;

/* Job rows: 12 int32 each (mode, inst, group, out, u0, u1, x0, x1, c0, c1,
 * tile_rows, tile_cols).  Group rows: 14 int32 each (orient, W, d1lo, d1hi,
 * ch0, nch, v2lo, v2hi, lanes, slots, hr_lo, hr_hi, hc_lo, hc_hi).  Item rows:
 * 5 int32 each (inst, dr, dc, bulk0, bulk1).  COVEST_ERR_SHAPE on a bad shape,
 * COVEST_ERR_UNSUPPORTED when P or Q exceeds the recurrence's limit,
 * COVEST_ERR_INVALID_ARG for a width other than 0, 4, 8, 12 or 16. */
int covest_plan_info_get(int64_t N, int64_t M, int64_t P, int64_t Q, int32_t n_slots, int32_t w0,
                         int32_t w1, covest_plan_info *out);
int covest_plan_tables(int64_t N, int64_t M, int64_t P, int64_t Q, int32_t n_slots, int32_t w0, int32_t w1,
                       int32_t *jobs, int32_t *groups, int32_t *items);

/* Plan of the matrix-core engine (COVEST_ENGINE_MATRIX) for n_cu compute
 * units.  The middle block is exact: rows [P-1, N-P+1), columns [Q-1, M-Q+1).
 * A first-factor line (a row of A for orientation 0, a column for 1) is
 * walked in k-groups of 4 second-factor positions; each workgroup job covers
 * a range of (block of 8 lines, k-group) pairs.  Bulk jobs (kind 0) add
 * their sums into partial row `out`; strip jobs (kind 1) cover one block and
 * one piece of its k-groups, and line l writes z row out + (l - line0), where
 * z rows are numbered piece * (individual lines) + individual index. */
typedef struct {
    int32_t mt, nt;             /* 16 x 16 tiles of the lag block: rows dr, columns dc  */
    int32_t Rm0, Rm1, Cm0, Cm1; /* middle rows / columns                               */
    int32_t n_ir, n_ic;         /* individual rows / columns                           */
    int32_t lag_stride;         /* (2P-1)Q                                             */
    int32_t n_bulk, n_jobs, n_items;
    int32_t zpieces;            /* pieces per strip line                               */
    int64_t ws_bytes, lds_main, lds_fin, main_products, fin_products;
} covest_mfma_plan_info;

/* Fills *out and, when non-null, the job rows (16 int32 each: inst, orient,
 * kind, out, line0, line_end, b0, kg0, b1, kg1, n_kg, pos_lo, pos_hi, k0, kin, 0;
 * kin: the k-groups [0, kin) whose four positions all lie inside the line,
 * whose first operand the kernel loads without a clamp)
 * and the finalize item rows (5 int32 each, as covest_plan_tables).
 * COVEST_ERR_UNSUPPORTED when the engine cannot run the shape. */
int covest_mfma_plan_get(int64_t N, int64_t M, int64_t P, int64_t Q, int32_t n_cu,
                         covest_mfma_plan_info *out, int32_t *jobs, int32_t *items);

/* Measurement run of the recurrence (covest_forward with lda = M, ldr = PQ):
 * the same result, and for every finalize item -- one unique combination
 * (dr, dc), the work unit the paper assigns to a core (Sec. 3.4, 5.1, Fig. 5)
 * -- the device's constant 100 MHz wall clock when its workgroup started and
 * when it ended: stamps[2i], stamps[2i+1] (device memory, n_stamps >= 2 x the
 * number of items, which is covest_counts' n_uc).  If items is non-null
 * (host, 5 int32 per item: inst, dr, dc, bulk0, bulk1) it receives the items
 * in stamp order.  The stamps cost one branch per workgroup; every other
 * entry point passes none.  Errors as covest_forward, plus
 * COVEST_ERR_INVALID_ARG for too few stamps. */
int covest_forward_stamped(const void *A, int64_t N, int64_t M, int64_t P, int64_t Q, void *R,
                           const covest_opts *opts, void *ws, size_t ws_bytes, uint64_t *stamps,
                           int64_t n_stamps, int32_t *items, hipStream_t stream);

/* Plan of the plain form's 16-bit matrix-core path (prec: COVEST_PREC_BF16X3,
 * _FP16X3, _BF16 or _FP16) for n_cu compute units.  A is first split into
 * npl packed planes of N rows with row stride ldp; each item sums the
 * positions [p0, p1) x [q0, q1) of one tm x tn output tile, staging pb
 * position rows x qb position columns of A at a time in LDS (row strides
 * stride_a and stride_b); tile t adds the partial tiles of the items listed
 * in item_index[item0 .. item1); one workgroup runs each item.  Rows:
 * items 6 int32 each (tr, tc, p0, p1, q0, q1), tiles 4 int32 each (tr, tc,
 * item0, item1).  Arrays may be null.  COVEST_ERR_UNSUPPORTED for FP64 or
 * FP32 (FP32 keeps 64 x 64 tiles). */
typedef struct {
    int32_t pb, qb, stride_a, stride_b, tm, tn, npl, ldp;
    int32_t n_items, n_tiles, n_index;
    int64_t lds, ws_bytes, planes_bytes;
} covest_hankel_plan_info;
int covest_hankel_plan_get(int64_t N, int64_t M, int64_t P, int64_t Q, int32_t prec, int32_t n_cu,
                           covest_hankel_plan_info *out, int32_t *items, int32_t *tiles, int32_t *item_index);

/* The engine COVEST_ENGINE_AUTO picks for one problem (batch = 0) or for a
 * problem of a batched plan (batch = 1): *engine = COVEST_ENGINE_VECTOR or
 * COVEST_ENGINE_MATRIX.  *fits = 1 when the matrix-core engine can run the
 * shape at all (what COVEST_ENGINE_MATRIX accepts).  Host only; ignores the
 * 2^31-element offset limit, which depends on lda. */
int covest_engine_choice(int64_t N, int64_t M, int64_t P, int64_t Q, int32_t batch, int32_t *engine,
                         int32_t *fits);

/* Plan of the lane engine (COVEST_ENGINE_LANE) for a grid of n_rows x n_cols
 * inputs of N x M at row step row_step (a single input: 1 x 1) on n_cu
 * compute units: whether the engine fits the shape, the register array of
 * column offsets (qmax), the second-factor ring rows and LDS row stride
 * (complex64 elements), the row steps per staged chunk, the dynamic LDS
 * bytes, the inputs per workgroup along a grid column (chain; the
 * environment's COVEST_AP_CHAIN is not applied here), the workgroups and the
 * threads per workgroup.  COVEST_ERR_SHAPE on a bad shape or grid. */
typedef struct {
    int32_t fits, qmax, ring, gstride, chunk, chain, n_blocks, threads;
    int64_t lds;
} covest_lane_plan_info;
int covest_lane_plan_get(int64_t N, int64_t M, int64_t P, int64_t Q, int64_t row_step, int64_t n_rows,
                         int64_t n_cols, int32_t n_cu, covest_lane_plan_info *out);

#ifdef __cplusplus
}
#endif

#endif /* COVEST_PLAN_H */
