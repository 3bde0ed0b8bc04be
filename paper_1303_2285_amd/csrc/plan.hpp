// plan.hpp -- host-side planning of the recurrence: unique combinations,
// lag groups, the middle / individual split, the job list of the main kernel
// and the finalize items.  No HIP calls; usable without a GPU.
#pragma once

#include <cstddef>
#include <cstdint>
#include <vector>

#include "covest_internal.hpp"
#include "hankel_internal.hpp"

namespace covest {

struct Counts {
    int64_t K, n_uc, um, eta, segments;
};

// Sec. 3.2-4.1 counts: K positions, |UC| (eq. 3.4), UM = sum of
// (N-|dr|)(M-|dc|) over UC (eqs. 3.5-3.6), eta = PQ(PQ+1)/2 (eq. 4.22) and the
// number of diagonal segments, sum of Q-|dc| over UC.
Counts method_counts(int64_t N, int64_t M, int64_t P, int64_t Q);

// Plan of one problem shape.  Job::inst is 0, outputs are relative to this
// shape's own workspace; batched plans offset them.
struct ShapePlan {
    int engine = 1;                      // 1: vector ring walk (rec_main), 2: matrix cores (rec_mfma)
    int N = 0, M = 0, P = 0, Q = 0;
    int W0 = 0, W1 = 0;
    int Rm0 = 0, Rm1 = 0, Cm0 = 0, Cm1 = 0, n_ir = 0, n_ic = 0;
    int lag_stride = 0, bandw = 0, slots0 = 0;
    int n_bulk = 0;                      // partial rows
    std::vector<LagGroup> groups;
    std::vector<Job> jobs;
    std::vector<FinItem> items;
    std::vector<double> job_cost;        // estimated wave-steps per job
    size_t lds_main = 0, lds_fin = 0;
    int fin_variant = 1;                 // kFinTable, kFinLean, kFinTableSmall, kFinScan or kFinScanSmall
    size_t ws_bytes = 0;                 // partial + zr + zc, FP64 complex
    int64_t main_products = 0;           // distinct products the main kernel keeps
    int64_t fin_products = 0;            // corner products the finalize computes
    // matrix-core engine only
    int mt = 0, nt = 0;                  // 16 x 16 tiles of the orientation-0 lag block (d1 = dr, d2 = dc)
    int zpieces = 1;                     // pieces per strip line
    std::vector<MJob> mjobs;
};

// n_slots: workgroups resident at once on the target device (2 per CU).
// w0 / w1 override the ring widths along columns / rows (0: the default choice).
ShapePlan make_shape_plan(int N, int M, int P, int Q, int n_slots, int w0 = 0, int w1 = 0);

// Matrix-core plan: one workgroup of kMWaves waves per compute unit (n_cu).
// Valid when mfma_fits(N, M, P, Q).  job_units > 0 (batches): jobs of about
// that many 8-line k-group steps instead of one job per compute unit.
ShapePlan make_mfma_plan(int N, int M, int P, int Q, int n_cu, double job_units = 0.0);

// The matrix-core engine needs a non-empty middle block and a lag block of at
// most 8 tiles (one wave holds all its sums); min_fill: the least share of
// the tiles' lags that are real (0: any).
bool mfma_fits(int N, int M, int P, int Q, double min_fill = 0.0);

// AUTO's choice of the matrix cores for a shape the kernel can run (measured
// on MI355X, both engines on the same inputs): a single problem almost always
// runs faster there, down to 4 x 4 windows (the vector engine's many small
// jobs cost more than the padding of a 16 x 16 tile), except lag blocks of 7
// or 8 tiles that are three quarters padding (P = 56..64 with Q = 4); in a
// batch the vector kernel's jobs fill the GPU better, and only windows whose
// tiles are at least 70% real go to the matrix cores.
bool mfma_preferred(int N, int M, int P, int Q, bool batch);

// Ring widths worth trying for a window extent n (the first is the default).
std::vector<int> ring_width_candidates(int n);

// Plan of the plain (matrix-core) form for one shape and precision.
struct HankelPlan {
    int N = 0, M = 0, P = 0, Q = 0, prec = 0;
    int pb = 0, qb = 0, stride_a = 0, stride_b = 0;
    std::vector<HItem> items;
    std::vector<HTile> tiles;
    size_t lds = 0;
    size_t ws_bytes = 0;     // FP32: FP64 partial tiles; 16-bit: planes + FP32 partial tiles
    // 16-bit forms
    int tm = 64, tn = 64;    // tile rows and columns
    int npl16 = 0;           // packed planes of A (1 plain, 2 split)
    int ldp = 0;             // plane row stride (elements)
    size_t planes_bytes = 0; // offset of the partial tiles in the workspace
    std::vector<int> item_index;   // tile t sums items item_index[tiles[t].item0 .. item1)
};

// n_cu: compute units of the device (work items are sized for ~8 per CU).
HankelPlan make_hankel_plan(int N, int M, int P, int Q, int prec, int n_cu);

// Limits of the recurrence form.
constexpr int kMaxWindow = 64;           // P, Q <= kMaxWindow
constexpr size_t kLdsBudget = 72 * 1024; // per workgroup, so two fit in 160 KB
constexpr size_t kFinTableMax = 96 * 1024;  // largest LDS table of the table finalize

}  // namespace covest
