// covest_internal.hpp -- types shared by the host planner and the HIP kernels.
//
// Vocabulary (Sec. 3 of the paper):
//   combination  lag (dr, dc) between the two factors of a product; every
//                upper-triangle entry of R belongs to exactly one unique
//                combination (eq. 3.3): dc >= 1, or dc = 0 with dr >= 0.
//   type A       the unique combinations with 0 <= dr < P, 0 <= dc < Q
//   type B       the unique combinations with -P < dr < 0, 1 <= dc < Q
//
// Work split.  For combination (dr, dc) the entry at window offset (i1, j1) is
// the sum of the product grid Pi[r][c] = A[r][c] * conj(A[r+dr][c+dc]) over the
// box of first-factor positions [i1, i1+Kr) x [j1, j1+Kc).  Every box contains
// the "middle" rows [Rm0, Rm1) and columns [Cm0, Cm1) (Rm0 >= P-1, Rm1 <= N-P+1,
// likewise for columns).  The remaining rows and columns are "individual".  So
//   - bulk jobs sum Pi over middle rows x middle columns (one number per lag),
//   - row-strip jobs sum Pi over middle columns for each individual row,
//   - column-strip jobs sum Pi over middle rows for each individual column,
// and the finalize pass adds the corner products (individual row and column)
// itself and slides the box over the window offsets: one step adds the row (or
// column) of sums that enters and subtracts the one that leaves (Sec. 3.3).
#pragma once

#include <cstdint>

namespace covest {

constexpr int kWaves = 4;          // waves per workgroup of the main kernel
constexpr int kThreads = 64 * kWaves;
constexpr int kFinMaxRows = 160;   // individual rows the table finalize handles (n_ir)
// finalize variants: LDS table (16 corner loads per thread in flight), one
// wave per combination, LDS table for at most kFinSmallCorners corner
// products, wave prefix sums (at most 63 individual columns and 63 rows),
// wave prefix sums for at most 31 individual rows (fewer registers)
enum { kFinTable = 0, kFinLean = 1, kFinTableSmall = 2, kFinScan = 3, kFinScanSmall = 4, kFinVariants = 5 };
constexpr int kFinSmallCorners = 4 * 256;

// A set of lanes of one wave slot: lane li has
//   d1 = d1lo + li / nch,   d2 chunk start = ch0 + (li % nch) * W
// and accumulates the W lags (d1, chunk + w).  In orientation 0 the walk runs
// along A's columns: (d1, d2) = (dr, dc).  In orientation 1 it runs along A's
// rows on the transposed input B = A^T: (d1, d2) = (dc, dr).
struct LagGroup {
    int orient;     // 0 or 1
    int W;          // ring width (4, 8, 12 or 16)
    int d1lo, d1hi; // [d1lo, d1hi)
    int ch0, nch;   // first chunk start and number of chunks
    int v2lo, v2hi; // lags with d2 outside [v2lo, v2hi) are computed but dropped
    int lanes;      // (d1hi - d1lo) * nch, at most 64
    int slots;      // 64 / lanes: independent rows per wave
    int hr_lo, hr_hi;  // tile rows: [x0 + hr_lo, x1 + hr_hi)
    int hc_lo, hc_hi;  // tile cols: [c0 + hc_lo, c1 + hc_hi)
};

enum JobMode : int { kJobBulk = 0, kJobStrip = 1 };

// One workgroup's work in the main kernel.
//   bulk:  units [u0, u1) of the middle region in band-major order; a unit is
//          one group of `slots` consecutive middle rows times one band of
//          kWaves*W middle columns.  Output: partial sums of every lag of the
//          group into partial row `out`.
//   strip: B rows [x0, x1) (at most kWaves*slots, one per wave slot), walked
//          over B columns [c0, c1).  Output: one row of sums per B row, into
//          strip row `out + (b_row - x0)`.
struct Job {
    int mode;
    int inst;
    int group;     // index into the LagGroup table
    int out;
    int u0, u1;
    int x0, x1;
    int c0, c1;
    int tile_rows; // bulk: rows per LDS sub-tile; strip: unused
    int tile_cols; // strip: B columns per LDS sub-tile; bulk: unused
    int pad0, pad1;
};

// One problem of the (possibly batched) workload, with its workspace layout.
struct Inst {
    const void *A;   // complex64, row stride lda
    void *R;         // complex128 or complex64, row stride ldr
    int64_t lda, ldr;
    int N, M, P, Q;
    int Kr, Kc;
    int Rm0, Rm1, Cm0, Cm1;   // middle rows / columns (see above)
    int n_ir, n_ic;           // individual rows / columns
    int lag_stride;           // (2P-1)*Q: canonical lag index (dr+P-1)*Q + dc
    int bandw;                // bulk band width in columns (kWaves * W of orientation 0)
    int slots0;               // slots of the orientation-0 groups (rows per bulk unit)
    double *partial;          // [n_bulk_jobs][lag_stride] complex FP64 (as 2 doubles)
    double *zr;               // [n_ir][lag_stride]
    double *zc;               // [n_ic][lag_stride]
    int out_fp64;             // R element: 1 complex128, 0 complex64
    int fill_full;            // 1: write the conjugate mirror too
    int normalize;            // 1: divide by K
    int zpieces;              // strip sums come in this many pieces: zr[piece][n_ir][lag]
};

// One finalize work item: a unique combination of one instance.
struct FinItem {
    int inst;
    int dr, dc;
    int bulk0, bulk1;   // partial rows that hold this lag's middle sums
};

struct MainArgs {
    const Job *jobs;
    const LagGroup *groups;
    const Inst *insts;
    int n_jobs;
    int xcd_remap;     // 1: give each XCD a contiguous block of jobs
    int use_inline;    // 1: every job uses inst_inline (single-problem calls)
    int pad;
    Inst inst_inline;
};

// ---------------------------------------------------------------------------
// Matrix-core form of the main pass.  For one first-factor line (a row of A in
// orientation 0, a column in orientation 1) the sums over a range of positions
// of every lag form a dense product:
//     T[d1][d2] = sum_{c'} conj(B[line + d1][c']) * x[c' - d2],
// with B = A (or A^T), c' the second factor's position and x the line itself,
// zero outside the position range.  The first operand is a block of 16 lines
// at one position (rows of B), the second a Toeplitz band of the line: both
// are read straight from A, and every product is still formed exactly once.
// A workgroup has kMWaves waves; wave w takes line line0 + kMWaves*blk + w of
// every block blk it visits, so the waves of a workgroup read neighbouring
// lines at the same positions.
constexpr int kMWaves = 8;
constexpr int kMThreads = 64 * kMWaves;
constexpr int kMXCap = 2048;   // first factors staged per wave (float2), orientation 0

enum MJobKind : int { kMBulk = 0, kMStrip = 1 };

// One workgroup of the matrix-core main kernel.  It visits the (block,
// k-group) pairs from (b0, kg0) up to, not including, (b1, kg1) in
// lexicographic order; a k-group is 4 consecutive second-factor positions
// starting at k0.  bulk: lines are middle lines, every wave's sums are added
// into partial row `out`.  strip: one block (b0 == b1 == 0); each wave writes
// its line's sums to z row out + (line - line0) (the piece is part of out).
struct MJob {
    int inst;
    int orient;          // 0: lines are rows of A, 1: columns
    int kind;            // MJobKind
    int out;
    int line0, line_end; // lines >= line_end are skipped
    int b0, kg0, b1, kg1;
    int n_kg;            // k-groups per line
    int pos_lo, pos_hi;  // first-factor positions [pos_lo, pos_hi) on every line
    int k0;              // second-factor position of k-group 0, lane 0
    int kin;             // k-groups [0, kin) have all 4 positions inside the line
                         // (loaded unchecked); later ones are clamped to its end
    int pad1;
};

// The problem descriptor travels in the kernel arguments, so that its fields
// (and everything derived from them) stay in scalar registers.
struct MfmaArgs {
    const MJob *jobs;
    int n_jobs;
    int xcd_remap;
    const Inst *insts;   // batches: job.inst indexes this table; single problems: null, inst below
    Inst inst;
};

struct FinArgs {
    const FinItem *items;
    const Inst *insts;
    int n_items;
    int use_inline;
    Inst inst_inline;
    unsigned long long *stamps;   // measurement runs only (else null): per item, the
                                  // 100 MHz wall clock at its workgroup's start and end
};

}  // namespace covest
