// adj_internal.hpp -- types shared by the host and the adjoint kernels.
#pragma once

#include <cstdint>

#include <hip/hip_runtime.h>

namespace covest {

constexpr int kAdjTR = 8;    // interior outputs per workgroup: rows
constexpr int kAdjTC = 64;   // interior outputs per workgroup: columns (kAdjRing per thread)
constexpr int kAdjRing = 8;  // interior outputs per thread (a ring of A values along dc)
constexpr int kAdjFL = 64;   // outputs per line job of the frame
constexpr int kAdjFrameLds = 64 * 1024;   // LDS of a frame job when no interior tile shares its launch
constexpr int kAdjBatch = 4;  // frame: lags whose table reads a thread issues before using any
// Matrix-core interior (windows up to 16 x 16): a wave walks kAdjMRows input
// rows of one 16-column output tile; a workgroup's kAdjMWaves waves take
// consecutive rows, kAdjMSpan in all.
constexpr int kAdjMRows = 8;
constexpr int kAdjMWaves = 8;
constexpr int kAdjMSpan = kAdjMRows * kAdjMWaves;
constexpr int kAdjMMaxWin = 16;

struct AdjArgs {
    const float2 *A;
    int64_t lda;
    const void *G;              // dL/dR, PQ x PQ: complex128 (g_fp64) or complex64
    int64_t ldg;
    void *dA;                   // N x M: complex128 (g_fp64) or complex64
    int64_t ldda;
    int g_fp64;                 // 1: G and dA are complex128
    int upper;                  // 1: only G's entries with k2 >= k1 count (H = triu(G) + triu(G)^H)
    int N, M, P, Q, Kr, Kc;
    int ir0, ir1, ic0, ic1;     // interior outputs [ir0, ir1) x [ic0, ic1)
    int ndc;                    // 2Q-1 rounded up to a multiple of kAdjRing
    double *tables;             // [(2P-1)(2Q-1)][(P+1)(Q+1)] complex FP64 prefix sums
    double *hfull;              // [(2P-1)(2Q-1)] complex FP64 full sums
    int normalize;
    int frame_lds;              // dynamic LDS bytes of the launch the frame jobs run in
    // matrix-core interior: outputs y in [0, ny), x in [0, nx) are dA[y+P-1][x+Q-1];
    // mtiles 16-column tiles x mranges ranges of kAdjMSpan input rows
    int ny, nx, mtiles, mranges;
    double *bnd;                // [mranges-1][2][2P-2][16 mtiles] complex FP64 partial rows
    // frame: the weights of the line jobs, per border row (lags in (dr, dc)
    // order) and per border column (lags in (dc, dr) order), complex FP64
    double *wrows, *wcols;
};

// n_frame_jobs: the frame's row, column and corner jobs (adj_frame decodes
// its job from the block index and the interior bounds)
hipError_t launch_adjoint(const AdjArgs &aa, int n_lags, size_t lds_tables, int n_interior_blocks,
                          size_t lds_interior, int64_t n_frame_jobs, hipStream_t s);

// LDS per weight row of a frame line job whose weight rows have Y entries:
// the row (padded to kAdjRing, one spare) and its A values, and at least a
// row of the final sum over x rows (kAdjFL outputs).
__host__ __device__ inline size_t adj_line_row_bytes(int Y)
{
    const int Yp = (Y + kAdjRing - 1) / kAdjRing * kAdjRing;
    const size_t row = (size_t)(Yp + 1) * 16 + (size_t)((kAdjFL + Yp) | 1) * 8;
    return row > (size_t)kAdjFL * 16 ? row : (size_t)kAdjFL * 16;
}

// Bytes of LDS of the matrix-core interior (rings and staged rows) for a P x Q window.
inline size_t adj_mfma_lds(int P, int Q)
{
    const int ks = (2 * Q - 1 + 3) / 4;
    return (size_t)kAdjMWaves * (kAdjMRows + 2 * P - 2 + 1) * 16 * 16 + (size_t)kAdjMWaves * kAdjMRows * (4 * ks + 16) * 8;
}

// The matrix-core form: the tables, the interior's spans, then the frame's
// jobs together with the output rows two spans share.
hipError_t launch_adjoint_mfma(const AdjArgs &aa, int n_lags, size_t lds_tables, int64_t n_frame_jobs,
                               size_t lds_frame, hipStream_t s);

}  // namespace covest
