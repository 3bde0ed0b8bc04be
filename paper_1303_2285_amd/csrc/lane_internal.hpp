// lane_internal.hpp -- the lane engine: one lane per unique combination,
// its entries by sliding a box sum over the window positions, for small
// inputs (the apertures of an image).  Shared by the host planner and the
// kernel.
#pragma once

#include <hip/hip_runtime.h>

#include <algorithm>
#include <cstddef>
#include <cstdint>

namespace covest {

constexpr int kLaneMaxQ = 16;       // column offsets per combination held in registers
constexpr int kLaneMaxLags = 512;   // unique combinations PQ + (P-1)(Q-1): one workgroup's lanes
constexpr int kLaneChunk = 4;       // row steps per staged chunk
constexpr int kLaneFBytes = 16;     // staged first factors: FP64
constexpr int kLaneGBytes = 8;      // staged second factors: complex64
constexpr size_t kLaneMaxLds = 64 * 1024;

// A grid of n_rows x n_cols inputs of N x M, input (a, b) starting at
// image[(a*row_step)*ld + b*col_step]; its R (PQ x PQ, row stride ldr) at
// R + (a*n_cols + b)*r_stride elements.  A single input is a 1 x 1 grid.
// Workgroup (chain c, column b) takes inputs a in [c*chain, c*chain + chain).
struct LaneArgs {
    const float2 *image;
    int64_t ld;
    int N, M, P, Q, Kr, Kc;
    int row_step, col_step, n_rows, n_cols;
    int chain;
    int n_lags;
    void *R;
    int64_t ldr, r_stride;
    int out_fp64, fill_full, normalize;
    int gstride;   // LDS row stride of the staged second-factor rows (elements)
    int ring;      // rows of each second-factor ring: kLaneChunk + P - 1
};

inline int lane_n_lags(int P, int Q) { return P * Q + (P - 1) * (Q - 1); }
inline int lane_ring(int P) { return kLaneChunk + P - 1; }
// Row stride of the second-factor rings: at least M + 2Q - 2, and 3 mod 16
// elements, which spreads the rows of neighbouring lags over the LDS banks
// (modelled: ~15% fewer bank conflicts than an odd stride at a 10 x 10 window).
inline int lane_gstride(int M, int Q)
{
    const int w = M + 2 * Q - 2;
    return w + ((3 - w % 16) + 16) % 16;
}

// Two second-factor rings (rows entering and leaving the box, complex64 with
// Q-1 zero columns on each side) and two chunks of first-factor rows (FP64).
// (FP64 rings measured 4% faster on the 1600² aperture grid and 5% slower on
// the dense one, at the cost of P = Q = 16 windows on rows of ~100.)
inline size_t lane_lds_bytes(int M, int P, int Q)
{
    return 2 * (size_t)lane_ring(P) * lane_gstride(M, Q) * kLaneGBytes + 2 * (size_t)kLaneChunk * M * kLaneFBytes;
}

inline int lane_qmax(int Q) { return Q <= 8 ? 8 : Q <= 12 ? 12 : 16; }

inline bool lane_fits(int N, int M, int P, int Q)
{
    return P >= 1 && Q >= 1 && P <= N && Q <= M && Q <= kLaneMaxQ && lane_n_lags(P, Q) <= kLaneMaxLags &&
           lane_lds_bytes(M, P, Q) <= kLaneMaxLds;
}

hipError_t prepare_lane_kernels();
hipError_t launch_lane(const LaneArgs &la, int n_blocks, size_t lds, hipStream_t stream);

}  // namespace covest
