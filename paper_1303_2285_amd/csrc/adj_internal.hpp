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
};

// n_frame_jobs: the frame's row, column and corner jobs (adj_frame decodes
// its job from the block index and the interior bounds)
hipError_t launch_adjoint(const AdjArgs &aa, int n_lags, size_t lds_tables, int n_interior_blocks,
                          size_t lds_interior, int64_t n_frame_jobs, hipStream_t s);

}  // namespace covest
