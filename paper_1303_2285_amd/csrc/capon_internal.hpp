// capon_internal.hpp -- the minimum-variance (Capon) spectrum of a batch of
// estimated covariance matrices: shared by the host entry point and the kernel.
#pragma once

#include <hip/hip_runtime.h>

#include <cstddef>
#include <cstdint>

namespace covest {

constexpr int kCaponMaxPQ = 128;     // the packed Cholesky factor lives in LDS
constexpr int kCaponMaxGrid = 4096;  // F1, F2 at most

// One workgroup per matrix.  LDS: the packed factor (n(n+1)/2), one column
// (n) and the lag sums ((2P-1)(2Q-1)), complex128.  Workspace per matrix: T
// (F1 x (2Q-1), the first DFT pass), complex128.
struct CaponArgs {
    const double2 *R;   // count x n x n, row-major
    double *S;          // count x F1 x F2
    double2 *T;         // count x F1 x (2Q-1)
    int n, P, Q, F1, F2;
};

inline size_t capon_lds_bytes(int n, int P, int Q)
{
    return 16 * ((size_t)n * (n + 1) / 2 + (size_t)n + (size_t)(2 * P - 1) * (2 * Q - 1));
}

inline size_t capon_ws_per_matrix(int n, int Q, int F1)
{
    (void)n;
    return 16 * (size_t)F1 * (2 * Q - 1);
}

hipError_t launch_capon(const CaponArgs &ca, int count, hipStream_t stream);

}  // namespace covest
