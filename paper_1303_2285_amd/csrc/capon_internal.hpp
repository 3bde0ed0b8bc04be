// capon_internal.hpp -- the minimum-variance (Capon) spectrum of a batch of
// estimated covariance matrices: shared by the host entry point and the kernel.
#pragma once

#include <hip/hip_runtime.h>

#include <cstddef>
#include <cstdint>

namespace covest {

constexpr int kCaponMaxPQ = 256;     // PQ at most
constexpr int kCaponLdsPQ = 128;     // up to this PQ the packed factor lives in LDS, above in the workspace
constexpr int kCaponMaxGrid = 4096;  // F1, F2 at most

// One workgroup per matrix.  LDS: the packed factor (n(n+1)/2, n <= 128
// only), two columns (2n) and the lag sums ((2P-1)(2Q-1)), complex128.
// Workspace per matrix: T (F1 x (2Q-1), the first DFT pass) and, for n > 128,
// the packed factor, complex128.
struct CaponArgs {
    const double2 *R;   // count x n x n, row-major
    double *S;          // count x F1 x F2
    double2 *T;         // count x F1 x (2Q-1)
    double2 *F;         // count x n(n+1)/2 (n > 128 only)
    int n, P, Q, F1, F2;
};

inline bool capon_factor_in_lds(int n) { return n <= kCaponLdsPQ; }

inline size_t capon_lds_bytes(int n, int P, int Q)
{
    const size_t tri = capon_factor_in_lds(n) ? (size_t)n * (n + 1) / 2 : 0;
    return 16 * (tri + 2 * (size_t)n + (size_t)(2 * P - 1) * (2 * Q - 1));
}

inline size_t capon_t_bytes(int Q, int F1) { return 16 * (size_t)F1 * (2 * Q - 1); }

inline size_t capon_ws_per_matrix(int n, int Q, int F1)
{
    return capon_t_bytes(Q, F1) + (capon_factor_in_lds(n) ? 0 : 16 * ((size_t)n * (n + 1) / 2));
}

hipError_t launch_capon(const CaponArgs &ca, int count, hipStream_t stream);

}  // namespace covest
