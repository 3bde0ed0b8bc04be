// hankel_internal.hpp -- types shared by the host planner and the matrix-core
// kernels of the plain (Hankel product) form.
#pragma once

#include <cstdint>

#include <hip/hip_runtime.h>

namespace covest {

// Matrix-core precisions of the plain form.
enum HankelPrec : int { kPrecF32 = 0, kPrecBF16 = 1, kPrecBF16x3 = 2, kPrecF16 = 3, kPrecF16x3 = 4 };

// FP32 accumulation inside the matrix core covers at most this many window
// positions before it is added into FP64 registers.
constexpr int kFlushPositions = 256;

// One work item: the 64 x 64 tile of R with rows [tr, tr+64) and columns
// [tc, tc+64) (tr <= tc), summed over window positions with p in [p0, p1).
struct HItem {
    int tr, tc, p0, p1;
};

// One output tile and the range of items whose partial tiles it sums.
struct HTile {
    int tr, tc, item0, item1;
};

struct HankelArgs {
    const float2 *A;
    int64_t lda;
    int N, M, P, Q, PQ, Kr, Kc;
    int pb, qb;               // LDS sub-tile: pb position rows x qb position columns
    int stride_a, stride_b;   // padded LDS row strides (4-byte elements)
    const HItem *items;
    const HTile *tiles;
    double *partial;          // [n_items][64*64] complex FP64
    void *R;                  // complex64, row stride ldr
    int64_t ldr;
    int fill_full, normalize;
};

hipError_t launch_hankel_main(const HankelArgs &ha, int prec, int n_items, size_t lds, hipStream_t s);
hipError_t launch_hankel_reduce(const HankelArgs &ha, int n_tiles, hipStream_t s);

}  // namespace covest
