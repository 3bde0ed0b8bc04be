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

// One work item: a tile of R with rows [tr, tr+TM) and columns [tc, tc+TN)
// (64 x 64 for FP32, 128 x 128 or 128 x 64 for the 16-bit forms), summed over
// the window positions (p, q) with p in [p0, p1) and q in [q0, q1).
struct HItem {
    int tr, tc, p0, p1, q0, q1;
};

// 16-bit forms: an item's FP32 accumulators sum at most this many positions
// (each matrix-core step rounds once per 8 positions); the split-K reduction
// adds the items' partial tiles in FP64.  The plain BF16 / FP16 forms, whose
// error is that of their 16-bit inputs, take twice as many; small-integer
// inputs stay exact either way (|sum| < 2^24).
constexpr int kItemPositions16 = 16384;
constexpr int kItemPositionsPlain16 = 32768;
inline int item_positions16(int prec)
{
    return prec == kPrecBF16 || prec == kPrecF16 ? kItemPositionsPlain16 : kItemPositions16;
}

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
    double *partial;          // FP32 form: [n_items][64*64] complex FP64
    // 16-bit forms
    const unsigned int *planes;   // [npl][N][ldp] packed (re, im) pairs: hi plane, then lo plane
    int64_t plane_elems;          // N * ldp
    int ldp;                      // plane row stride: M plus zero columns the staging may read
    float2 *partial32;            // [n_items][128 * tn] complex FP32
    int tn;                       // tile columns: 128 or 64
    const int *item_index;        // tile t sums partial32 of items item_index[item0 .. item1)
    void *R;                  // complex64, row stride ldr
    int64_t ldr;
    int fill_full, normalize;
};

hipError_t launch_hankel_main(const HankelArgs &ha, int prec, int n_items, size_t lds, hipStream_t s);
hipError_t launch_hankel_reduce(const HankelArgs &ha, int n_tiles, hipStream_t s);
// 16-bit forms: B1 (A into packed 16-bit planes), B2 on 128-row tiles, B3.
hipError_t launch_hankel_split(const HankelArgs &ha, int prec, hipStream_t s);
hipError_t launch_hankel_main16(const HankelArgs &ha, int prec, int n_items, size_t lds, hipStream_t s);
hipError_t launch_hankel_reduce16(const HankelArgs &ha, int n_tiles, hipStream_t s);

}  // namespace covest
