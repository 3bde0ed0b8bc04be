// hankel_kernels.hip -- kernel family b: R = X X^H / K as a dense product on
// the CDNA4 matrix cores (gfx950).
//
// This is the plain method of the paper (eq. 2.2 as a matrix product, every
// product recomputed for every window position; Sec. 4.1 counts its work).
// Row k = i + P*j of X at window position (p, q) is A[p+i][q+j] (eq. 2.1), so
// the operand tiles of X are read straight from rectangles of A staged in LDS:
// no im2col buffer exists.
//
// Complex arithmetic on real matrix cores: the MFMA reduction dimension holds
// (position, real/imaginary part) pairs.  With a = x1 and b = x2 = (re, im),
//   Re(x1 conj(x2)) = x1.re x2.re + x1.im x2.im   -> B operand (re, im)
//   Im(x1 conj(x2)) = x1.re (-x2.im) + x1.im x2.re -> B operand (-im, re)
// so one A operand feeds two products, one per part.
//
// Precisions (template parameter):
//   kPrecF32    v_mfma_f32_32x32x2_f32, one position per instruction
//   kPrecBF16   v_mfma_f32_32x32x16_bf16, 8 positions per instruction, hi only
//   kPrecBF16x3 hi*hi + hi*lo + lo*hi with x = hi + lo in bf16
//   kPrecF16    v_mfma_f32_32x32x16_f16, hi only
//   kPrecF16x3  hi*hi + (hi*lo + lo*hi) * 2^-11, lo stored scaled by 2^11
//
// FP32 (hankel_main): 64 x 64 tiles, A converted while it is staged, FP32
// accumulation inside the matrix core for kFlushPositions positions, then FP64
// registers; each item writes an FP64 partial tile, hankel_reduce sums them.
//
// 16-bit forms (hankel_split, hankel_main16, hankel_reduce16): A is split
// once into packed 16-bit planes (B1), so staging is a plain copy; a wave owns
// a 64 x 64 block (64 x 32 for FP16x3) and every operand it reads feeds four
// (two) matrix instructions; the FP32 accumulators sum one item of at most
// item_positions16(prec) positions, and the reduction adds the items' FP32 partial
// tiles in FP64 in a fixed order (B3).
#include <hip/hip_runtime.h>
#include <hip/hip_bf16.h>
#include <hip/hip_fp16.h>

#include "device_util.hpp"
#include "hankel_internal.hpp"

namespace covest {

typedef float floatx4 __attribute__((ext_vector_type(4)));
typedef float floatx16 __attribute__((ext_vector_type(16)));
typedef __bf16 bf16x8 __attribute__((ext_vector_type(8)));
typedef _Float16 halfx8 __attribute__((ext_vector_type(8)));
typedef unsigned int uintx4 __attribute__((ext_vector_type(4)));

constexpr int kHThreads = 256;
// 64-column chunks of one staged row of the 16-bit forms (sub-tile width up
// to 256 positions plus a column span below 64)
constexpr int kStageChunks = 5;
// workgroups per output tile in the 16-bit reduction (128 / this many rows each)
constexpr int kReduceChunks = 32;

template <int PREC> struct PrecTraits;
template <> struct PrecTraits<kPrecF32> { static constexpr int planes = 3, step = 4; static constexpr bool split = false, half = false; };
template <> struct PrecTraits<kPrecBF16> { static constexpr int planes = 2, step = 8; static constexpr bool split = false, half = false; };
template <> struct PrecTraits<kPrecBF16x3> { static constexpr int planes = 4, step = 8; static constexpr bool split = true, half = false; };
template <> struct PrecTraits<kPrecF16> { static constexpr int planes = 2, step = 8; static constexpr bool split = false, half = true; };
template <> struct PrecTraits<kPrecF16x3> { static constexpr int planes = 4, step = 8; static constexpr bool split = true, half = true; };

// 16-bit conversions (round to nearest even)
__device__ __forceinline__ unsigned short f2bf(float x)
{
    const unsigned int u = __float_as_uint(x);
    if ((u & 0x7f800000u) == 0x7f800000u) return (unsigned short)((u >> 16) | ((u & 0xffff) ? 0x40 : 0));
    const unsigned int r = u + 0x7fffu + ((u >> 16) & 1u);
    return (unsigned short)(r >> 16);
}
__device__ __forceinline__ float bf2f(unsigned short h) { return __uint_as_float((unsigned int)h << 16); }
__device__ __forceinline__ unsigned short f2h(float x)
{
    const _Float16 h = (_Float16)x;
    return __builtin_bit_cast(unsigned short, h);
}
__device__ __forceinline__ float h2f(unsigned short h) { return (float)__builtin_bit_cast(_Float16, h); }

__device__ __forceinline__ unsigned int pack2(unsigned short lo, unsigned short hi)
{
    return (unsigned int)lo | ((unsigned int)hi << 16);
}

// Planes of one staged element x = (re, im):
//   F32:   [0] re, [1] im, [2] -im                         (float each)
//   16-bit: [0] (re, im) hi, [1] (-im, re) hi, [2] (re, im) lo, [3] (-im, re) lo
template <int PREC>
__device__ __forceinline__ void make_planes(float re, float im, unsigned int (&pl)[4])
{
    if constexpr (PREC == kPrecF32) {
        pl[0] = __float_as_uint(re);
        pl[1] = __float_as_uint(im);
        pl[2] = __float_as_uint(-im);
        pl[3] = 0;
    } else {
        constexpr bool half = PrecTraits<PREC>::half;
        const unsigned short rh = half ? f2h(re) : f2bf(re);
        const unsigned short ih = half ? f2h(im) : f2bf(im);
        const unsigned short nih = (unsigned short)(ih ^ 0x8000u);   // exact negation
        pl[0] = pack2(rh, ih);
        pl[1] = pack2(nih, rh);
        if constexpr (PrecTraits<PREC>::split) {
            const float rhf = half ? h2f(rh) : bf2f(rh);
            const float ihf = half ? h2f(ih) : bf2f(ih);
            const float sc = half ? 2048.0f : 1.0f;   // fp16 lo kept in the normal range
            const unsigned short rl = half ? f2h((re - rhf) * sc) : f2bf(re - rhf);
            const unsigned short il = half ? f2h((im - ihf) * sc) : f2bf(im - ihf);
            const unsigned short nil = (unsigned short)(il ^ 0x8000u);
            pl[2] = pack2(rl, il);
            pl[3] = pack2(nil, rl);
        } else {
            pl[2] = pl[3] = 0;
        }
    }
}

// Four consecutive 4-byte LDS elements; the start need only be 4-byte aligned
// (a lane's window column offset can be odd).
__device__ __forceinline__ uintx4 ld4(const unsigned int *p)
{
    uintx4 v;
    v[0] = p[0];
    v[1] = p[1];
    v[2] = p[2];
    v[3] = p[3];
    return v;
}

__device__ __forceinline__ floatx16 mfma_f32(float a, float b, floatx16 c)
{
    return __builtin_amdgcn_mfma_f32_32x32x2f32(a, b, c, 0, 0, 0);
}

template <bool HALF>
__device__ __forceinline__ floatx16 mfma16(uintx4 a, uintx4 b, floatx16 c)
{
    if constexpr (HALF)
        return __builtin_amdgcn_mfma_f32_32x32x16_f16(__builtin_bit_cast(halfx8, a), __builtin_bit_cast(halfx8, b), c, 0, 0, 0);
    else
        return __builtin_amdgcn_mfma_f32_32x32x16_bf16(__builtin_bit_cast(bf16x8, a), __builtin_bit_cast(bf16x8, b), c, 0, 0, 0);
}

// FP32 form.  One work item: a 64 x 64 tile of R over window positions with
// p in [p0, p1); wave w owns the 32 x 32 block (w >> 1, w & 1) of the tile.
// The FP32 matrix instruction takes one position per lane half, so each
// operand read feeds 8 instructions and the staging cost is small beside them.
template <int PREC>
__global__ void __launch_bounds__(kHThreads, 2) hankel_main(HankelArgs ha)
{
    static_assert(PREC == kPrecF32, "the 16-bit forms run hankel_main16");
    using T = PrecTraits<PREC>;
    constexpr int NPL = T::planes;
    extern __shared__ unsigned int hl[];
    const HItem it = ha.items[blockIdx.x];
    const int P = ha.P, Q = ha.Q, PQ = ha.PQ, Kc = ha.Kc;
    const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
    const int h = lane >> 5, m = lane & 31;

    // column windows of A needed by the tile's rows (A operand) and columns (B operand)
    const int ja_lo = it.tr / P, ja_hi = min(Q - 1, min(PQ - 1, it.tr + 63) / P);
    const int jb_lo = it.tc / P, jb_hi = min(Q - 1, min(PQ - 1, it.tc + 63) / P);
    const bool same = it.tr == it.tc;
    const int PB = ha.pb, QB = ha.qb;
    const int rows = PB + P - 1;
    const int wa = QB + (ja_hi - ja_lo), wb = QB + (jb_hi - jb_lo);
    const int sa = ha.stride_a, sb = ha.stride_b;           // padded row strides (elements)
    const int plane_a = (rows + 1) * sa, plane_b = (rows + 1) * sb;
    unsigned int *LA = hl;
    unsigned int *LB = same ? hl : hl + NPL * plane_a;

    // This lane's row (A) and column (B) of X; out-of-range rows read a zero row.
    const int ka = it.tr + 32 * (wave >> 1) + m;
    const int kb = it.tc + 32 * (wave & 1) + m;
    const int base_a = ka < PQ ? (ka % P) * sa + (ka / P - ja_lo) : rows * sa;
    const int base_b = kb < PQ ? (kb % P) * sb + (kb / P - jb_lo) : rows * sb;
    const int step_a = ka < PQ ? sa : 0, step_b = kb < PQ ? sb : 0;   // the zero row stays put

    floatx16 acc_re = {}, acc_im = {};
    double dre[16], dim[16];
#pragma unroll
    for (int r = 0; r < 16; ++r) dre[r] = dim[r] = 0.0;
    int since_flush = 0;

    auto flush = [&]() {
#pragma unroll
        for (int r = 0; r < 16; ++r) {
            dre[r] += (double)acc_re[r];
            dim[r] += (double)acc_im[r];
        }
        acc_re = floatx16{};
        acc_im = floatx16{};
        since_flush = 0;
    };

    for (int ps = it.p0; ps < it.p1; ps += PB) {
        const int pe = min(it.p1, ps + PB);
        for (int qs = 0; qs < Kc; qs += QB) {
            const int qe = min(Kc, qs + QB);
            __syncthreads();
            // stage rows [ps, ps + rows) of A, columns [qs + j_lo, qs + j_lo + w)
            for (int win = 0; win < (same ? 1 : 2); ++win) {
                unsigned int *L = win ? LB : LA;
                const int jlo = win ? jb_lo : ja_lo;
                const int w = win ? wb : wa;
                const int s = win ? sb : sa;
                const int plane = win ? plane_b : plane_a;
                for (int e = threadIdx.x; e < (rows + 1) * w; e += kHThreads) {
                    const int rr = e / w, cc = e - rr * w;
                    const int ar = ps + rr, ac = qs + jlo + cc;
                    float2 v = make_float2(0.f, 0.f);
                    if (rr < rows && ar < ha.N && ac < ha.M) v = ha.A[(int64_t)ar * ha.lda + ac];
                    unsigned int pl[4];
                    make_planes<PREC>(v.x, v.y, pl);
#pragma unroll
                    for (int k = 0; k < NPL; ++k) L[k * plane + rr * s + cc] = pl[k];
                }
            }
            __syncthreads();
            for (int p = ps; p < pe; ++p) {
                const int roff_a = base_a + (p - ps) * step_a;
                const int roff_b = base_b + (p - ps) * step_b;
                for (int q = qs; q < qe; q += T::step) {
                    const int c = q - qs;
                    // lane half h: part h of x1 and x2, and part (-im | re) for Im
                    floatx4 a = __builtin_bit_cast(floatx4, ld4(&LA[h * plane_a + roff_a + c]));
                    const floatx4 b = __builtin_bit_cast(floatx4, ld4(&LB[h * plane_b + roff_b + c]));
                    const floatx4 b2 = __builtin_bit_cast(floatx4, ld4(&LB[(h ? 0 : 2) * plane_b + roff_b + c]));
                    if (q + 4 > qe) {
#pragma unroll
                        for (int t = 0; t < 4; ++t)
                            if (q + t >= qe) a[t] = 0.f;
                    }
#pragma unroll
                    for (int t = 0; t < 4; ++t) {
                        acc_re = mfma_f32(a[t], b[t], acc_re);
                        acc_im = mfma_f32(a[t], b2[t], acc_im);
                    }
                    since_flush += 4;
                    if (since_flush >= kFlushPositions) flush();
                }
            }
        }
    }
    flush();

    // FP64 partial tile of this item: element (row, col) of the 64 x 64 tile.
    // 32x32 accumulator layout: register r of lane l holds row 8*(r/4) + 4*(l/32) + r%4,
    // column l%32.
    double *out = ha.partial + (int64_t)blockIdx.x * 64 * 64 * 2;
#pragma unroll
    for (int r = 0; r < 16; ++r) {
        const int row = 32 * (wave >> 1) + 8 * (r >> 2) + 4 * h + (r & 3);
        const int col = 32 * (wave & 1) + m;
        reinterpret_cast<double2 *>(out)[row * 64 + col] = make_double2(dre[r], dim[r]);
    }
}

// Sum the partial tiles of every tile in item order, divide by K and store the
// upper triangle (and the conjugate mirror).
__global__ void __launch_bounds__(256) hankel_reduce(HankelArgs ha)
{
    const HTile t = ha.tiles[blockIdx.x];
    const double K = (double)ha.Kr * (double)ha.Kc;
    for (int e = threadIdx.x; e < 64 * 64; e += 256) {
        const int row = e >> 6, col = e & 63;
        const int k1 = t.tr + row, k2 = t.tc + col;
        if (k1 >= ha.PQ || k2 >= ha.PQ || k2 < k1) continue;
        double sr = 0.0, si = 0.0;
        for (int i = t.item0; i < t.item1; ++i) {
            const double2 v = reinterpret_cast<const double2 *>(ha.partial + (int64_t)i * 64 * 64 * 2)[e];
            sr += v.x;
            si += v.y;
        }
        if (ha.normalize) {
            sr = sr / K;
            si = si / K;
        }
        if (k1 == k2) si = 0.0;
        float2 *R = static_cast<float2 *>(ha.R);
        R[(int64_t)k1 * ha.ldr + k2] = make_float2((float)sr, (float)si);
        if (ha.fill_full && k1 != k2) R[(int64_t)k2 * ha.ldr + k1] = make_float2((float)sr, -(float)si);
    }
}

// ------------------------------------------------------- 16-bit forms ----
// B1: A once into packed 16-bit planes.  Plane 0 holds (re, im) hi of every
// element, plane 1 (split forms) its (re, im) lo (fp16 lo scaled by 2^11).
template <int PREC>
__global__ void __launch_bounds__(256) hankel_split(HankelArgs ha)
{
    constexpr bool half = PrecTraits<PREC>::half;
    for (int n = blockIdx.y; n < ha.N; n += gridDim.y) {
        for (int c = blockIdx.x * 256 + threadIdx.x; c < ha.ldp; c += gridDim.x * 256) {
            unsigned int pl[4] = {0u, 0u, 0u, 0u};     // padding columns hold zeros
            if (c < ha.M) {
                const float2 v = ha.A[(int64_t)n * ha.lda + c];
                make_planes<PREC>(v.x, v.y, pl);
            }
            unsigned int *dst = const_cast<unsigned int *>(ha.planes) + (int64_t)n * ha.ldp + c;
            dst[0] = pl[0];
            if constexpr (PrecTraits<PREC>::split) dst[ha.plane_elems] = pl[2];
        }
    }
}

// (re, im) -> (-im, re): the B operand of the imaginary part.
__device__ __forceinline__ unsigned int swap_neg(unsigned int x)
{
    return __builtin_amdgcn_alignbit(x, x, 16) ^ 0x8000u;
}

__device__ __forceinline__ uintx4 swap_neg4(uintx4 v)
{
    uintx4 r;
#pragma unroll
    for (int t = 0; t < 4; ++t) r[t] = swap_neg(v[t]);
    return r;
}

// B2 for the 16-bit forms.  One workgroup: the tile rows [tr, tr + 128) x
// columns [tc, tc + 64 WN) of R over the item's positions.  Wave w owns the
// 64 x 32 WN block (w >> 1, w & 1): two 32-row A fragments times WN 32-row B
// fragments, so every fragment read from LDS feeds 2 WN (A) or 4 (B) matrix
// instructions.  Accumulation stays in FP32 for the whole item; the item
// writes its partial tile and hankel_reduce16 adds the partials in FP64.
template <int PREC, int WN>
__global__ void __launch_bounds__(kHThreads, 2) hankel_main16(HankelArgs ha)
{
    using T = PrecTraits<PREC>;
    constexpr bool SPLIT = T::split, HALF = T::half;
    constexpr bool ACC2 = SPLIT && HALF;          // fp16 cross terms carry the 2^11 scale
    constexpr int NPL = SPLIT ? 2 : 1;
    constexpr int TN = 64 * WN;
    extern __shared__ unsigned int hl[];
    const int item = xcd_block(blockIdx.x, gridDim.x);
    const HItem it = ha.items[item];
    const int P = ha.P, Q = ha.Q, PQ = ha.PQ;
    const int tid = threadIdx.x, lane = tid & 63, wave = tid >> 6;
    const int h = lane >> 5, m = lane & 31;
    const bool same = TN == 128 && it.tr == it.tc;
    const int ja_lo = it.tr / P, ja_hi = min(Q - 1, min(PQ - 1, it.tr + 127) / P);
    const int jb_lo = it.tc / P, jb_hi = min(Q - 1, min(PQ - 1, it.tc + TN - 1) / P);
    const int rows = ha.pb + P - 1;                 // staged rows of A for pb position rows
    const int sa = ha.stride_a, sb = ha.stride_b;
    const int plane_a = (rows + 1) * sa, plane_b = (rows + 1) * sb;
    unsigned int *LA = hl;
    unsigned int *LB = same ? hl : hl + NPL * plane_a;

    // Row `rows` of every staged plane is a zero row: lanes whose row of X
    // lies past PQ read it at every position.
    for (int e = tid; e < sa; e += kHThreads)
#pragma unroll
        for (int k = 0; k < NPL; ++k) LA[k * plane_a + rows * sa + e] = 0u;
    if (!same)
        for (int e = tid; e < sb; e += kHThreads)
#pragma unroll
            for (int k = 0; k < NPL; ++k) LB[k * plane_b + rows * sb + e] = 0u;

    // This lane's rows of X: A fragments f (rows tr + 64 (w >> 1) + 32 f + m),
    // B fragments g (rows tc + 32 WN (w & 1) + 32 g + m).
    int oa[2], da[2], ob[WN], db[WN];
#pragma unroll
    for (int f = 0; f < 2; ++f) {
        const int k = it.tr + 64 * (wave >> 1) + 32 * f + m;
        oa[f] = k < PQ ? (k % P) * sa + (k / P - ja_lo) + 4 * h : rows * sa + 4 * h;
        da[f] = k < PQ ? sa : 0;
    }
#pragma unroll
    for (int g = 0; g < WN; ++g) {
        const int k = it.tc + 32 * WN * (wave & 1) + 32 * g + m;
        ob[g] = k < PQ ? (k % P) * sb + (k / P - jb_lo) + 4 * h : rows * sb + 4 * h;
        db[g] = k < PQ ? sb : 0;
    }

    floatx16 cre[2][WN], cim[2][WN], xre[2][WN], xim[2][WN];
#pragma unroll
    for (int f = 0; f < 2; ++f)
#pragma unroll
        for (int g = 0; g < WN; ++g) {
            cre[f][g] = floatx16{};
            cim[f][g] = floatx16{};
            if constexpr (ACC2) {
                xre[f][g] = floatx16{};
                xim[f][g] = floatx16{};
            }
        }

    const unsigned int *src_base = ha.planes;
    for (int ps = it.p0; ps < it.p1; ps += ha.pb) {
        const int np = min(it.p1, ps + ha.pb) - ps;   // position rows in this sub-block
        const int nrows = np + P - 1;                 // rows of A they read
        for (int qs = it.q0; qs < it.q1; qs += ha.qb) {
            const int cw = min(it.q1, qs + ha.qb) - qs;   // positions per row in this sub-block
            __syncthreads();
            // stage rows [ps, ps + nrows) x columns [qs + j_lo, qs + j_lo + cw + span) of the planes
#pragma unroll
            for (int side = 0; side < 2; ++side) {
                if (side == 1 && same) break;
                unsigned int *L = side ? LB : LA;
                const int jlo = side ? jb_lo : ja_lo;
                const int width = cw + (side ? jb_hi - jb_lo : ja_hi - ja_lo);
                const int s = side ? sb : sa;
                const int plane = side ? plane_b : plane_a;
                // rows ps + rr < N always (p < Kr, i < P); columns past M read the
                // planes' zero padding.  All chunks of a row are loaded before any is stored.
                // YR rows per wave per pass: their loads are all in flight before
                // the first store.
                constexpr int YR = SPLIT ? 2 : 4;
                for (int r4 = wave; r4 < nrows; r4 += YR * (kHThreads / 64)) {
                    unsigned int v[YR][kStageChunks][NPL];
#pragma unroll
                    for (int y = 0; y < YR; ++y) {
                        const int rr = r4 + y * (kHThreads / 64);
                        if (rr < nrows) {
                            const unsigned int *src = src_base + (int64_t)(ps + rr) * ha.ldp + qs + jlo + lane;
#pragma unroll
                            for (int u = 0; u < kStageChunks; ++u)
                                if (64 * u < width)
#pragma unroll
                                    for (int k = 0; k < NPL; ++k) v[y][u][k] = src[k * ha.plane_elems + 64 * u];
                        }
                    }
#pragma unroll
                    for (int y = 0; y < YR; ++y) {
                        const int rr = r4 + y * (kHThreads / 64);
                        if (rr < nrows) {
#pragma unroll
                            for (int u = 0; u < kStageChunks; ++u)
                                if (64 * u < width && lane + 64 * u < width)
#pragma unroll
                                    for (int k = 0; k < NPL; ++k) L[k * plane + rr * s + lane + 64 * u] = v[y][u][k];
                        }
                    }
                }
            }
            __syncthreads();
            for (int pr = 0; pr < np; ++pr) {
                const unsigned int *pa[2], *pbp[WN];
#pragma unroll
                for (int f = 0; f < 2; ++f) pa[f] = LA + oa[f] + pr * da[f];
#pragma unroll
                for (int g = 0; g < WN; ++g) pbp[g] = LB + ob[g] + pr * db[g];
                for (int c = 0; c < cw; c += 8) {
                    uintx4 a[2], al[2], b[WN], bl[WN];
#pragma unroll
                    for (int f = 0; f < 2; ++f) {
                        a[f] = ld4(pa[f] + c);
                        if constexpr (SPLIT) al[f] = ld4(pa[f] + plane_a + c);
                    }
#pragma unroll
                    for (int g = 0; g < WN; ++g) {
                        b[g] = ld4(pbp[g] + c);
                        if constexpr (SPLIT) bl[g] = ld4(pbp[g] + plane_b + c);
                    }
                    if (c + 8 > cw) {
                        // positions past the sub-block: zero both operands
#pragma unroll
                        for (int t = 0; t < 4; ++t) {
                            if (c + 4 * h + t >= cw) {
#pragma unroll
                                for (int f = 0; f < 2; ++f) {
                                    a[f][t] = 0u;
                                    if constexpr (SPLIT) al[f][t] = 0u;
                                }
#pragma unroll
                                for (int g = 0; g < WN; ++g) {
                                    b[g][t] = 0u;
                                    if constexpr (SPLIT) bl[g][t] = 0u;
                                }
                            }
                        }
                    }
#pragma unroll
                    for (int g = 0; g < WN; ++g) {
                        const uintx4 bi = swap_neg4(b[g]);
                        uintx4 bli = {};
                        if constexpr (SPLIT) bli = swap_neg4(bl[g]);
#pragma unroll
                        for (int f = 0; f < 2; ++f) {
                            cre[f][g] = mfma16<HALF>(a[f], b[g], cre[f][g]);
                            cim[f][g] = mfma16<HALF>(a[f], bi, cim[f][g]);
                            if constexpr (SPLIT && !ACC2) {
                                cre[f][g] = mfma16<HALF>(a[f], bl[g], cre[f][g]);
                                cre[f][g] = mfma16<HALF>(al[f], b[g], cre[f][g]);
                                cim[f][g] = mfma16<HALF>(a[f], bli, cim[f][g]);
                                cim[f][g] = mfma16<HALF>(al[f], bi, cim[f][g]);
                            } else if constexpr (ACC2) {
                                xre[f][g] = mfma16<HALF>(a[f], bl[g], xre[f][g]);
                                xre[f][g] = mfma16<HALF>(al[f], b[g], xre[f][g]);
                                xim[f][g] = mfma16<HALF>(a[f], bli, xim[f][g]);
                                xim[f][g] = mfma16<HALF>(al[f], bi, xim[f][g]);
                            }
                        }
                    }
                }
            }
        }
    }

    // FP32 partial tile of this item, element (row, col) of the 128 x TN tile.
    // 32x32 accumulator layout: register r of lane l holds row 8*(r/4) + 4*(l/32) + r%4,
    // column l%32.
    const int lane_off = (64 * (wave >> 1) + 4 * h) * TN + 32 * WN * (wave & 1) + m;
    float2 *out = ha.partial32 + (int64_t)item * 128 * TN + lane_off;
#pragma unroll
    for (int f = 0; f < 2; ++f)
#pragma unroll
        for (int g = 0; g < WN; ++g)
#pragma unroll
            for (int r = 0; r < 16; ++r) {
                const int row = 32 * f + 8 * (r >> 2) + (r & 3);
                const int col = 32 * g;
                float re = cre[f][g][r], im = cim[f][g][r];
                if constexpr (ACC2) {
                    re += xre[f][g][r] * (1.0f / 2048.0f);
                    im += xim[f][g][r] * (1.0f / 2048.0f);
                }
                out[row * TN + col] = make_float2(re, im);
            }
}

// B3 for the 16-bit forms: every tile sums its items' FP32 partial tiles in
// FP64, in item (position) order, divides by K and stores the upper triangle
// (and the conjugate mirror).
template <int TN>
__global__ void __launch_bounds__(256) hankel_reduce16(HankelArgs ha)
{
    // workgroup b: tile b / kReduceChunks, rows [RB c, RB c + RB) of it
    constexpr int RB = 128 / kReduceChunks;
    const HTile t = ha.tiles[blockIdx.x / kReduceChunks];
    const int r0 = (blockIdx.x % kReduceChunks) * RB;
    const double K = (double)ha.Kr * (double)ha.Kc;
    for (int e = r0 * TN + threadIdx.x; e < (r0 + RB) * TN; e += 256) {
        const int row = e / TN, col = e % TN;
        const int k1 = t.tr + row, k2 = t.tc + col;
        if (k1 >= ha.PQ || k2 >= ha.PQ || k2 < k1) continue;
        double sr = 0.0, si = 0.0;
        for (int i = t.item0; i < t.item1; ++i) {
            const float2 v = ha.partial32[(int64_t)ha.item_index[i] * 128 * TN + e];
            sr += (double)v.x;
            si += (double)v.y;
        }
        if (ha.normalize) {
            sr = sr / K;
            si = si / K;
        }
        if (k1 == k2) si = 0.0;
        float2 *R = static_cast<float2 *>(ha.R);
        R[(int64_t)k1 * ha.ldr + k2] = make_float2((float)sr, (float)si);
        if (ha.fill_full && k1 != k2) R[(int64_t)k2 * ha.ldr + k1] = make_float2((float)sr, -(float)si);
    }
}

template <int PREC, int WN>
static hipError_t launch_main16_t(const HankelArgs &ha, int n, size_t lds, hipStream_t s)
{
    static const hipError_t attr = hipFuncSetAttribute(reinterpret_cast<const void *>(&hankel_main16<PREC, WN>),
                                                       hipFuncAttributeMaxDynamicSharedMemorySize, 160 * 1024);
    if (attr != hipSuccess) return attr;
    hipLaunchKernelGGL((hankel_main16<PREC, WN>), dim3(n), dim3(kHThreads), lds, s, ha);
    return hipGetLastError();
}

hipError_t launch_hankel_split(const HankelArgs &ha, int prec, hipStream_t s)
{
    const dim3 grid((ha.ldp + 255) / 256, min(ha.N, 65535));
    switch (prec) {
    case kPrecBF16: hipLaunchKernelGGL(hankel_split<kPrecBF16>, grid, dim3(256), 0, s, ha); break;
    case kPrecBF16x3: hipLaunchKernelGGL(hankel_split<kPrecBF16x3>, grid, dim3(256), 0, s, ha); break;
    case kPrecF16: hipLaunchKernelGGL(hankel_split<kPrecF16>, grid, dim3(256), 0, s, ha); break;
    case kPrecF16x3: hipLaunchKernelGGL(hankel_split<kPrecF16x3>, grid, dim3(256), 0, s, ha); break;
    default: return hipErrorInvalidValue;
    }
    return hipGetLastError();
}

hipError_t launch_hankel_main16(const HankelArgs &ha, int prec, int n_items, size_t lds, hipStream_t s)
{
    switch (prec) {
    case kPrecBF16: return launch_main16_t<kPrecBF16, 2>(ha, n_items, lds, s);
    case kPrecBF16x3: return launch_main16_t<kPrecBF16x3, 2>(ha, n_items, lds, s);
    case kPrecF16: return launch_main16_t<kPrecF16, 2>(ha, n_items, lds, s);
    case kPrecF16x3: return launch_main16_t<kPrecF16x3, 1>(ha, n_items, lds, s);
    default: return hipErrorInvalidValue;
    }
}

hipError_t launch_hankel_reduce16(const HankelArgs &ha, int n_tiles, hipStream_t s)
{
    const dim3 grid(n_tiles * kReduceChunks);
    if (ha.tn == 128) hipLaunchKernelGGL(hankel_reduce16<128>, grid, dim3(256), 0, s, ha);
    else hipLaunchKernelGGL(hankel_reduce16<64>, grid, dim3(256), 0, s, ha);
    return hipGetLastError();
}

template <int PREC>
static hipError_t launch_main_t(const HankelArgs &ha, int n, size_t lds, hipStream_t s)
{
    static const hipError_t attr = hipFuncSetAttribute(reinterpret_cast<const void *>(&hankel_main<PREC>),
                                                       hipFuncAttributeMaxDynamicSharedMemorySize, 160 * 1024);
    if (attr != hipSuccess) return attr;
    hipLaunchKernelGGL(hankel_main<PREC>, dim3(n), dim3(kHThreads), lds, s, ha);
    return hipGetLastError();
}

hipError_t launch_hankel_main(const HankelArgs &ha, int prec, int n_items, size_t lds, hipStream_t s)
{
    switch (prec) {
    case kPrecF32: return launch_main_t<kPrecF32>(ha, n_items, lds, s);
    default: return hipErrorInvalidValue;
    }
}

hipError_t launch_hankel_reduce(const HankelArgs &ha, int n_tiles, hipStream_t s)
{
    hipLaunchKernelGGL(hankel_reduce, dim3(n_tiles), dim3(256), 0, s, ha);
    return hipGetLastError();
}

}  // namespace covest
