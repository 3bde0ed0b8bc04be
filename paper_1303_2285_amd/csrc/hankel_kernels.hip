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
// Every form accumulates in FP32 inside the matrix core for kFlushPositions
// positions, then adds into FP64 registers; each work item writes an FP64
// partial tile and hankel_reduce sums the partials in a fixed order.
#include <hip/hip_runtime.h>
#include <hip/hip_bf16.h>
#include <hip/hip_fp16.h>

#include "hankel_internal.hpp"

namespace covest {

typedef float floatx4 __attribute__((ext_vector_type(4)));
typedef float floatx16 __attribute__((ext_vector_type(16)));
typedef __bf16 bf16x8 __attribute__((ext_vector_type(8)));
typedef _Float16 halfx8 __attribute__((ext_vector_type(8)));
typedef unsigned int uintx4 __attribute__((ext_vector_type(4)));

constexpr int kHThreads = 256;

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

// One work item: a 64 x 64 tile of R over window positions with p in [p0, p1).
// Wave w owns the 32 x 32 block (w >> 1, w & 1) of the tile.
template <int PREC>
__global__ void __launch_bounds__(kHThreads, 2) hankel_main(HankelArgs ha)
{
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

    floatx16 acc_re = {}, acc_im = {}, acc_re2 = {}, acc_im2 = {};
    double dre[16], dim[16];
#pragma unroll
    for (int r = 0; r < 16; ++r) dre[r] = dim[r] = 0.0;
    int since_flush = 0;

    auto flush = [&]() {
#pragma unroll
        for (int r = 0; r < 16; ++r) {
            if constexpr (PREC == kPrecF16x3) {
                dre[r] += (double)acc_re[r] + (double)acc_re2[r] * (1.0 / 2048.0);
                dim[r] += (double)acc_im[r] + (double)acc_im2[r] * (1.0 / 2048.0);
            } else {
                dre[r] += (double)acc_re[r];
                dim[r] += (double)acc_im[r];
            }
        }
        acc_re = floatx16{};
        acc_im = floatx16{};
        acc_re2 = floatx16{};
        acc_im2 = floatx16{};
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
                    if constexpr (PREC == kPrecF32) {
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
                    } else {
                        // lane half h: positions q + 4h .. q + 4h + 3, (re, im) pairs
                        const int cc = c + 4 * h;
                        uintx4 ahi = ld4(&LA[0 * plane_a + roff_a + cc]);
                        const uintx4 bhi = ld4(&LB[0 * plane_b + roff_b + cc]);
                        const uintx4 rhi = ld4(&LB[1 * plane_b + roff_b + cc]);
                        uintx4 alo = {}, blo = {}, rlo = {};
                        if constexpr (T::split) {
                            alo = ld4(&LA[2 * plane_a + roff_a + cc]);
                            blo = ld4(&LB[2 * plane_b + roff_b + cc]);
                            rlo = ld4(&LB[3 * plane_b + roff_b + cc]);
                        }
                        if (q + 8 > qe) {
#pragma unroll
                            for (int t = 0; t < 4; ++t)
                                if (q + 4 * h + t >= qe) {
                                    ahi[t] = 0u;
                                    alo[t] = 0u;
                                }
                        }
                        acc_re = mfma16<T::half>(ahi, bhi, acc_re);
                        acc_im = mfma16<T::half>(ahi, rhi, acc_im);
                        if constexpr (T::split) {
                            if constexpr (T::half) {
                                acc_re2 = mfma16<true>(ahi, blo, acc_re2);
                                acc_re2 = mfma16<true>(alo, bhi, acc_re2);
                                acc_im2 = mfma16<true>(ahi, rlo, acc_im2);
                                acc_im2 = mfma16<true>(alo, rhi, acc_im2);
                            } else {
                                acc_re = mfma16<false>(ahi, blo, acc_re);
                                acc_re = mfma16<false>(alo, bhi, acc_re);
                                acc_im = mfma16<false>(ahi, rlo, acc_im);
                                acc_im = mfma16<false>(alo, rhi, acc_im);
                            }
                        }
                        since_flush += 8;
                    }
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

template <int PREC>
static hipError_t launch_main_t(const HankelArgs &ha, int n, size_t lds, hipStream_t s)
{
    static bool attr = false;
    if (!attr) {
        hipError_t e = hipFuncSetAttribute(reinterpret_cast<const void *>(&hankel_main<PREC>),
                                           hipFuncAttributeMaxDynamicSharedMemorySize, 160 * 1024);
        if (e != hipSuccess) return e;
        attr = true;
    }
    hipLaunchKernelGGL(hankel_main<PREC>, dim3(n), dim3(kHThreads), lds, s, ha);
    return hipGetLastError();
}

hipError_t launch_hankel_main(const HankelArgs &ha, int prec, int n_items, size_t lds, hipStream_t s)
{
    switch (prec) {
    case kPrecF32: return launch_main_t<kPrecF32>(ha, n_items, lds, s);
    case kPrecBF16: return launch_main_t<kPrecBF16>(ha, n_items, lds, s);
    case kPrecBF16x3: return launch_main_t<kPrecBF16x3>(ha, n_items, lds, s);
    case kPrecF16: return launch_main_t<kPrecF16>(ha, n_items, lds, s);
    case kPrecF16x3: return launch_main_t<kPrecF16x3>(ha, n_items, lds, s);
    default: return hipErrorInvalidValue;
    }
}

hipError_t launch_hankel_reduce(const HankelArgs &ha, int n_tiles, hipStream_t s)
{
    hipLaunchKernelGGL(hankel_reduce, dim3(n_tiles), dim3(256), 0, s, ha);
    return hipGetLastError();
}

}  // namespace covest
