// rec_mfma.hip -- main pass of the recurrence (kernel family a) on the FP64
// matrix cores of gfx950.
//
// It produces the same three kinds of sums as rec_main (middle block, row
// strips, column strips; see covest_internal.hpp) but forms them as dense
// products.  For a first-factor line x (a row of A in orientation 0, a column
// in orientation 1) and lag (d1, d2) -- d1 across lines, d2 along them -- the
// strip sum over the first-factor positions [lo, hi) is
//
//     T[d1][d2] = sum_c x[c] * conj(B[line + d1][c + d2])
//               = sum_{c'} conj(B[line + d1][c']) * xz[c' - d2],
//
// xz being x with zeros outside [lo, hi).  With the second factor's position
// c' as the reduction index, the first operand (16 lags d1 by 4 positions)
// is a block of A and the second (4 positions by 16 lags d2) a Toeplitz band
// of the line, so one v_mfma_f64_16x16x4 adds 4 positions of 256 lags, and
// every product x[c] * conj(y) is formed once, as in the paper's method
// (Sec. 3.3), not once per output entry.
//
// Complex arithmetic: the four real parts of a complex multiply-add are four
// real products over the same 4 positions,
//     Re T += yr*xr + yi*xi,      Im T += yr*xi + yi*(-xr),
// i.e. four MFMAs per 16 x 16 tile pair per k-group.  Operands come straight
// from A (complex64) and are widened to FP64 in registers; products of two
// floats are exact in FP64, sums accumulate in FP64 inside the matrix core.
//
// MFMA lane layout of v_mfma_f64_16x16x4 (gfx950): lane l supplies A[l%16][l/16]
// and B[l/16][l%16]; result register r of lane l holds D[l/16 + 4r][l%16].
#include <hip/hip_runtime.h>

#include "covest_internal.hpp"
#include "device_util.hpp"

namespace covest {

typedef double v4d __attribute__((ext_vector_type(4)));
// Loads through a global-address-space pointer compile to global_load (not
// flat_load, which also waits on the LDS counter).  The host pass of the
// compiler has no address spaces.
#if defined(__HIP_DEVICE_COMPILE__)
typedef __attribute__((address_space(1))) const float2 gfloat2;
#else
typedef const float2 gfloat2;
#endif

__device__ __forceinline__ v4d mfma64(double a, double b, v4d c)
{
    return __builtin_amdgcn_mfma_f64_16x16x4f64(a, b, c, 0, 0, 0);
}

// Lag (d1, d2) of orientation OR -> (dr, dc); true if it is a unique
// combination (eq. 3.3) of the window.
template <int OR>
__device__ __forceinline__ bool unique_lag(const Inst &in, int d1, int d2, int &dr, int &dc)
{
    dr = OR ? d2 : d1;
    dc = OR ? d1 : d2;
    return dc >= 0 && dc < in.Q && dr > -in.P && dr < in.P && (dc > 0 || dr >= 0);
}

// One workgroup's job.  MT x NT tiles of 16 x 16 lags: rows d1 = d1lo + 16m + i,
// columns d2 = d2lo + 16n + j.
template <int MT, int NT, int OR>
__device__ __forceinline__ void mfma_job(const MJob &job, const Inst &in, double *red)
{
    constexpr int T = MT * NT;
    const int lane = threadIdx.x & 63;
    // the wave index is uniform across the wave: keep it in a scalar register
    // so that branches on it (idle lines, the reduction tree) stay uniform
    const int wave = __builtin_amdgcn_readfirstlane(threadIdx.x >> 6);
    const int i16 = lane & 15, kq = lane >> 4;
    const gfloat2 *A = (const gfloat2 *)in.A;
    // element offsets fit in 32 bits (the planner checks N * lda < 2^31)
    const uint32_t ls = OR ? 1u : (uint32_t)in.lda;   // between lines
    const uint32_t ps = OR ? (uint32_t)in.lda : 1u;   // between positions along a line
    const int nlines = OR ? in.M : in.N;
    const int npos = OR ? in.N : in.M;
    const int d1lo = OR ? 0 : -(in.P - 1);
    const int d2lo = OR ? -(in.P - 1) : 0;

    v4d acc[T][2];
#pragma unroll
    for (int t = 0; t < T; ++t) acc[t][0] = acc[t][1] = (v4d){0.0, 0.0, 0.0, 0.0};

    for (int bl = job.b0; bl <= job.b1; ++bl) {
        const int kga = bl == job.b0 ? job.kg0 : 0;
        const int kgb = bl == job.b1 ? job.kg1 : job.n_kg;
        const int line = job.line0 + bl * kMWaves + wave;
        if (kga >= kgb || line >= job.line_end) continue;

        // Operand lines of this lane.  A line outside A only meets lags whose
        // sums the finalize never reads (or padding lags); its index is
        // clamped so that every load stays inside A.
        uint32_t aoff[MT];
#pragma unroll
        for (int m = 0; m < MT; ++m) {
            const int q = min(max(line + d1lo + 16 * m + i16, 0), nlines - 1);
            aoff[m] = (uint32_t)q * ls;
        }
        const uint32_t xline = (uint32_t)line * ls;
        int xlag[NT];
#pragma unroll
        for (int n = 0; n < NT; ++n) xlag[n] = d2lo + 16 * n + i16;

        // Loads of one k-group: unconditional, from clamped (in-bounds)
        // indices; x values outside the position range are zeroed after.
        float2 an[MT], xn[NT];
        bool xok[NT];
        auto load = [&](int kg) {
            const int pos = job.k0 + 4 * kg + kq;
            const uint32_t pc = (uint32_t)min(pos, npos - 1) * ps;
#pragma unroll
            for (int m = 0; m < MT; ++m) an[m] = A[aoff[m] + pc];
#pragma unroll
            for (int n = 0; n < NT; ++n) {
                const int xp = pos - xlag[n];
                xok[n] = xp >= job.pos_lo && xp < job.pos_hi;
                xn[n] = A[xline + (uint32_t)min(max(xp, 0), npos - 1) * ps];
            }
        };
        load(kga);
        for (int kg = kga; kg < kgb; ++kg) {
            double yr[MT], yi[MT], xr[NT], xi[NT], nxr[NT];
#pragma unroll
            for (int m = 0; m < MT; ++m) {
                yr[m] = (double)an[m].x;
                yi[m] = (double)an[m].y;
            }
#pragma unroll
            for (int n = 0; n < NT; ++n) {
                xr[n] = xok[n] ? (double)xn[n].x : 0.0;
                xi[n] = xok[n] ? (double)xn[n].y : 0.0;
                nxr[n] = -xr[n];
            }
            // next k-group's loads overlap this one's products (the last
            // iteration reloads its own k-group: harmless, branch-free); the
            // scheduling barriers keep the compiler from moving the loads
            // back behind the conversions above
            __builtin_amdgcn_sched_barrier(0);
            load(min(kg + 1, kgb - 1));
            __builtin_amdgcn_sched_barrier(0);
#pragma unroll
            for (int m = 0; m < MT; ++m)
#pragma unroll
                for (int n = 0; n < NT; ++n) {
                    acc[m * NT + n][0] = mfma64(yr[m], xr[n], acc[m * NT + n][0]);
                    acc[m * NT + n][1] = mfma64(yr[m], xi[n], acc[m * NT + n][1]);
                }
#pragma unroll
            for (int m = 0; m < MT; ++m)
#pragma unroll
                for (int n = 0; n < NT; ++n) {
                    acc[m * NT + n][0] = mfma64(yi[m], xi[n], acc[m * NT + n][0]);
                    acc[m * NT + n][1] = mfma64(yi[m], nxr[n], acc[m * NT + n][1]);
                }
        }
    }

    // Write this lane's sums of unique lags into one row of lag_stride
    // complex values; val(t, c, r) is register r of part c of tile t.
    auto write_row = [&](double2 *row, auto val) {
#pragma unroll
        for (int m = 0; m < MT; ++m)
#pragma unroll
            for (int n = 0; n < NT; ++n)
#pragma unroll
                for (int r = 0; r < 4; ++r) {
                    int dr, dc;
                    if (unique_lag<OR>(in, d1lo + 16 * m + kq + 4 * r, d2lo + 16 * n + i16, dr, dc))
                        row[(dr + in.P - 1) * in.Q + dc] = make_double2(val(m * NT + n, 0, r), val(m * NT + n, 1, r));
                }
    };

    if (job.kind == kMStrip) {
        const int line = job.line0 + wave;
        if (line < job.line_end) {
            double *z = OR ? in.zc : in.zr;
            write_row(reinterpret_cast<double2 *>(z + (int64_t)(job.out + wave) * in.lag_stride * 2),
                      [&](int t, int c, int r) { return acc[t][c][r]; });
        }
        return;
    }

    // Bulk: the waves' sums are added in a fixed order through LDS -- slot s
    // (s < 4) gets wave s+4 plus wave s, slot s (s < 2) then adds slot s+2,
    // and slot 0 adds slot 1 -- and wave 0 writes one partial row.  The
    // registers are only read here, never updated.
    constexpr int V = T * 8;   // doubles per lane
    auto at = [&](int slot, int t, int c, int r) -> double & {
        return red[((slot * V) + (t * 2 + c) * 4 + r) * 64 + lane];
    };
    if (wave >= 4) {
#pragma unroll
        for (int t = 0; t < T; ++t)
#pragma unroll
            for (int c = 0; c < 2; ++c)
#pragma unroll
                for (int r = 0; r < 4; ++r) at(wave - 4, t, c, r) = acc[t][c][r];
    }
    __syncthreads();
    if (wave < 4) {
#pragma unroll
        for (int t = 0; t < T; ++t)
#pragma unroll
            for (int c = 0; c < 2; ++c)
#pragma unroll
                for (int r = 0; r < 4; ++r) at(wave, t, c, r) = at(wave, t, c, r) + acc[t][c][r];
    }
    __syncthreads();
    if (wave < 2) {
#pragma unroll
        for (int t = 0; t < T; ++t)
#pragma unroll
            for (int c = 0; c < 2; ++c)
#pragma unroll
                for (int r = 0; r < 4; ++r) at(wave, t, c, r) = at(wave, t, c, r) + at(wave + 2, t, c, r);
    }
    __syncthreads();
    if (wave == 0)
        write_row(reinterpret_cast<double2 *>(in.partial + (int64_t)job.out * in.lag_stride * 2),
                  [&](int t, int c, int r) { return at(0, t, c, r) + at(1, t, c, r); });
}

// One workgroup per job; orientation-1 jobs use the transposed tile shape
// (their d1 runs over Q column lags, d2 over 2P-1 row lags).
template <int MT, int NT>
__global__ void __launch_bounds__(kMThreads, 2) rec_mfma(MfmaArgs ma)
{
    extern __shared__ double red[];
    int b = blockIdx.x;
    if (ma.xcd_remap) b = xcd_block(b, ma.n_jobs);
    const MJob job = ma.jobs[b];
    const Inst in = ma.use_inline ? ma.inst_inline : ma.insts[job.inst];
    if (job.orient == 0) mfma_job<MT, NT, 0>(job, in, red);
    else mfma_job<NT, MT, 1>(job, in, red);
}

template <int MT, int NT>
static hipError_t launch_mt_nt(const MfmaArgs &ma, int n_blocks, size_t lds, hipStream_t stream)
{
    static hipError_t attr = hipFuncSetAttribute(reinterpret_cast<const void *>(&rec_mfma<MT, NT>),
                                                 hipFuncAttributeMaxDynamicSharedMemorySize, 150 * 1024);
    if (attr != hipSuccess) return attr;
    hipLaunchKernelGGL((rec_mfma<MT, NT>), dim3(n_blocks), dim3(kMThreads), lds, stream, ma);
    return hipGetLastError();
}

hipError_t launch_rec_mfma(const MfmaArgs &ma, int mt, int nt, int n_blocks, size_t lds, hipStream_t stream)
{
#define COVEST_MT_NT(a, b) \
    if (mt == a && nt == b) return launch_mt_nt<a, b>(ma, n_blocks, lds, stream);
    COVEST_MT_NT(1, 1) COVEST_MT_NT(1, 2) COVEST_MT_NT(1, 3) COVEST_MT_NT(1, 4)
    COVEST_MT_NT(2, 1) COVEST_MT_NT(2, 2) COVEST_MT_NT(2, 3) COVEST_MT_NT(2, 4)
    COVEST_MT_NT(3, 1) COVEST_MT_NT(3, 2) COVEST_MT_NT(4, 1) COVEST_MT_NT(4, 2)
    COVEST_MT_NT(5, 1) COVEST_MT_NT(6, 1) COVEST_MT_NT(7, 1) COVEST_MT_NT(8, 1)
#undef COVEST_MT_NT
    return hipErrorInvalidValue;
}

}  // namespace covest
