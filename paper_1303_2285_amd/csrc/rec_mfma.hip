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
// Complex arithmetic: conj(y) * x over 4 positions takes three real products
// (the three-multiplication form of a complex product):
//     K1 += (yr - yi) * xr,   K2 += yr * (xi - xr),   K3 += (-yi) * (xr + xi),
//     Re T = K1 - K3 = sum yr*xr + yi*xi,   Im T = K1 + K2 = sum yr*xi - yi*xr,
// i.e. three MFMAs per 16 x 16 tile per k-group, into three accumulators that
// are combined once per job.  Lag blocks of more than 4 tile rows keep the
// four-product form (Re += yr*xr + yi*xi, Im += yr*xi + yi*(-xr)) in two
// accumulators, which their registers allow; blocks of up to 4 rows (at
// most 8 tiles) hold three accumulators per tile for all their tiles at once
// (the 4 x 2 and 2 x 4 blocks spill a few values, outside the k-group loop).
// Operands come straight from A (complex64) and are widened to FP64 in
// registers; a product of two floats, and of a float and a sum or difference
// of two floats, is exact in FP64 (the sum is, for parts within 2^28 of each
// other), and sums accumulate in FP64 inside the matrix core.
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

// Widen 4 positions of the operands and return the MFMAs that add them
// (issued by the caller after the next loads).  Four-product form: two
// accumulators per tile (Re, Im).
template <int MT, int NT>
__device__ __forceinline__ auto kgroup_products4(const float2 (&an)[MT], const float2 (&xn)[NT])
{
    double yr[MT], yi[MT], xr[NT], xi[NT], nxr[NT];
#pragma unroll
    for (int m = 0; m < MT; ++m) {
        yr[m] = (double)an[m].x;
        yi[m] = (double)an[m].y;
    }
#pragma unroll
    for (int n = 0; n < NT; ++n) {
        xr[n] = (double)xn[n].x;
        xi[n] = (double)xn[n].y;
        nxr[n] = (double)(-xn[n].x);
    }
    return [=](v4d (&acc)[MT * NT][2]) {
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
    };
}

// Three-product form: three accumulators per tile (K1, K2, K3).
template <int MT, int NT>
__device__ __forceinline__ auto kgroup_products3(const float2 (&an)[MT], const float2 (&xn)[NT])
{
    double sy[MT], yr[MT], nyi[MT], xr[NT], dmc[NT], cpd[NT];
#pragma unroll
    for (int m = 0; m < MT; ++m) {
        yr[m] = (double)an[m].x;
        nyi[m] = (double)(-an[m].y);
        sy[m] = yr[m] + nyi[m];
    }
#pragma unroll
    for (int n = 0; n < NT; ++n) {
        xr[n] = (double)xn[n].x;
        const double xi = (double)xn[n].y;
        dmc[n] = xi - xr[n];
        cpd[n] = xr[n] + xi;
    }
    return [=](v4d (&acc)[MT * NT][3]) {
#pragma unroll
        for (int m = 0; m < MT; ++m)
#pragma unroll
            for (int n = 0; n < NT; ++n) {
                acc[m * NT + n][0] = mfma64(sy[m], xr[n], acc[m * NT + n][0]);
                acc[m * NT + n][1] = mfma64(yr[m], dmc[n], acc[m * NT + n][1]);
                acc[m * NT + n][2] = mfma64(nyi[m], cpd[n], acc[m * NT + n][2]);
            }
    };
}

template <int MT, int NT, int C>
__device__ __forceinline__ auto kgroup_products(const float2 (&an)[MT], const float2 (&xn)[NT])
{
    if constexpr (C == 3)
        return kgroup_products3<MT, NT>(an, xn);
    else
        return kgroup_products4<MT, NT>(an, xn);
}

// Run k-groups [k_a, k_b): the loads of k-group kg + D are issued before
// kg's products, so they overlap (the last iterations reload the last
// k-group: harmless); the scheduling barriers keep the compiler from moving
// the loads back behind the conversions.  A k-group of MT * NT tiles takes
// 3 or 4 MT NT MFMAs, so small lag blocks keep more k-groups in flight (D) to
// cover the load latency.
template <int MT, int NT, int C, class Load>
__device__ __forceinline__ void run_kgroups(int k_a, int k_b, v4d (&acc)[MT * NT][C], Load load)
{
    // an empty range loads nothing (its first load would be k-group k_a - 1)
    if (k_a >= k_b) return;
    constexpr int D = MT * NT >= 8 ? 1 : MT * NT >= 4 ? 2 : 4;
    float2 an[D][MT], xn[D][NT];
#pragma unroll
    for (int d = 0; d < D; ++d) load(min(k_a + d, k_b - 1), an[d], xn[d]);
    for (int kg = k_a; kg < k_b; kg += D) {
#pragma unroll
        for (int d = 0; d < D; ++d) {
            if (D == 1 || kg + d < k_b) {
                auto mf = kgroup_products<MT, NT, C>(an[d], xn[d]);
                __builtin_amdgcn_sched_barrier(0);
                load(min(kg + d + D, k_b - 1), an[d], xn[d]);
                __builtin_amdgcn_sched_barrier(0);
                mf(acc);
            }
        }
    }
}

// One workgroup's job.  MT x NT tiles of 16 x 16 lags: rows d1 = d1lo + 16m + i,
// columns d2 = d2lo + 16n + j.
//
// The first operand (16 lines by 4 positions per tile) is read with plain
// loads: a wave-uniform base plus loop-invariant lane offsets, no vector
// arithmetic.  They stay inside A because orientation 0 ends every line's
// k-groups at the row's last column (the planner's k0), and orientation 1
// clamps its positions in the one k-group that can pass row N-1.  The
// line's own values (the second operand), zeroed outside [pos_lo, pos_hi),
// are staged per wave in LDS, kMXCap of them at a time, and read from there.
// The planner sets job.kin, the k-groups that need no clamp: 0 for a line of
// fewer than 4 positions past k0.
template <int MT, int NT, int OR, int C>
__device__ __forceinline__ void mfma_pass(const MJob &job, const Inst &in, double *red)
{
    constexpr int T = MT * NT;
    constexpr int span = 16 * NT - 1;      // lane lags d2 in [d2lo, d2lo + span]
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
    // k-groups whose 4 positions all lie inside A (the planner counts them)
    const int kin = job.kin;

    v4d acc[T][C];
#pragma unroll
    for (int t = 0; t < T; ++t)
#pragma unroll
        for (int c = 0; c < C; ++c) acc[t][c] = (v4d){0.0, 0.0, 0.0, 0.0};
    float2 *xb = reinterpret_cast<float2 *>(red) + wave * kMXCap;
    const int chunk = (kMXCap - span) / 4;   // k-groups per staged chunk

    for (int bl = job.b0; bl <= job.b1; ++bl) {
        const int kga = bl == job.b0 ? job.kg0 : 0;
        const int kgb = bl == job.b1 ? job.kg1 : job.n_kg;
        const int line = job.line0 + bl * kMWaves + wave;
        if (kga >= kgb || line >= job.line_end) continue;

        // Operand lines of this lane.  A line outside A only meets lags whose
        // sums the finalize never reads (or padding lags); its index is
        // clamped so that every load stays inside A.
        int q[MT];
        uint32_t aoff[MT];
#pragma unroll
        for (int m = 0; m < MT; ++m) {
            q[m] = min(max(line + d1lo + 16 * m + i16, 0), nlines - 1);
            aoff[m] = (uint32_t)q[m] * ls + (uint32_t)kq * ps;
        }
        const uint32_t xline = (uint32_t)line * ls;

        for (int kc = kga; kc < kgb; kc += chunk) {
            const int kce = min(kgb, kc + chunk);
            const int xbase = job.k0 + 4 * kc - (d2lo + span);   // position of xb[0]
            const int len = 4 * (kce - kc) + span;
            // The previous chunk's reads were issued before these writes, and a
            // wave's LDS operations run in order.  The loads go out 8 at a time
            // before any is stored, so their latencies overlap.
            for (int i0 = lane; i0 < len; i0 += 8 * 64) {
                float2 v[8];
#pragma unroll
                for (int u = 0; u < 8; ++u) {
                    const int p = xbase + i0 + 64 * u;
                    const bool ok = p >= job.pos_lo && p < job.pos_hi;
                    v[u] = A[xline + (uint32_t)(ok ? p : job.pos_lo) * ps];
                    if (!ok) v[u] = make_float2(0.f, 0.f);
                }
#pragma unroll
                for (int u = 0; u < 8; ++u)
                    if (i0 + 64 * u < len) xb[i0 + 64 * u] = v[u];
            }
            __builtin_amdgcn_fence(__ATOMIC_RELEASE, "wavefront");
            __builtin_amdgcn_wave_barrier();
            __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "wavefront");
            // lane (kq, j) of tile n reads position k0 + 4 kg + kq - (d2lo + 16 n + j)
            const float2 *xl = xb + (kq - i16 + span);
            auto load = [&](int kg, const uint32_t(&off)[MT], float2(&an)[MT], float2(&xn)[NT]) {
                const gfloat2 *Ak = A + (uint32_t)(job.k0 + 4 * kg) * ps;
#pragma unroll
                for (int m = 0; m < MT; ++m) an[m] = Ak[off[m]];
#pragma unroll
                for (int n = 0; n < NT; ++n) xn[n] = xl[4 * (kg - kc) - 16 * n];
            };
            const int kplain = min(kce, kin);
            run_kgroups<MT, NT, C>(kc, kplain, acc,
                                [&](int kg, float2(&an)[MT], float2(&xn)[NT]) { load(kg, aoff, an, xn); });
            if (kplain < kce) {
                // the last k-group of a line can pass A's last position: clamp
                // it (at most one k-group, the planner's kin is n_kg - 1 or
                // n_kg; orientation 0 never gets here)
                const int pos = job.k0 + 4 * kplain + kq;
                uint32_t off[MT];
#pragma unroll
                for (int m = 0; m < MT; ++m)
                    off[m] = (uint32_t)q[m] * ls + (uint32_t)(min(pos, npos - 1) - (job.k0 + 4 * kplain)) * ps;
                run_kgroups<MT, NT, C>(kplain, kce, acc,
                                    [&](int kg, float2(&an)[MT], float2(&xn)[NT]) { load(kg, off, an, xn); });
            }
        }
    }

    // Re and Im of every tile
    v4d res[T][2];
#pragma unroll
    for (int t = 0; t < T; ++t) {
        if constexpr (C == 3) {
            res[t][0] = acc[t][0] - acc[t][2];
            res[t][1] = acc[t][0] + acc[t][1];
        } else {
            res[t][0] = acc[t][0];
            res[t][1] = acc[t][1];
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
                      [&](int t, int c, int r) { return res[t][c][r]; });
        }
        return;
    }

    // Bulk: the waves' sums are added in a fixed order through LDS -- slot s
    // (s < 4) gets wave s+4 plus wave s, slot s (s < 2) then adds slot s+2,
    // and slot 0 adds slot 1 -- and wave 0 writes one partial row.  The
    // registers are only read here, never updated.
    constexpr int V = T * 8;   // doubles per lane
    __syncthreads();   // the LDS held the staged lines until now
    auto at = [&](int slot, int t, int c, int r) -> double & {
        return red[((slot * V) + (t * 2 + c) * 4 + r) * 64 + lane];
    };
    if (wave >= 4) {
#pragma unroll
        for (int t = 0; t < T; ++t)
#pragma unroll
            for (int c = 0; c < 2; ++c)
#pragma unroll
                for (int r = 0; r < 4; ++r) at(wave - 4, t, c, r) = res[t][c][r];
    }
    __syncthreads();
    if (wave < 4) {
#pragma unroll
        for (int t = 0; t < T; ++t)
#pragma unroll
            for (int c = 0; c < 2; ++c)
#pragma unroll
                for (int r = 0; r < 4; ++r) at(wave, t, c, r) = at(wave, t, c, r) + res[t][c][r];
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

// A job: lag blocks of at most 4 tile rows take the three-product form,
// larger ones the four-product form; every tile of the block in one walk
// over the job's lines.
template <int MT, int NT, int OR>
__device__ __forceinline__ void mfma_job(const MJob &job, const Inst &in, double *red)
{
    mfma_pass<MT, NT, OR, (MT <= 4 ? 3 : 2)>(job, in, red);
}

// One workgroup per job; orientation-1 jobs use the transposed tile shape
// (their d1 runs over Q column lags, d2 over 2P-1 row lags).  BATCH: the
// job's problem comes from the instance table (jobs of many problems, longest
// first, in one launch).
template <int MT, int NT, bool BATCH>
__global__ void __launch_bounds__(kMThreads, 2) rec_mfma(MfmaArgs ma)
{
    extern __shared__ double red[];
    int b = blockIdx.x;
    if (ma.xcd_remap) b = xcd_block(b, ma.n_jobs);
    const MJob job = ma.jobs[b];
    if constexpr (BATCH) {
        const Inst in = ma.insts[job.inst];
        if (job.orient == 0) mfma_job<MT, NT, 0>(job, in, red);
        else mfma_job<NT, MT, 1>(job, in, red);
    } else {
        const Inst &in = ma.inst;
        if (job.orient == 0) mfma_job<MT, NT, 0>(job, in, red);
        else mfma_job<NT, MT, 1>(job, in, red);
    }
}

template <int MT, int NT, bool BATCH>
static hipError_t launch_mt_nt_b(const MfmaArgs &ma, int n_blocks, size_t lds, hipStream_t stream)
{
    static hipError_t attr = hipFuncSetAttribute(reinterpret_cast<const void *>(&rec_mfma<MT, NT, BATCH>),
                                                 hipFuncAttributeMaxDynamicSharedMemorySize, 150 * 1024);
    if (attr != hipSuccess) return attr;
    hipLaunchKernelGGL((rec_mfma<MT, NT, BATCH>), dim3(n_blocks), dim3(kMThreads), lds, stream, ma);
    return hipGetLastError();
}

template <int MT, int NT>
static hipError_t launch_mt_nt(const MfmaArgs &ma, int n_blocks, size_t lds, hipStream_t stream)
{
    if (ma.insts) return launch_mt_nt_b<MT, NT, true>(ma, n_blocks, lds, stream);
    return launch_mt_nt_b<MT, NT, false>(ma, n_blocks, lds, stream);
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
