// lane_kernels.hip -- the lane engine: one lane per unique combination
// (Sec. 3.1), for grids of small inputs such as the apertures of an image.
//
// The paper's combination-parallel method gives each core one combination
// (dr, dc) at a time and computes that combination's entries, which lie on
// segments of one diagonal of R (Sec. 3.3, eq. 3.8).  Here each lane of a
// workgroup holds one combination of one input for the whole input, so that
// no partial sums leave the lane:
//
//   entry (i1, j1) of combination (dr, dc) is the sum of the product grid
//   Z[x][y] = A[x][y] * conj(A[x+dr][y+dc]) over the box of first-factor
//   positions [i1, i1 + Kr) x [j1, j1 + Kc).
//
// The lane walks the input row by row.  For every row it forms the window
// sums of the row over the Q column offsets j1 -- the first window directly,
// each next one from the last by adding the column that enters and taking
// away the column that leaves (the shift rule of Sec. 3.3 along a row) --
// and adds them to B[j1], the box sums of the current box start i1.  After
// the first Kr rows B holds the entries of i1 = 0; each further row step
// moves the box down by one row, adding the window sums of the entering row
// and taking away those of the leaving row (the shift rule along a column).
// The entries are divided by K and written as they complete: no finalize
// pass, no workspace.
//
// Inputs of one grid column that overlap (apertures at a row step below the
// box height) can share one walk: after the entries of input a the box keeps
// sliding down the image to the first box of input a+1 (a "chain"), which
// costs two rows per step instead of a new first box of Kr rows.  The host
// chains inputs when that is cheaper and the grid still fills the device.
//
// Operands: the first factor A[x][y] is the same for every lane (every lane
// walks the same positions) and is read from LDS as a broadcast, converted to
// FP64 when staged; the second factors of a lane, A[x+dr][y+dc], are read from
// rings of staged complex64 rows with Q-1 zero columns on each side (and zero
// rows below the chain), converted when used.  Every product is an exact FP64
// product of two floats and every sum an FP64 sum; on small-integer inputs
// the entries are exact.
#include "lane_internal.hpp"

#include <type_traits>

#include "device_util.hpp"

namespace covest {

namespace {

__device__ __forceinline__ double2 to_d(const float2 v) { return make_double2((double)v.x, (double)v.y); }
__device__ __forceinline__ double2 to_d(const double2 v) { return v; }

// Element types of the staged first-factor rows and second-factor rings
// (sizes kLaneFBytes, kLaneGBytes).
typedef double2 fstage_t;
typedef float2 gstage_t;
static_assert(sizeof(fstage_t) == kLaneFBytes && sizeof(gstage_t) == kLaneGBytes, "LDS element sizes");
__device__ __forceinline__ void put(double2 &d, const float2 v) { d = to_d(v); }
__device__ __forceinline__ void put(float2 &d, const float2 v) { d = v; }

// acc += x * conj(y)
__device__ __forceinline__ void lmac(double2 &acc, const double2 x, const double2 y)
{
    acc.x = fma(x.x, y.x, acc.x);
    acc.x = fma(x.y, y.y, acc.x);
    acc.y = fma(x.y, y.x, acc.y);
    acc.y = fma(-x.x, y.y, acc.y);
}

// acc -= x * conj(y)
__device__ __forceinline__ void lmsub(double2 &acc, const double2 x, const double2 y)
{
    acc.x = fma(-x.x, y.x, acc.x);
    acc.x = fma(-x.y, y.y, acc.x);
    acc.y = fma(-x.y, y.x, acc.y);
    acc.y = fma(x.x, y.y, acc.y);
}

__device__ __forceinline__ double2 dadd(const double2 a, const double2 b) { return make_double2(a.x + b.x, a.y + b.y); }

// One block of the row walk: 4 products -- 4 columns of the entering row, or
// (SLIDE) 2 columns of the entering row and the same 2 of the leaving row.
// The first factors are LDS broadcasts (every lane reads the same address).
template <bool SLIDE>
__device__ __forceinline__ void blk_load(fstage_t (&f)[4], gstage_t (&g)[4], const fstage_t *fi, const gstage_t *gi,
                                         const fstage_t *fo, const gstage_t *go, int y)
{
#pragma unroll
    for (int j = 0; j < 4; ++j) {
        if (!SLIDE) {
            f[j] = fi[y + j];
            g[j] = gi[y + j];
        } else if (j < 2) {
            f[j] = fi[y + j];
            g[j] = gi[y + j];
        } else {
            f[j] = fo[y + j - 2];
            g[j] = go[y + j - 2];
        }
    }
}

template <bool SLIDE>
__device__ __forceinline__ void blk_prod(double2 (&s)[4], const fstage_t (&f)[4], const gstage_t (&g)[4], int j0,
                                         int j1)
{
#pragma unroll
    for (int j = 0; j < 4; ++j) {
        if (j < j0 || j >= j1) continue;
        if (!SLIDE || j < 2)
            lmac(s[j], to_d(f[j]), to_d(g[j]));
        else
            lmsub(s[j], to_d(f[j]), to_d(g[j]));
    }
}

// One row step: the window sums over the Q column offsets of the entering row
// minus, when SLIDE, those of the leaving row, added to B.  fi/fo: first
// factors of the entering / leaving row (FP64 in LDS); gi/go: this lane's
// second factors, offset by dc (column y at gi[y]).
//
// The first window (Kc columns) runs in blocks of 4 products, loaded one
// block ahead: the first product of a block waits for its loads, then the
// next block's loads go out, then the other three products run while they
// arrive.  Two register sets alternate so that nothing is copied.
template <int QMAX, bool SLIDE>
__device__ __forceinline__ void row_step(double2 (&B)[QMAX], const fstage_t *fi, const gstage_t *gi, const fstage_t *fo,
                                         const gstage_t *go, int Kc, int Q)
{
    double2 s[4];
#pragma unroll
    for (int j = 0; j < 4; ++j) s[j] = make_double2(0.0, 0.0);
    constexpr int step = SLIDE ? 2 : 4;   // columns per block
    const int nb = Kc / step;
    if (nb > 0) {
        fstage_t fA[4], fB[4];
        gstage_t gA[4], gB[4];
        blk_load<SLIDE>(fA, gA, fi, gi, fo, go, 0);
        int k = 0;
        for (; k + 2 <= nb; k += 2) {
            blk_prod<SLIDE>(s, fA, gA, 0, 1);
            __builtin_amdgcn_sched_barrier(0);
            blk_load<SLIDE>(fB, gB, fi, gi, fo, go, (k + 1) * step);
            __builtin_amdgcn_sched_barrier(0);
            blk_prod<SLIDE>(s, fA, gA, 1, 4);
            blk_prod<SLIDE>(s, fB, gB, 0, 1);
            __builtin_amdgcn_sched_barrier(0);
            // (the last pass reloads the last block: no branch, so that the
            // two register sets stay two sets without copies)
            blk_load<SLIDE>(fA, gA, fi, gi, fo, go, min(k + 2, nb - 1) * step);
            __builtin_amdgcn_sched_barrier(0);
            blk_prod<SLIDE>(s, fB, gB, 1, 4);
        }
        if (k < nb) blk_prod<SLIDE>(s, fA, gA, 0, 4);
    }
    for (int y = nb * step; y < Kc; ++y) {
        lmac(s[0], to_d(fi[y]), to_d(gi[y]));
        if (SLIDE) lmsub(s[1], to_d(fo[y]), to_d(go[y]));
    }
    double2 S = dadd(dadd(s[0], s[1]), dadd(s[2], s[3]));
    B[0] = dadd(B[0], S);
#pragma unroll
    for (int e = 1; e < QMAX; ++e) {
        if (e < Q) {
            const int yi = Kc - 1 + e, yo = e - 1;   // column entering and column leaving the window
            lmac(S, to_d(fi[yi]), to_d(gi[yi]));
            lmsub(S, to_d(fi[yo]), to_d(gi[yo]));
            if (SLIDE) {
                lmsub(S, to_d(fo[yi]), to_d(go[yi]));
                lmac(S, to_d(fo[yo]), to_d(go[yo]));
            }
            B[e] = dadd(B[e], S);
        }
        // keep the loads of each offset next to their use (the whole unrolled
        // run's loads at once would take more registers than three waves per
        // SIMD leave)
        __builtin_amdgcn_sched_barrier(0);
    }
}

// One entry of R: the value (divided by K when asked) at offset `up` (the
// upper-triangle position of the entry or of its conjugate, `conj_up` telling
// which), and the exact mirror at `mir` when the whole R is asked for.
__device__ __forceinline__ void lane_store(const LaneArgs &la, void *Rq, int64_t up, int64_t mir, double2 v,
                                           bool conj_up, bool diag)
{
    if (la.normalize) {
        const double K = (double)la.Kr * (double)la.Kc;
        v.x = v.x / K;
        v.y = v.y / K;
    }
    if (diag) v.y = 0.0;
    if (conj_up) v.y = -v.y;
    if (la.out_fp64) {
        double2 *R = static_cast<double2 *>(Rq);
        R[up] = v;
        if (la.fill_full && !diag) R[mir] = make_double2(v.x, -v.y);
    } else {
        float2 *R = static_cast<float2 *>(Rq);
        const float2 f = make_float2((float)v.x, (float)v.y);
        R[up] = f;
        if (la.fill_full && !diag) R[mir] = make_float2(f.x, -f.y);
    }
}

template <int QMAX>
__global__ void __launch_bounds__(kLaneMaxLags) __attribute__((amdgpu_waves_per_eu(3))) lane_main(LaneArgs la)
{
    extern __shared__ __align__(16) unsigned char lane_lds[];
    const int P = la.P, Q = la.Q, N = la.N, M = la.M, Kr = la.Kr, Kc = la.Kc;
    const int ring = la.ring, gstride = la.gstride, rs = la.row_step;
    const int T = blockDim.x, lt = threadIdx.x;
    gstage_t *Gi = reinterpret_cast<gstage_t *>(lane_lds);
    gstage_t *Go = Gi + (size_t)ring * gstride;
    fstage_t *Fi = reinterpret_cast<fstage_t *>(Go + (size_t)ring * gstride);
    fstage_t *Fo = Fi + (size_t)kLaneChunk * M;

    // workgroup -> (chain, grid column)
    const int wg = xcd_block(blockIdx.x, gridDim.x);
    const int b = wg % la.n_cols, a0 = (wg / la.n_cols) * la.chain;
    const int L = min(la.chain, la.n_rows - a0);
    const float2 *img = la.image + (int64_t)a0 * rs * la.ld + (int64_t)b * la.col_step;
    const int rows_walk = (L - 1) * rs + N;   // image rows of the chain; rows below read as zero
    const int s_end = rows_walk - 1;          // row step s brings row s into the box

    // this lane's combination: dr = 0 with dc in [0, Q), then dr >= 1 with dc in (-Q, Q)
    const bool live = lt < la.n_lags;
    int dr = 0, dc = live ? lt : 0;
    if (live && lt >= Q) {
        const int u = lt - Q;
        dr = 1 + u / (2 * Q - 1);
        dc = u % (2 * Q - 1) - (Q - 1);
    }
    const int nr = P - dr;                                  // box starts i1 in [0, nr)
    const int j1lo = max(0, -dc), j1hi = Q - max(0, dc);   // column offsets j1 in [j1lo, j1hi)
    const bool diag = dr == 0 && dc == 0;

    // staging, every thread a share
    auto stage_f = [&](fstage_t *dst, int r_first, int n_rows_) {
        for (int e = lt; e < n_rows_ * M; e += T) {
            const int rr = e / M, y = e - rr * M;
            put(dst[e], img[(int64_t)(r_first + rr) * la.ld + y]);
        }
    };
    const int gc = M + 2 * Q - 2;
    auto stage_g = [&](gstage_t *buf, int r_lo, int r_hi) {
        for (int e = lt; e < (r_hi - r_lo) * gc; e += T) {
            const int rr = e / gc, cc = e - rr * gc;
            const int r = r_lo + rr, y = cc - (Q - 1);
            float2 v = make_float2(0.f, 0.f);
            if (r < rows_walk && y >= 0 && y < M) v = img[(int64_t)r * la.ld + y];
            put(buf[(r % ring) * gstride + cc], v);
        }
    };

    double2 B[QMAX];
#pragma unroll
    for (int e = 0; e < QMAX; ++e) B[e] = make_double2(0.0, 0.0);

    // Entry (i1, j1) of this lane's combination is R[k1][k2] with k1 = i1 + P*j1,
    // k2 = k1 + dr + P*dc: below the diagonal when dr + P*dc < 0, so the
    // upper triangle gets its conjugate at (k2, k1).  Along j1 both offsets
    // move by P*(ldr + 1).
    const int kd = dr + P * dc;
    const bool below = kd < 0;
    const int64_t ostep = (int64_t)P * (la.ldr + 1);
    const size_t esz = la.out_fp64 ? 16 : 8;

    // B holds box start t (chain rows): entry row i1 = t - q*rs of every
    // input q of the chain with 0 <= i1 < P
    auto emit = [&](int t) {
        const int q_lo = t >= P ? (t - P + rs) / rs : 0;
        const int q_hi = min(L - 1, t / rs);
        for (int q = q_lo; q <= q_hi; ++q) {
            const int i1 = t - q * rs;
            if (!live || i1 >= nr) continue;
            void *Rq = static_cast<char *>(la.R) + ((int64_t)(a0 + q) * la.n_cols + b) * la.r_stride * esz;
            const int64_t k1 = i1, k2 = i1 + kd;   // at j1 = 0
            int64_t up = below ? k2 * la.ldr + k1 : k1 * la.ldr + k2;
            int64_t mir = below ? k1 * la.ldr + k2 : k2 * la.ldr + k1;
#pragma unroll
            for (int e = 0; e < QMAX; ++e) {
                // one entry at a time: the empty asm orders this entry's
                // division after the previous entry's store, so the divisions
                // of all offsets are never live at once
                double2 v = B[e];
                asm volatile("" : "+v"(v.x), "+v"(v.y) : : "memory");
                if (e >= j1lo && e < j1hi) lane_store(la, Rq, up, mir, v, below, diag);
                up += ostep;
                mir += ostep;
            }
        }
    };

    int gi_next = 0, go_next = 0;   // next chain row to stage into each ring
    // Steps [from, to) in chunks.  SLIDE steps (s >= Kr) also take away the
    // row leaving the box and emit.  The two kinds are separate loops so that
    // B passes through one row-step body in each.
    auto phase = [&](auto slide_c, int from, int to) {
        constexpr bool SLIDE = decltype(slide_c)::value;
        for (int s0 = from; s0 < to; s0 += kLaneChunk) {
            const int s1 = min(to, s0 + kLaneChunk);
            {
                // rows entering the box at steps [s0, s1): first factors, and
                // the second factors of every lag (P - 1 rows further down)
                stage_f(Fi, s0, s1 - s0);
                stage_g(Gi, gi_next, s1 + P - 1);
                gi_next = s1 + P - 1;
                if (SLIDE) {   // rows leaving the box: Kr rows above
                    stage_f(Fo, s0 - Kr, s1 - s0);
                    stage_g(Go, max(go_next, s0 - Kr), s1 - Kr + P - 1);
                    go_next = s1 - Kr + P - 1;
                }
            }
            __syncthreads();
            {
                for (int s = s0; s < s1; ++s) {
                    int gs = s % ring + dr;
                    if (gs >= ring) gs -= ring;
                    const gstage_t *gi = Gi + gs * gstride + (dc + Q - 1);
                    const fstage_t *fi = Fi + (size_t)(s - s0) * M;
                    if (SLIDE) {
                        int go_s = (s - Kr) % ring + dr;
                        if (go_s >= ring) go_s -= ring;
                        row_step<QMAX, true>(B, fi, gi, Fo + (size_t)(s - s0) * M,
                                             Go + go_s * gstride + (dc + Q - 1), Kc, Q);
                        emit(s - (Kr - 1));
                    } else {
                        row_step<QMAX, false>(B, fi, gi, nullptr, nullptr, Kc, Q);
                    }
                }
            }
            __syncthreads();
        }
    };

    phase(std::integral_constant<bool, false>{}, 0, Kr);
    emit(0);
    phase(std::integral_constant<bool, true>{}, Kr, s_end + 1);
}

}  // namespace

hipError_t prepare_lane_kernels()
{
    static hipError_t status = [] {
        const void *fns[] = {reinterpret_cast<const void *>(&lane_main<8>),
                             reinterpret_cast<const void *>(&lane_main<12>),
                             reinterpret_cast<const void *>(&lane_main<16>)};
        for (const void *f : fns) {
            hipError_t e = hipFuncSetAttribute(f, hipFuncAttributeMaxDynamicSharedMemorySize, (int)kLaneMaxLds);
            if (e != hipSuccess) return e;
        }
        return hipSuccess;
    }();
    return status;
}

hipError_t launch_lane(const LaneArgs &la, int n_blocks, size_t lds, hipStream_t stream)
{
    hipError_t e = prepare_lane_kernels();
    if (e != hipSuccess) return e;
    const int threads = (la.n_lags + 63) / 64 * 64;
    switch (lane_qmax(la.Q)) {
    case 8: hipLaunchKernelGGL(lane_main<8>, dim3(n_blocks), dim3(threads), lds, stream, la); break;
    case 12: hipLaunchKernelGGL(lane_main<12>, dim3(n_blocks), dim3(threads), lds, stream, la); break;
    default: hipLaunchKernelGGL(lane_main<16>, dim3(n_blocks), dim3(threads), lds, stream, la); break;
    }
    return hipGetLastError();
}

}  // namespace covest
