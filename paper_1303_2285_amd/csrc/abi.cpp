// abi.cpp -- the C ABI of libcovest (declared in include/covest.h).
//
// Argument checking, plan caching (host job tables uploaded once per shape and
// device), workspace layout, kernel launches and optional event timing.  No
// arithmetic of the method happens here.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <cstdarg>
#include <cstdio>
#include <cstdlib>
#include <cstring>
#include <fstream>
#include <sstream>
#include <map>
#include <memory>
#include <mutex>
#include <string>
#include <tuple>
#include <vector>

#include "covest.h"
#include "covest_plan.h"
#include "adj_internal.hpp"
#include "capon_internal.hpp"
#include "lane_internal.hpp"
#include "launch.hpp"
#include "noalloc_internal.hpp"
#include "plan.hpp"

using namespace covest;

namespace {

thread_local std::string g_err;

int fail(int status, const char *fmt, ...)
{
    char buf[512];
    va_list ap;
    va_start(ap, fmt);
    vsnprintf(buf, sizeof(buf), fmt, ap);
    va_end(ap);
    g_err = buf;
    return status;
}

int ok()
{
    g_err.clear();
    return COVEST_OK;
}

bool sync_mode()
{
    static const bool on = [] {
        const char *s = std::getenv("COVEST_SYNC");
        return s && s[0] == '1';
    }();
    return on;
}

#define HIP_TRY(expr)                                                                    \
    do {                                                                                 \
        hipError_t e_ = (expr);                                                          \
        if (e_ != hipSuccess)                                                            \
            return fail(COVEST_ERR_HIP, "%s failed: %s", #expr, hipGetErrorString(e_)); \
    } while (0)

// ---------------------------------------------------------------- timing ----
struct Pending {
    std::string name;
    hipEvent_t a, b;
};
std::mutex g_tmu;
bool g_timing = false;
std::vector<Pending> g_pending;
std::map<std::string, std::pair<int64_t, double>> g_totals;

template <class F>
hipError_t timed(const char *name, hipStream_t s, F &&launch)
{
    bool on;
    {
        std::lock_guard<std::mutex> lk(g_tmu);
        on = g_timing;
    }
    if (!on) return launch();
    hipEvent_t a, b;
    hipError_t e = hipEventCreate(&a);
    if (e != hipSuccess) return e;
    e = hipEventCreate(&b);
    if (e != hipSuccess) return e;
    (void)hipEventRecord(a, s);
    e = launch();
    (void)hipEventRecord(b, s);
    std::lock_guard<std::mutex> lk(g_tmu);
    g_pending.push_back({name, a, b});
    return e;
}

// ------------------------------------------------------------ validation ----
covest_opts resolve_opts(const covest_opts *o)
{
    covest_opts r{};
    r.form = COVEST_FORM_AUTO;
    r.prec = COVEST_PREC_FP64;
    r.fill = COVEST_FILL_FULL;
    r.normalize = 1;
    r.ring_cols = r.ring_rows = 0;
    r.engine = COVEST_ENGINE_AUTO;
    if (o) r = *o;
    return r;
}

int check_opts(const covest_opts &o)
{
    if (o.form < COVEST_FORM_AUTO || o.form > COVEST_FORM_HANKEL_MFMA)
        return fail(COVEST_ERR_INVALID_ARG, "unknown form %d", (int)o.form);
    if (o.prec < COVEST_PREC_FP64 || o.prec > COVEST_PREC_FP16)
        return fail(COVEST_ERR_INVALID_ARG, "unknown precision %d", (int)o.prec);
    if (o.fill != COVEST_FILL_FULL && o.fill != COVEST_FILL_UPPER)
        return fail(COVEST_ERR_INVALID_ARG, "unknown fill %d", (int)o.fill);
    for (int w : {o.ring_cols, o.ring_rows})
        if (w != 0 && w != 4 && w != 8 && w != 12 && w != 16)
            return fail(COVEST_ERR_INVALID_ARG, "ring widths are 0, 4, 8, 12 or 16 (got %d)", w);
    if (o.engine < COVEST_ENGINE_AUTO || o.engine > COVEST_ENGINE_LANE)
        return fail(COVEST_ERR_INVALID_ARG, "unknown engine %d", (int)o.engine);
    return COVEST_OK;
}

int check_shape(int64_t N, int64_t M, int64_t P, int64_t Q)
{
    if (N < 1 || M < 1 || P < 1 || Q < 1 || P > N || Q > M)
        return fail(COVEST_ERR_SHAPE, "need 1 <= P <= N and 1 <= Q <= M (N=%lld M=%lld P=%lld Q=%lld)",
                    (long long)N, (long long)M, (long long)P, (long long)Q);
    if (N > (1 << 20) || M > (1 << 20))
        return fail(COVEST_ERR_SHAPE, "N and M are limited to 2^20");
    return COVEST_OK;
}

bool use_recurrence(const covest_opts &o)
{
    return o.form == COVEST_FORM_AUTO || o.form == COVEST_FORM_RECURRENCE;
}

// ------------------------------------------------------------ plan cache ----
struct DevPlan {
    ShapePlan sp;
    Job *d_jobs = nullptr;
    LagGroup *d_groups = nullptr;
    FinItem *d_items = nullptr;
    MJob *d_mjobs = nullptr;
    int xcd_remap = 0;
};

using PlanKey = std::tuple<int, int, int, int, int, int, int, int>;
std::mutex g_pmu;
std::map<PlanKey, std::unique_ptr<DevPlan>> g_plans;

int cus_of_device(int dev)
{
    int cus = 0;
    if (hipDeviceGetAttribute(&cus, hipDeviceAttributeMultiprocessorCount, dev) != hipSuccess || cus <= 0)
        cus = 256;
    return cus;
}

int n_slots_for_device(int dev) { return 2 * cus_of_device(dev); }

// Engine of the recurrence's main pass for this shape and options: 1 vector,
// 2 matrix cores, 0 when the requested engine cannot run the shape.
// 2: matrix cores, 1: vector units, 0: the forced matrix engine cannot run
// this shape.  AUTO takes the matrix cores above min_fill.
int pick_engine(int N, int M, int P, int Q, const covest_opts &o, bool batch = false)
{
    if (o.engine == COVEST_ENGINE_MATRIX) return mfma_fits(N, M, P, Q) ? 2 : 0;
    if (o.engine == COVEST_ENGINE_VECTOR) return 1;
    return (mfma_preferred(N, M, P, Q, batch) && o.ring_cols == 0 && o.ring_rows == 0) ? 2 : 1;
}

ShapePlan plan_for(int N, int M, int P, int Q, int cus, int w0, int w1, int engine)
{
    if (engine == 2) return make_mfma_plan(N, M, P, Q, cus);
    return make_shape_plan(N, M, P, Q, 2 * cus, w0, w1);
}

template <class T>
hipError_t upload(T **dst, const std::vector<T> &src)
{
    *dst = nullptr;
    if (src.empty()) return hipSuccess;
    hipError_t e = hipMalloc(reinterpret_cast<void **>(dst), sizeof(T) * src.size());
    if (e != hipSuccess) return e;
    return hipMemcpy(*dst, src.data(), sizeof(T) * src.size(), hipMemcpyHostToDevice);
}

int get_plan(int N, int M, int P, int Q, int w0, int w1, int engine, DevPlan **out)
{
    int dev = 0;
    HIP_TRY(hipGetDevice(&dev));
    auto key = std::make_tuple(dev, N, M, P, Q, w0, w1, engine);
    std::lock_guard<std::mutex> lk(g_pmu);
    auto it = g_plans.find(key);
    if (it != g_plans.end()) {
        *out = it->second.get();
        return COVEST_OK;
    }
    auto dp = std::make_unique<DevPlan>();
    dp->sp = plan_for(N, M, P, Q, cus_of_device(dev), w0, w1, engine);
    HIP_TRY(upload(&dp->d_jobs, dp->sp.jobs));
    HIP_TRY(upload(&dp->d_groups, dp->sp.groups));
    HIP_TRY(upload(&dp->d_items, dp->sp.items));
    HIP_TRY(upload(&dp->d_mjobs, dp->sp.mjobs));
    dp->xcd_remap = 1;
    *out = dp.get();
    g_plans.emplace(key, std::move(dp));
    return COVEST_OK;
}

std::mutex g_hmu;
std::map<PlanKey, std::shared_ptr<const ShapePlan>> g_host_plans;

// Host-only planning, cached (workspace queries must work without a device).
std::shared_ptr<const ShapePlan> host_plan(int N, int M, int P, int Q, int w0, int w1, int engine)
{
    int dev = 0, cus = 256;
    if (hipGetDevice(&dev) == hipSuccess) cus = cus_of_device(dev);
    auto key = std::make_tuple(cus, N, M, P, Q, w0, w1, engine);
    std::lock_guard<std::mutex> lk(g_hmu);
    auto it = g_host_plans.find(key);
    if (it != g_host_plans.end()) return it->second;
    auto sp = std::make_shared<const ShapePlan>(plan_for(N, M, P, Q, cus, w0, w1, engine));
    g_host_plans.emplace(key, sp);
    return sp;
}

Inst make_inst(const ShapePlan &sp, const void *A, int64_t lda, void *R, int64_t ldr, void *ws,
               const covest_opts &o)
{
    Inst in{};
    in.A = A;
    in.R = R;
    in.lda = lda;
    in.ldr = ldr;
    in.N = sp.N;
    in.M = sp.M;
    in.P = sp.P;
    in.Q = sp.Q;
    in.Kr = sp.N - sp.P + 1;
    in.Kc = sp.M - sp.Q + 1;
    in.Rm0 = sp.Rm0;
    in.Rm1 = sp.Rm1;
    in.Cm0 = sp.Cm0;
    in.Cm1 = sp.Cm1;
    in.n_ir = sp.n_ir;
    in.n_ic = sp.n_ic;
    in.lag_stride = sp.lag_stride;
    in.bandw = sp.bandw;
    in.slots0 = sp.slots0;
    double *base = static_cast<double *>(ws);
    in.partial = base;
    in.zr = base + (size_t)2 * sp.lag_stride * sp.n_bulk;
    in.zc = in.zr + (size_t)2 * sp.lag_stride * sp.n_ir * sp.zpieces;
    in.out_fp64 = o.prec == COVEST_PREC_FP64 ? 1 : 0;
    in.fill_full = o.fill == COVEST_FILL_FULL ? 1 : 0;
    in.normalize = o.normalize ? 1 : 0;
    in.zpieces = sp.zpieces;
    return in;
}

int finish_call(hipStream_t stream)
{
    HIP_TRY(hipGetLastError());
    if (sync_mode()) {
        HIP_TRY(hipStreamSynchronize(stream));
        HIP_TRY(hipGetLastError());
    }
    return ok();
}

// Engine of the main pass for one call: 1 vector, 2 matrix cores; a status
// when the requested engine cannot run the shape.
int rec_engine(int N, int M, int P, int Q, int64_t lda, const covest_opts &o, int *engine)
{
    if (o.engine == COVEST_ENGINE_LANE)
        return fail(COVEST_ERR_UNSUPPORTED, "the lane engine runs covest_forward, _ex, _noalloc and aperture "
                                            "plans only");
    if (P > kMaxWindow || Q > kMaxWindow)
        return fail(COVEST_ERR_UNSUPPORTED, "the recurrence form supports P, Q <= %d", kMaxWindow);
    if (o.prec != COVEST_PREC_FP64 && o.prec != COVEST_PREC_FP32)
        return fail(COVEST_ERR_UNSUPPORTED, "the recurrence form computes in FP64 (prec FP64 or FP32 output)");
    int e = pick_engine(N, M, P, Q, o);
    if (e == 0)
        return fail(COVEST_ERR_UNSUPPORTED, "the matrix-core engine needs N >= 2P-1, M >= 2Q-1 and a lag "
                                            "block of at most 8 tiles of 16 x 16 with little padding");
    // the matrix-core kernel addresses A with 32-bit element offsets
    if (e == 2 && (int64_t)N * lda + M >= ((int64_t)1 << 31)) {
        if (o.engine == COVEST_ENGINE_MATRIX)
            return fail(COVEST_ERR_UNSUPPORTED, "the matrix-core engine needs N * lda < 2^31");
        e = 1;
    }
    *engine = e;
    return COVEST_OK;
}

// Device copies of one shape plan's tables.
struct DevTables {
    const Job *jobs;
    const LagGroup *groups;
    const FinItem *items;
    const MJob *mjobs;
    int xcd_remap;
};

// The recurrence's launches for one problem: main pass (matrix cores or
// vector units), then the finalize.
int rec_launch(const ShapePlan &sp, const DevTables &t, const Inst &in, hipStream_t stream,
               unsigned long long *stamps = nullptr)
{
    if (!sp.mjobs.empty()) {
        MfmaArgs ma{};
        ma.jobs = t.mjobs;
        ma.n_jobs = (int)sp.mjobs.size();
        ma.xcd_remap = t.xcd_remap;
        ma.inst = in;
        HIP_TRY(timed("rec_mfma", stream, [&] {
            return launch_rec_mfma(ma, sp.mt, sp.nt, (int)sp.mjobs.size(), sp.lds_main, stream);
        }));
    } else if (!sp.jobs.empty()) {
        MainArgs ma{};
        ma.jobs = t.jobs;
        ma.groups = t.groups;
        ma.insts = nullptr;
        ma.n_jobs = (int)sp.jobs.size();
        ma.xcd_remap = t.xcd_remap;
        ma.use_inline = 1;
        ma.inst_inline = in;
        HIP_TRY(timed("rec_main", stream, [&] {
            return launch_rec_main(ma, (int)sp.jobs.size(), sp.lds_main, stream);
        }));
    }
    FinArgs fa{};
    fa.items = t.items;
    fa.insts = nullptr;
    fa.n_items = (int)sp.items.size();
    fa.use_inline = 1;
    fa.inst_inline = in;
    fa.stamps = stamps;
    HIP_TRY(timed("rec_finalize", stream, [&] {
        return launch_rec_finalize(fa, (int)sp.items.size(), sp.lds_fin, sp.fin_variant, stream);
    }));
    return finish_call(stream);
}

int rec_forward(const void *A, int64_t lda, int N, int M, int P, int Q, void *R, int64_t ldr,
                const covest_opts &o, void *ws, size_t ws_bytes, hipStream_t stream,
                unsigned long long *stamps = nullptr, int64_t n_stamps = 0)
{
    int engine = 0;
    int st = rec_engine(N, M, P, Q, lda, o, &engine);
    if (st != COVEST_OK) return st;
    DevPlan *dp = nullptr;
    st = get_plan(N, M, P, Q, o.ring_cols, o.ring_rows, engine, &dp);
    if (st != COVEST_OK) return st;
    const ShapePlan &sp = dp->sp;
    if (ws_bytes < sp.ws_bytes || (sp.ws_bytes > 0 && ws == nullptr))
        return fail(COVEST_ERR_WORKSPACE, "workspace of %zu bytes needed, %zu given", sp.ws_bytes, ws_bytes);
    if (stamps && n_stamps < 2 * (int64_t)sp.items.size())
        return fail(COVEST_ERR_INVALID_ARG, "stamps hold %lld values, the finalize has %zu items (2 each)",
                    (long long)n_stamps, sp.items.size());
    const Inst in = make_inst(sp, A, lda, R, ldr, ws, o);
    return rec_launch(sp, DevTables{dp->d_jobs, dp->d_groups, dp->d_items, dp->d_mjobs, dp->xcd_remap}, in,
                      stream, stamps);
}

// ------------------------------------------------------ fixed scratch ----
// covest_forward_noalloc: the same plan and kernels as rec_forward, with the
// plan's tables and the workspace in the device's fixed scratch array instead
// of cached device allocations and a caller workspace.  The tables are copied
// into the scratch when the shape differs from the one whose tables it holds.
size_t align256(size_t b) { return (b + 255) / 256 * 256; }

struct ScratchLayout {
    size_t jobs, groups, items, mjobs, ws, total;
};

ScratchLayout scratch_layout(const ShapePlan &sp)
{
    ScratchLayout l{};
    l.jobs = 0;
    l.groups = l.jobs + align256(sizeof(Job) * sp.jobs.size());
    l.items = l.groups + align256(sizeof(LagGroup) * sp.groups.size());
    l.mjobs = l.items + align256(sizeof(FinItem) * sp.items.size());
    l.ws = l.mjobs + align256(sizeof(MJob) * sp.mjobs.size());
    l.total = l.ws + sp.ws_bytes;
    return l;
}

std::mutex g_smu;
std::map<int, PlanKey> g_scratch_tables;   // device -> plan whose tables its scratch holds

template <class T>
hipError_t copy_table(unsigned char *dst, const std::vector<T> &src, hipStream_t stream)
{
    if (src.empty()) return hipSuccess;
    return hipMemcpyAsync(dst, src.data(), sizeof(T) * src.size(), hipMemcpyHostToDevice, stream);
}

int rec_forward_noalloc(const void *A, int64_t lda, int N, int M, int P, int Q, void *R, int64_t ldr,
                        const covest_opts &o, hipStream_t stream)
{
    int engine = 0;
    int st = rec_engine(N, M, P, Q, lda, o, &engine);
    if (st != COVEST_OK) return st;
    const auto sp = host_plan(N, M, P, Q, o.ring_cols, o.ring_rows, engine);
    const ScratchLayout l = scratch_layout(*sp);
    if (l.total > kNoallocScratchBytes)
        return fail(COVEST_ERR_WORKSPACE, "this shape needs %zu bytes of scratch; the fixed scratch holds %zu",
                    l.total, (size_t)kNoallocScratchBytes);
    void *base_v = nullptr;
    HIP_TRY(noalloc_scratch(&base_v));
    unsigned char *base = static_cast<unsigned char *>(base_v);
    int dev = 0;
    HIP_TRY(hipGetDevice(&dev));
    int cus = cus_of_device(dev);
    const PlanKey key = std::make_tuple(cus, N, M, P, Q, o.ring_cols, o.ring_rows, engine);
    {
        std::lock_guard<std::mutex> lk(g_smu);
        auto it = g_scratch_tables.find(dev);
        if (it == g_scratch_tables.end() || it->second != key) {
            if (it != g_scratch_tables.end()) g_scratch_tables.erase(it);
            HIP_TRY(copy_table(base + l.jobs, sp->jobs, stream));
            HIP_TRY(copy_table(base + l.groups, sp->groups, stream));
            HIP_TRY(copy_table(base + l.items, sp->items, stream));
            HIP_TRY(copy_table(base + l.mjobs, sp->mjobs, stream));
            g_scratch_tables.emplace(dev, key);
        }
    }
    const DevTables t{reinterpret_cast<const Job *>(base + l.jobs),
                      reinterpret_cast<const LagGroup *>(base + l.groups),
                      reinterpret_cast<const FinItem *>(base + l.items),
                      reinterpret_cast<const MJob *>(base + l.mjobs), 1};
    const Inst in = make_inst(*sp, A, lda, R, ldr, base + l.ws, o);
    return rec_launch(*sp, t, in, stream);
}

// ----------------------------------------------------------- lane engine ----
int lane_check(int N, int M, int P, int Q, const covest_opts &o)
{
    if (o.prec != COVEST_PREC_FP64 && o.prec != COVEST_PREC_FP32)
        return fail(COVEST_ERR_UNSUPPORTED, "the lane engine computes in FP64 (prec FP64 or FP32 output)");
    if (!lane_fits(N, M, P, Q))
        return fail(COVEST_ERR_UNSUPPORTED,
                    "the lane engine needs Q <= %d, PQ + (P-1)(Q-1) <= %d and %zu bytes of staged rows "
                    "<= %zu (N=%d M=%d P=%d Q=%d)",
                    kLaneMaxQ, kLaneMaxLags, lane_lds_bytes(M, P, Q), kLaneMaxLds, N, M, P, Q);
    return COVEST_OK;
}

// Inputs per workgroup along a grid column.  A new box costs Kr + 2(P-1)
// row walks (the first Kr rows, then two per window row); the next input of
// a chain costs 2*row_step (its box slides down from the previous input's).
// Chains are as long as keep four workgroups per compute unit.
int lane_chain(int N, int P, int64_t row_step, int64_t n_rows, int64_t n_cols, int cus, bool env)
{
    if (env) {
        if (const char *e = std::getenv("COVEST_AP_CHAIN")) {
            const long v = std::strtol(e, nullptr, 10);
            if (v >= 1) return (int)std::min<int64_t>(v, n_rows);
        }
    }
    const int Kr = N - P + 1;
    if (2 * row_step >= (int64_t)Kr + 2 * (P - 1)) return 1;
    const int64_t target = 4 * (int64_t)cus;
    return (int)std::max<int64_t>(1, std::min<int64_t>(n_rows, n_rows * n_cols / target));
}

LaneArgs make_lane_args(const void *image, int64_t ld, int N, int M, int P, int Q, int64_t row_step,
                        int64_t col_step, int64_t n_rows, int64_t n_cols, int chain, void *R, int64_t ldr,
                        int64_t r_stride, const covest_opts &o)
{
    LaneArgs la{};
    la.image = static_cast<const float2 *>(image);
    la.ld = ld;
    la.N = N;
    la.M = M;
    la.P = P;
    la.Q = Q;
    la.Kr = N - P + 1;
    la.Kc = M - Q + 1;
    la.row_step = (int)row_step;
    la.col_step = (int)col_step;
    la.n_rows = (int)n_rows;
    la.n_cols = (int)n_cols;
    la.chain = chain;
    la.n_lags = lane_n_lags(P, Q);
    la.R = R;
    la.ldr = ldr;
    la.r_stride = r_stride;
    la.out_fp64 = o.prec == COVEST_PREC_FP64 ? 1 : 0;
    la.fill_full = o.fill == COVEST_FILL_FULL ? 1 : 0;
    la.normalize = o.normalize ? 1 : 0;
    la.gstride = lane_gstride(M, Q);
    la.ring = lane_ring(P);
    return la;
}

int lane_blocks(const LaneArgs &la) { return la.n_cols * ((la.n_rows + la.chain - 1) / la.chain); }

int lane_run(const LaneArgs &la, hipStream_t stream)
{
    HIP_TRY(timed("lane_main", stream, [&] {
        return launch_lane(la, lane_blocks(la), lane_lds_bytes(la.M, la.P, la.Q), stream);
    }));
    return finish_call(stream);
}

// One input on the lane engine: a 1 x 1 grid.
int lane_forward(const void *A, int64_t lda, int N, int M, int P, int Q, void *R, int64_t ldr,
                 const covest_opts &o, hipStream_t stream)
{
    int st = lane_check(N, M, P, Q, o);
    if (st != COVEST_OK) return st;
    return lane_run(make_lane_args(A, lda, N, M, P, Q, 1, 1, 1, 1, 1, R, ldr, 0, o), stream);
}

// ------------------------------------------------------------ plain form ----
int hankel_prec(covest_precision p)
{
    switch (p) {
    case COVEST_PREC_FP32: return kPrecF32;
    case COVEST_PREC_BF16X3: return kPrecBF16x3;
    case COVEST_PREC_FP16X3: return kPrecF16x3;
    case COVEST_PREC_BF16: return kPrecBF16;
    case COVEST_PREC_FP16: return kPrecF16;
    default: return -1;
    }
}

struct DevHankel {
    HankelPlan hp;
    HItem *d_items = nullptr;
    HTile *d_tiles = nullptr;
    int *d_item_index = nullptr;
};
std::map<std::tuple<int, int, int, int, int, int>, std::unique_ptr<DevHankel>> g_hplans;

int cu_count(int dev)
{
    int cus = 0;
    if (hipDeviceGetAttribute(&cus, hipDeviceAttributeMultiprocessorCount, dev) != hipSuccess || cus <= 0)
        cus = 256;
    return cus;
}

std::shared_ptr<const HankelPlan> host_hankel_plan(int N, int M, int P, int Q, int prec)
{
    static std::mutex mu;
    static std::map<std::tuple<int, int, int, int, int, int>, std::shared_ptr<const HankelPlan>> cache;
    int dev = 0, cus = 256;
    if (hipGetDevice(&dev) == hipSuccess) cus = cu_count(dev);
    auto key = std::make_tuple(cus, N, M, P, Q, prec);
    std::lock_guard<std::mutex> lk(mu);
    auto it = cache.find(key);
    if (it != cache.end()) return it->second;
    auto hp = std::make_shared<const HankelPlan>(make_hankel_plan(N, M, P, Q, prec, cus));
    cache.emplace(key, hp);
    return hp;
}

int get_hankel_plan(int N, int M, int P, int Q, int prec, DevHankel **out)
{
    int dev = 0;
    HIP_TRY(hipGetDevice(&dev));
    auto key = std::make_tuple(dev, N, M, P, Q, prec);
    std::lock_guard<std::mutex> lk(g_pmu);
    auto it = g_hplans.find(key);
    if (it != g_hplans.end()) {
        *out = it->second.get();
        return COVEST_OK;
    }
    auto dh = std::make_unique<DevHankel>();
    dh->hp = make_hankel_plan(N, M, P, Q, prec, cu_count(dev));
    HIP_TRY(upload(&dh->d_items, dh->hp.items));
    HIP_TRY(upload(&dh->d_tiles, dh->hp.tiles));
    HIP_TRY(upload(&dh->d_item_index, dh->hp.item_index));
    *out = dh.get();
    g_hplans.emplace(key, std::move(dh));
    return COVEST_OK;
}

int hankel_forward(const void *A, int64_t lda, int N, int M, int P, int Q, void *R, int64_t ldr,
                   const covest_opts &o, void *ws, size_t ws_bytes, hipStream_t stream)
{
    const int prec = hankel_prec(o.prec);
    if (prec < 0) return fail(COVEST_ERR_UNSUPPORTED, "the matrix-core form has no FP64 precision");
    if (P > kMaxWindow || Q > kMaxWindow)
        return fail(COVEST_ERR_UNSUPPORTED, "the matrix-core form supports P, Q <= %d", kMaxWindow);
    DevHankel *dh = nullptr;
    int st = get_hankel_plan(N, M, P, Q, prec, &dh);
    if (st != COVEST_OK) return st;
    const HankelPlan &hp = dh->hp;
    if (ws_bytes < hp.ws_bytes || ws == nullptr)
        return fail(COVEST_ERR_WORKSPACE, "workspace of %zu bytes needed, %zu given", hp.ws_bytes, ws_bytes);
    HankelArgs ha{};
    ha.A = static_cast<const float2 *>(A);
    ha.lda = lda;
    ha.N = N;
    ha.M = M;
    ha.P = P;
    ha.Q = Q;
    ha.PQ = P * Q;
    ha.Kr = N - P + 1;
    ha.Kc = M - Q + 1;
    ha.pb = hp.pb;
    ha.qb = hp.qb;
    ha.stride_a = hp.stride_a;
    ha.stride_b = hp.stride_b;
    ha.items = dh->d_items;
    ha.tiles = dh->d_tiles;
    ha.R = R;
    ha.ldr = ldr;
    ha.fill_full = o.fill == COVEST_FILL_FULL ? 1 : 0;
    ha.normalize = o.normalize ? 1 : 0;
    if (prec != kPrecF32) {
        ha.planes = static_cast<const unsigned int *>(ws);
        ha.ldp = hp.ldp;
        ha.plane_elems = (int64_t)N * hp.ldp;
        ha.partial32 = reinterpret_cast<float2 *>(static_cast<char *>(ws) + hp.planes_bytes);
        ha.tn = hp.tn;
        ha.item_index = dh->d_item_index;
        HIP_TRY(timed("hankel_split", stream, [&] { return launch_hankel_split(ha, prec, stream); }));
        HIP_TRY(timed("hankel_main16", stream, [&] {
            return launch_hankel_main16(ha, prec, (int)hp.items.size(), hp.lds, stream);
        }));
        HIP_TRY(timed("hankel_reduce16", stream, [&] {
            return launch_hankel_reduce16(ha, (int)hp.tiles.size(), stream);
        }));
        return finish_call(stream);
    }
    ha.partial = static_cast<double *>(ws);
    HIP_TRY(timed("hankel_main", stream, [&] {
        return launch_hankel_main(ha, prec, (int)hp.items.size(), hp.lds, stream);
    }));
    HIP_TRY(timed("hankel_reduce", stream, [&] {
        return launch_hankel_reduce(ha, (int)hp.tiles.size(), stream);
    }));
    return finish_call(stream);
}

// --------------------------------------------------------------- adjoint ----
struct AdjGeom {
    int ir0, ir1, ic0, ic1, ndc, n_lags, interior_blocks;
    int64_t frame_jobs;
    size_t lds_tables, lds_interior, ws_bytes;
    // matrix-core interior (windows up to 16 x 16 with an interior)
    bool mfma;
    int ny, nx, mtiles, mranges;
    size_t lds_frame;   // LDS of the frame's launch
    // workspace byte offsets: prefix tables, full sums, line-job weights,
    // boundary rows of the matrix-core interior
    size_t off_tables, off_hfull, off_wrows, off_wcols, off_bnd;
};

AdjGeom adj_geometry(int N, int M, int P, int Q)
{
    AdjGeom g{};
    const int Kr = N - P + 1, Kc = M - Q + 1;
    g.n_lags = (2 * P - 1) * (2 * Q - 1);
    g.ndc = ((2 * Q - 1 + kAdjRing - 1) / kAdjRing) * kAdjRing;
    g.lds_tables = (size_t)(P + 1) * (Q + 1) * 16;
    const int rows = kAdjTR + 2 * (P - 1);
    const int stride = (kAdjTC + g.ndc) | 1;
    g.lds_interior = std::max((size_t)(2 * P - 1) * g.ndc * 16 + (size_t)rows * stride * 8,
                              (size_t)256 * kAdjRing * 16);
    const bool interior = Kr > P - 1 && Kc > Q - 1 && g.lds_interior <= 150 * 1024;
    if (interior) {
        g.ir0 = P - 1;
        g.ir1 = Kr;
        g.ic0 = Q - 1;
        g.ic1 = Kc;
        g.interior_blocks = ((g.ir1 - g.ir0 + kAdjTR - 1) / kAdjTR) * ((g.ic1 - g.ic0 + kAdjTC - 1) / kAdjTC);
    } else {
        g.ir0 = g.ir1 = N;   // no interior: the frame is every output
        g.ic0 = g.ic1 = 0;
        g.interior_blocks = 0;
    }
    // frame jobs: border rows x interior-column lines, border columns x
    // interior-row lines, border rows x border columns
    const int64_t nbr = N - (g.ir1 - g.ir0), nbc = M - (g.ic1 - g.ic0);
    g.frame_jobs = nbr * ((g.ic1 - g.ic0 + kAdjFL - 1) / kAdjFL) + nbc * ((g.ir1 - g.ir0 + kAdjFL - 1) / kAdjFL) +
                   nbr * nbc;
    size_t off = 0;
    g.off_tables = off;
    off += (size_t)g.n_lags * (P + 1) * (Q + 1) * 16;
    g.off_hfull = off;
    off += (size_t)g.n_lags * 16;
    g.off_wrows = off;
    g.off_wcols = off;
    if (interior) {
        off += (size_t)nbr * g.n_lags * 16;
        g.off_wcols = off;
        off += (size_t)nbc * g.n_lags * 16;
    }
    g.off_bnd = off;
    g.ws_bytes = off;
    g.mfma = interior && P <= kAdjMMaxWin && Q <= kAdjMMaxWin;
    if (g.mfma) {
        g.ny = g.ir1 - g.ir0;
        g.nx = g.ic1 - g.ic0;
        g.mtiles = (g.nx + 15) / 16;
        g.mranges = (N + kAdjMSpan - 1) / kAdjMSpan;
        g.ws_bytes += (size_t)(g.mranges - 1) * 2 * (2 * P - 2) * 16 * g.mtiles * 16;
        // the frame: every weight row of the wider line kind in one slab (at
        // most 32 rows), and at least the corner jobs' 256-entry sum
        const size_t row_slab = (size_t)std::min(2 * P - 1, 32) * adj_line_row_bytes(2 * Q - 1);
        const size_t col_slab = (size_t)std::min(2 * Q - 1, 32) * adj_line_row_bytes(2 * P - 1);
        g.lds_frame = std::min<size_t>(kAdjFrameLds, std::max<size_t>({256 * 16, row_slab, col_slab}));
    }
    return g;
}

}  // namespace

// -------------------------------------------------------------- batches ----
// A batched plan: one work list for every problem (longest job first), the
// persistent main kernel, one matrix-core launch per lag-block shape and one
// finalize launch per finalize variant, all captured in one graph.
struct covest_plan {
    int device = 0;
    covest_opts opts{};
    int64_t count = 0;
    hipStream_t own_stream = nullptr;
    hipStream_t side_stream = nullptr;           // second branch of the captured graph
    hipEvent_t ev_fork = nullptr, ev_join = nullptr;
    Job *d_jobs = nullptr;
    LagGroup *d_groups = nullptr;
    Inst *d_insts = nullptr;
    // finalize items per engine of their problem (0 vector, 1 matrix cores) and variant
    FinItem *d_items[2][kFinVariants] = {};
    unsigned int *d_counter = nullptr;
    void *d_ws = nullptr;
    int n_jobs = 0, n_items[2][kFinVariants] = {}, grid = 0;
    size_t lds_main = 0, lds_fin[kFinVariants] = {};
    // matrix-core jobs, one launch per lag-block shape (mt x nt tiles)
    struct MfmaLaunch {
        int mt = 0, nt = 0, n_jobs = 0;
        MJob *d_jobs = nullptr;
        size_t lds = 0;
    };
    std::vector<MfmaLaunch> mfma;
    int n_matrix = 0;   // problems on the matrix-core engine
    // aperture plans on the lane engine: one launch, no tables, no graph
    bool lane = false;
    LaneArgs lane_args{};
    hipGraph_t graph = nullptr;
    hipGraphExec_t exec = nullptr;
    double est_cost = 0.0;
};

namespace {

void free_plan(covest_plan *p)
{
    if (!p) return;
    if (p->exec) (void)hipGraphExecDestroy(p->exec);
    if (p->graph) (void)hipGraphDestroy(p->graph);
    void *bufs[] = {p->d_jobs, p->d_groups, p->d_insts, p->d_counter, p->d_ws};
    for (void *b : bufs)
        if (b) (void)hipFree(b);
    for (auto &per_engine : p->d_items)
        for (FinItem *b : per_engine)
            if (b) (void)hipFree(b);
    for (auto &l : p->mfma)
        if (l.d_jobs) (void)hipFree(l.d_jobs);
    if (p->own_stream) (void)hipStreamDestroy(p->own_stream);
    if (p->side_stream) (void)hipStreamDestroy(p->side_stream);
    if (p->ev_fork) (void)hipEventDestroy(p->ev_fork);
    if (p->ev_join) (void)hipEventDestroy(p->ev_join);
    delete p;
}

// ------------------------------------------------------------- autotuner --
// Ring widths (tile shapes of the vector kernel) per (P, Q) class, chosen by
// timing the class's problems as the batch runs them.  Results are kept for
// the process and, when COVEST_TUNE_CACHE names a file, in that file
// ("P Q W0 W1" per line).  COVEST_TUNE=0 keeps the default widths.
std::mutex g_tune_mu;
std::map<std::pair<int, int>, std::pair<int, int>> g_tune;
bool g_tune_loaded = false;

const char *tune_path() { return std::getenv("COVEST_TUNE_CACHE"); }

// COVEST_WORKERS=n (n >= 1), read when a batched plan is built, caps the
// persistent kernel at n workgroups: every job still runs, claimed by n
// workers (speedup against the number of workers, as in Sec. 5.1, Fig. 4).
int worker_cap()
{
    const char *s = std::getenv("COVEST_WORKERS");
    if (!s || !*s) return 0;
    const long n = std::strtol(s, nullptr, 10);
    return n > 0 && n <= (1 << 20) ? (int)n : 0;
}

void tune_load_locked()
{
    if (g_tune_loaded) return;
    g_tune_loaded = true;
    const char *path = tune_path();
    if (!path) return;
    std::ifstream f(path);
    std::string line;
    int n = 0;
    while (std::getline(f, line)) {
        std::istringstream is(line);
        int P, Q, w0, w1;
        if (!(is >> P >> Q >> w0 >> w1) || P < 1 || Q < 1 ||
            (w0 != 4 && w0 != 8 && w0 != 12 && w0 != 16) || (w1 != 4 && w1 != 8 && w1 != 12 && w1 != 16)) {
            std::fprintf(stderr, "libcovest: ignoring malformed tune cache line in %s: '%s'\n", path, line.c_str());
            continue;
        }
        g_tune[{P, Q}] = {w0, w1};
        ++n;
    }
}

void tune_store_locked(int P, int Q, int w0, int w1)
{
    g_tune[{P, Q}] = {w0, w1};
    const char *path = tune_path();
    if (!path) return;
    std::ofstream f(path, std::ios::app);
    if (f) f << P << " " << Q << " " << w0 << " " << w1 << "\n";
}

bool tuning_enabled()
{
    const char *s = std::getenv("COVEST_TUNE");
    return !(s && s[0] == '0');
}

// Time the vector kernel on every problem of one (P, Q) class with ring
// widths (w0, w1), as the batch runs them: each problem split into jobs in
// proportion to its cost, all jobs longest first in one persistent launch
// (events on a private stream, best of three after a warm-up).  The kernel
// writes only workspace sums, so no output is touched.
using Widths = std::map<std::pair<int, int>, std::pair<int, int>>;

int time_class(const covest_problem_ex *pr, const std::vector<int64_t> &members, const covest_opts &o,
               int resident, const Widths &widths, size_t lds_cap, hipStream_t s, float *best_ms)
{
    auto wfor = [&](const covest_problem_ex &p) {
        auto it = widths.find({(int)p.P, (int)p.Q});
        return it == widths.end() ? std::make_pair(0, 0) : it->second;
    };
    std::vector<double> cost(members.size(), 0.0);
    double total = 0.0;
    for (size_t t = 0; t < members.size(); ++t) {
        const covest_problem_ex &p = pr[members[t]];
        const auto w = wfor(p);
        for (double c : make_shape_plan(p.N, p.M, p.P, p.Q, 1, w.first, w.second).job_cost) cost[t] += c;
        total += cost[t];
    }
    const double target = std::max(1.0, total / (3.0 * resident));
    std::vector<ShapePlan> plans;
    size_t ws_off = 0, lds = 0;
    std::vector<size_t> ws_base;
    for (size_t t = 0; t < members.size(); ++t) {
        const covest_problem_ex &p = pr[members[t]];
        const int slots = (int)std::max<int64_t>(1, std::min<int64_t>(resident, std::llround(cost[t] / target)));
        const auto w = wfor(p);
        plans.push_back(make_shape_plan(p.N, p.M, p.P, p.Q, slots, w.first, w.second));
        ws_base.push_back(ws_off);
        ws_off += (plans.back().ws_bytes + 255) / 256 * 256;
        lds = std::max(lds, plans.back().lds_main);
    }
    if (lds > lds_cap) {   // would lower the occupancy of the whole batch's launch
        *best_ms = 1e30f;
        return COVEST_OK;
    }
    lds = lds_cap;   // the batch launches with the largest LDS of any of its problems
    void *ws = nullptr;
    HIP_TRY(hipMalloc(&ws, std::max<size_t>(ws_off, 256)));
    std::vector<Job> jobs;
    std::vector<double> jcost;
    std::vector<LagGroup> groups;
    std::vector<Inst> insts;
    for (size_t t = 0; t < plans.size(); ++t) {
        const ShapePlan &sp = plans[t];
        const covest_problem_ex &p = pr[members[t]];
        const int goff = (int)groups.size();
        groups.insert(groups.end(), sp.groups.begin(), sp.groups.end());
        for (size_t j = 0; j < sp.jobs.size(); ++j) {
            Job jb = sp.jobs[j];
            jb.inst = (int)t;
            jb.group += goff;
            jobs.push_back(jb);
            jcost.push_back(sp.job_cost[j]);
        }
        insts.push_back(make_inst(sp, p.A, p.lda, p.R, p.ldr, static_cast<char *>(ws) + ws_base[t], o));
    }
    std::vector<size_t> order(jobs.size());
    for (size_t j = 0; j < order.size(); ++j) order[j] = j;
    std::stable_sort(order.begin(), order.end(), [&](size_t a, size_t b) { return jcost[a] > jcost[b]; });
    std::vector<Job> sorted;
    for (size_t j : order) sorted.push_back(jobs[j]);
    Job *dj = nullptr;
    LagGroup *dg = nullptr;
    Inst *di = nullptr;
    unsigned int *counter = nullptr;
    hipEvent_t a = nullptr, b = nullptr;
    hipError_t e = upload(&dj, sorted);
    if (e == hipSuccess) e = upload(&dg, groups);
    if (e == hipSuccess) e = upload(&di, insts);
    if (e == hipSuccess) e = hipMalloc(&counter, 256);
    if (e == hipSuccess) e = hipEventCreate(&a);
    if (e == hipSuccess) e = hipEventCreate(&b);
    float best = 1e30f;
    if (e == hipSuccess && !sorted.empty()) {
        MainArgs ma{};
        ma.jobs = dj;
        ma.groups = dg;
        ma.insts = di;
        ma.n_jobs = (int)sorted.size();
        ma.use_inline = 0;
        const int grid = std::max(1, std::min(resident, ma.n_jobs));
        for (int rep = 0; rep < 4 && e == hipSuccess; ++rep) {
            (void)hipEventRecord(a, s);
            e = launch_rec_persistent(ma, counter, grid, lds, s);
            (void)hipEventRecord(b, s);
            if (e == hipSuccess) e = hipEventSynchronize(b);
            float ms = 0.f;
            if (e == hipSuccess && rep > 0 && hipEventElapsedTime(&ms, a, b) == hipSuccess) best = std::min(best, ms);
        }
    }
    if (a) (void)hipEventDestroy(a);
    if (b) (void)hipEventDestroy(b);
    for (void *ptr : {(void *)dj, (void *)dg, (void *)di, (void *)counter, ws})
        if (ptr) (void)hipFree(ptr);
    if (e != hipSuccess) return fail(COVEST_ERR_HIP, "autotune launch: %s", hipGetErrorString(e));
    *best_ms = best;
    return COVEST_OK;
}

// Widths for every (P, Q) class of the batch that runs on the vector engine.
// Per class, a coordinate search (the column width, then the row width) over
// ring_width_candidates, timing the class's problems as the batch runs them;
// a candidate needs no more LDS than the batch's default plans (all vector
// jobs share one launch: a wider tile for one class would lower the
// occupancy of every other) and must be at least 3% faster.  A class's
// choice is then kept only if the launch of the whole batch's vector jobs
// gets at least 2% faster with it: the classes' jobs run side by side, and
// a choice that wins alone can lose in the mix (measured: choices made alone
// made the 512-problem batch 8% slower than the defaults).
int autotune(const covest_problem_ex *pr, int64_t count, const std::vector<int> &engine, const covest_opts &o,
             int resident, std::map<std::pair<int, int>, std::pair<int, int>> *out)
{
    std::map<std::pair<int, int>, std::vector<int64_t>> classes;
    for (int64_t i = 0; i < count; ++i)
        if (engine[i] == 1) classes[{(int)pr[i].P, (int)pr[i].Q}].push_back(i);   // vector engine only
    size_t lds_cap = 0;
    for (auto &kv : classes)
        for (int64_t i : kv.second)
            lds_cap = std::max(lds_cap, make_shape_plan(pr[i].N, pr[i].M, pr[i].P, pr[i].Q, 1).lds_main);
    std::lock_guard<std::mutex> lk(g_tune_mu);
    tune_load_locked();
    hipStream_t s = nullptr;
    std::vector<int64_t> all;   // every vector-engine problem of the batch
    for (auto &kv : classes) all.insert(all.end(), kv.second.begin(), kv.second.end());
    Widths chosen, pending;
    for (auto &kv : classes) {
        const int P = kv.first.first, Q = kv.first.second;
        auto hit = g_tune.find(kv.first);
        if (hit != g_tune.end()) {
            chosen[kv.first] = hit->second;
            continue;
        }
        chosen[kv.first] = {ring_width_candidates(Q)[0], ring_width_candidates(P)[0]};
        if (tuning_enabled()) pending[kv.first] = chosen[kv.first];
    }
    int st = COVEST_OK;
    if (!pending.empty()) {
        HIP_TRY(hipStreamCreateWithFlags(&s, hipStreamNonBlocking));
        // the whole batch's vector launch with the current choices
        float whole;
        st = time_class(pr, all, o, resident, chosen, lds_cap, s, &whole);
        for (auto &kv : pending) {
            if (st != COVEST_OK) break;
            const int P = kv.first.first, Q = kv.first.second;
            const std::vector<int> c0 = ring_width_candidates(Q), c1 = ring_width_candidates(P);
            int b0 = c0[0], b1 = c1[0];
            float best;
            st = time_class(pr, classes[kv.first], o, resident, {{kv.first, {b0, b1}}}, lds_cap, s, &best);
            auto try_widths = [&](int w0, int w1) {
                float ms;
                st = time_class(pr, classes[kv.first], o, resident, {{kv.first, {w0, w1}}}, lds_cap, s, &ms);
                if (st == COVEST_OK && ms < 0.97f * best) {
                    best = ms;
                    b0 = w0;
                    b1 = w1;
                }
            };
            for (size_t k = 1; k < c0.size() && st == COVEST_OK; ++k) try_widths(c0[k], b1);
            for (size_t k = 1; k < c1.size() && st == COVEST_OK; ++k) try_widths(b0, c1[k]);
            if (st == COVEST_OK && std::make_pair(b0, b1) != chosen[kv.first]) {
                Widths trial = chosen;
                trial[kv.first] = {b0, b1};
                float ms;
                st = time_class(pr, all, o, resident, trial, lds_cap, s, &ms);
                if (st == COVEST_OK && ms < 0.98f * whole) {
                    whole = ms;
                    chosen = trial;
                }
            }
            if (st == COVEST_OK) tune_store_locked(P, Q, chosen[kv.first].first, chosen[kv.first].second);
        }
        (void)hipStreamDestroy(s);
    }
    if (st != COVEST_OK) return st;
    for (auto &kv : chosen) (*out)[kv.first] = kv.second;
    return COVEST_OK;
}

int build_batched(covest_plan *plan, const covest_problem_ex *pr, int64_t count, const covest_opts &o,
                  hipStream_t stream)
{
    HIP_TRY(hipGetDevice(&plan->device));
    const int cus = cu_count(plan->device);
    const int resident = 2 * cus;
    HIP_TRY(prepare_rec_kernels());
    // engine per problem, as for a single call
    std::vector<int> engine(count);
    for (int64_t i = 0; i < count; ++i) {
        int e = pick_engine(pr[i].N, pr[i].M, pr[i].P, pr[i].Q, o, true);
        if (e == 0)
            return fail(COVEST_ERR_UNSUPPORTED, "problem %lld: the matrix-core engine does not fit %dx%d, %dx%d",
                        (long long)i, pr[i].N, pr[i].M, pr[i].P, pr[i].Q);
        if (e == 2 && (int64_t)pr[i].N * pr[i].lda + pr[i].M >= ((int64_t)1 << 31)) {
            if (o.engine == COVEST_ENGINE_MATRIX)
                return fail(COVEST_ERR_UNSUPPORTED, "problem %lld: the matrix-core engine needs N * lda < 2^31",
                            (long long)i);
            e = 1;
        }
        engine[i] = e;
    }
    std::map<std::pair<int, int>, std::pair<int, int>> widths;
    if (!o.ring_cols && !o.ring_rows) {
        int st = autotune(pr, count, engine, o, resident, &widths);
        if (st != COVEST_OK) return st;
    }
    auto wfor = [&](int P, int Q) {
        if (o.ring_cols || o.ring_rows) return std::make_pair(o.ring_cols, o.ring_rows);
        auto it = widths.find({P, Q});
        return it == widths.end() ? std::make_pair(0, 0) : it->second;
    };
    // first pass: cost of every problem with a coarse plan (vector engine:
    // wave-steps; matrix-core engine: 8-line k-group steps)
    std::vector<double> cost(count, 0.0);
    double total = 0.0;
    std::map<std::pair<int, int>, double> total_m;   // per matrix-core launch (mt x nt tiles)
    auto tiles = [&](int64_t i) { return std::make_pair((2 * pr[i].P - 1 + 15) / 16, (pr[i].Q + 15) / 16); };
    for (int64_t i = 0; i < count; ++i) {
        const auto w = wfor(pr[i].P, pr[i].Q);
        const ShapePlan sp = engine[i] == 2 ? make_mfma_plan(pr[i].N, pr[i].M, pr[i].P, pr[i].Q, 1)
                                            : make_shape_plan(pr[i].N, pr[i].M, pr[i].P, pr[i].Q, 1, w.first, w.second);
        for (double c : sp.job_cost) cost[i] += c;
        if (engine[i] == 2) total_m[tiles(i)] += cost[i];
        else total += cost[i];
    }
    // second pass: split each problem into jobs of about a third of a
    // resident slot's share (the matrix-core kernel holds one workgroup per
    // CU; each of its launches is balanced on its own)
    const double target = std::max(1.0, total / (3.0 * resident));
    std::vector<Job> jobs;
    std::vector<double> jcost;
    std::vector<LagGroup> groups;
    std::vector<Inst> insts(count);
    std::vector<FinItem> items[2][kFinVariants];   // [engine is matrix cores][variant]
    size_t ws_off = 0;
    std::vector<size_t> ws_base(count);
    std::vector<ShapePlan> plans(count);
    for (int64_t i = 0; i < count; ++i) {
        const auto w = wfor(pr[i].P, pr[i].Q);
        if (engine[i] == 2) {
            plans[i] = make_mfma_plan(pr[i].N, pr[i].M, pr[i].P, pr[i].Q, cus,
                                      std::max(1.0, total_m[tiles(i)] / (3.0 * cus)));
        } else {
            const int slots = (int)std::max<int64_t>(1, std::min<int64_t>(resident, std::llround(cost[i] / target)));
            plans[i] = make_shape_plan(pr[i].N, pr[i].M, pr[i].P, pr[i].Q, slots, w.first, w.second);
        }
        ws_base[i] = ws_off;
        ws_off += (plans[i].ws_bytes + 255) / 256 * 256;
    }
    HIP_TRY(hipMalloc(&plan->d_ws, std::max<size_t>(ws_off, 256)));
    struct MGroup {
        std::vector<MJob> jobs;
        std::vector<double> cost;
        size_t lds = 0;
    };
    std::map<std::pair<int, int>, MGroup> mgroups;   // (mt, nt) -> matrix-core jobs
    for (int64_t i = 0; i < count; ++i) {
        const ShapePlan &sp = plans[i];
        if (engine[i] == 2) {
            MGroup &mg = mgroups[{sp.mt, sp.nt}];
            for (size_t j = 0; j < sp.mjobs.size(); ++j) {
                MJob mj = sp.mjobs[j];
                mj.inst = (int)i;
                mg.jobs.push_back(mj);
                mg.cost.push_back(sp.job_cost[j]);
            }
            mg.lds = std::max(mg.lds, sp.lds_main);
            ++plan->n_matrix;
        }
        const int goff = (int)groups.size();
        groups.insert(groups.end(), sp.groups.begin(), sp.groups.end());
        for (size_t j = 0; j < sp.jobs.size(); ++j) {
            Job jb = sp.jobs[j];
            jb.inst = (int)i;
            jb.group += goff;
            jobs.push_back(jb);
            jcost.push_back(sp.job_cost[j]);
        }
        const int var = sp.fin_variant;
        for (FinItem it : sp.items) {
            it.inst = (int)i;
            items[engine[i] == 2][var].push_back(it);
        }
        if (engine[i] != 2) plan->lds_main = std::max(plan->lds_main, sp.lds_main);
        plan->lds_fin[var] = std::max(plan->lds_fin[var], sp.lds_fin);
        insts[i] = make_inst(sp, pr[i].A, pr[i].lda, pr[i].R, pr[i].ldr,
                             static_cast<char *>(plan->d_ws) + ws_base[i], o);
    }
    // longest job first (stable, so equal jobs keep their spatial order)
    std::vector<size_t> order(jobs.size());
    for (size_t j = 0; j < order.size(); ++j) order[j] = j;
    std::stable_sort(order.begin(), order.end(), [&](size_t a, size_t b) { return jcost[a] > jcost[b]; });
    std::vector<Job> sorted;
    sorted.reserve(jobs.size());
    for (size_t j : order) sorted.push_back(jobs[j]);
    plan->est_cost = total;
    plan->n_jobs = (int)sorted.size();
    for (int g = 0; g < 2; ++g)
        for (int v = 0; v < kFinVariants; ++v) plan->n_items[g][v] = (int)items[g][v].size();
    plan->grid = std::max(1, std::min(resident, plan->n_jobs));
    if (const int cap = worker_cap()) plan->grid = std::min(plan->grid, cap);
    HIP_TRY(upload(&plan->d_jobs, sorted));
    HIP_TRY(upload(&plan->d_groups, groups));
    HIP_TRY(upload(&plan->d_insts, insts));
    for (int g = 0; g < 2; ++g)
        for (int v = 0; v < kFinVariants; ++v) HIP_TRY(upload(&plan->d_items[g][v], items[g][v]));
    HIP_TRY(hipMalloc(&plan->d_counter, 256));
    for (auto &kv : mgroups) {
        // longest first: the hardware hands out workgroups in block order
        MGroup &mg = kv.second;
        std::vector<size_t> ord(mg.jobs.size());
        for (size_t j = 0; j < ord.size(); ++j) ord[j] = j;
        std::stable_sort(ord.begin(), ord.end(), [&](size_t a, size_t b) { return mg.cost[a] > mg.cost[b]; });
        std::vector<MJob> mjs;
        mjs.reserve(ord.size());
        for (size_t j : ord) mjs.push_back(mg.jobs[j]);
        covest_plan::MfmaLaunch l;
        l.mt = kv.first.first;
        l.nt = kv.first.second;
        l.n_jobs = (int)mjs.size();
        l.lds = mg.lds;
        plan->mfma.push_back(l);
        HIP_TRY(upload(&plan->mfma.back().d_jobs, mjs));
    }

    // capture: counter reset + persistent main kernel + finalize kernels
    hipStream_t cs = stream;
    if (cs == nullptr) {
        HIP_TRY(hipStreamCreateWithFlags(&plan->own_stream, hipStreamNonBlocking));
        cs = plan->own_stream;
    }
    // The vector kernel and the matrix-core launches touch disjoint problems:
    // they are two branches of the graph, joined before the finalize, so that
    // one fills the CUs the other's tail leaves idle.
    const bool branch = plan->n_jobs > 0 && !plan->mfma.empty();
    if (branch) {
        HIP_TRY(hipStreamCreateWithFlags(&plan->side_stream, hipStreamNonBlocking));
        HIP_TRY(hipEventCreateWithFlags(&plan->ev_fork, hipEventDisableTiming));
        HIP_TRY(hipEventCreateWithFlags(&plan->ev_join, hipEventDisableTiming));
    }
    HIP_TRY(hipStreamBeginCapture(cs, hipStreamCaptureModeThreadLocal));
    hipError_t e = hipSuccess;
    hipStream_t ms = cs;
    if (branch) {
        e = hipEventRecord(plan->ev_fork, cs);
        if (e == hipSuccess) e = hipStreamWaitEvent(plan->side_stream, plan->ev_fork, 0);
        ms = plan->side_stream;
    }
    if (e == hipSuccess && plan->n_jobs > 0) {
        MainArgs ma{};
        ma.jobs = plan->d_jobs;
        ma.groups = plan->d_groups;
        ma.insts = plan->d_insts;
        ma.n_jobs = plan->n_jobs;
        ma.use_inline = 0;
        e = launch_rec_persistent(ma, plan->d_counter, plan->grid, plan->lds_main, cs);
    }
    for (const auto &l : plan->mfma) {
        if (e != hipSuccess) break;
        MfmaArgs ma{};
        ma.jobs = l.d_jobs;
        ma.n_jobs = l.n_jobs;
        ma.xcd_remap = 0;
        ma.insts = plan->d_insts;
        e = launch_rec_mfma(ma, l.mt, l.nt, l.n_jobs, l.lds, ms);
    }
    // each engine's finalize follows its own main pass, on its own branch
    for (int g = 0; g < 2; ++g) {
        hipStream_t fs = g == 1 ? ms : cs;
        for (int v = 0; v < kFinVariants && e == hipSuccess; ++v) {
            if (plan->n_items[g][v] == 0) continue;
            FinArgs fa{};
            fa.items = plan->d_items[g][v];
            fa.insts = plan->d_insts;
            fa.n_items = plan->n_items[g][v];
            fa.use_inline = 0;
            e = launch_rec_finalize(fa, plan->n_items[g][v], plan->lds_fin[v], v, fs);
        }
    }
    if (branch && e == hipSuccess) {
        e = hipEventRecord(plan->ev_join, ms);
        if (e == hipSuccess) e = hipStreamWaitEvent(cs, plan->ev_join, 0);
    }
    hipGraph_t g = nullptr;
    const hipError_t e2 = hipStreamEndCapture(cs, &g);
    if (e != hipSuccess) {
        if (g) (void)hipGraphDestroy(g);
        return fail(COVEST_ERR_HIP, "batched launch capture failed: %s", hipGetErrorString(e));
    }
    if (e2 != hipSuccess) return fail(COVEST_ERR_HIP, "hipStreamEndCapture: %s", hipGetErrorString(e2));
    plan->graph = g;
    HIP_TRY(hipGraphInstantiate(&plan->exec, plan->graph, nullptr, nullptr, 0));
    return COVEST_OK;
}

// The checks and plan construction shared by the batched entry points.
int create_batched(covest_plan **out, const covest_problem_ex *problems, int64_t count, const covest_opts *opts,
                   hipStream_t stream)
{
    covest_opts o = resolve_opts(opts);
    int st = check_opts(o);
    if (st != COVEST_OK) return st;
    if (o.form == COVEST_FORM_HANKEL_MFMA)
        return fail(COVEST_ERR_UNSUPPORTED, "batched plans use the recurrence form");
    if (o.engine == COVEST_ENGINE_LANE)
        return fail(COVEST_ERR_UNSUPPORTED, "batched plans run on the vector or matrix engines; aperture plans "
                                            "take the lane engine");
    if (o.prec != COVEST_PREC_FP64 && o.prec != COVEST_PREC_FP32)
        return fail(COVEST_ERR_UNSUPPORTED, "batched plans compute in FP64 (prec FP64 or FP32 output)");
    for (int64_t i = 0; i < count; ++i) {
        const covest_problem_ex &p = problems[i];
        st = check_shape(p.N, p.M, p.P, p.Q);
        if (st != COVEST_OK) return fail(st, "problem %lld: %s", (long long)i, g_err.c_str());
        if (!p.A || !p.R) return fail(COVEST_ERR_INVALID_ARG, "problem %lld: null A or R", (long long)i);
        if (p.lda < p.M || p.ldr < (int64_t)p.P * p.Q)
            return fail(COVEST_ERR_INVALID_ARG, "problem %lld: lda %lld < M or ldr %lld < PQ", (long long)i,
                        (long long)p.lda, (long long)p.ldr);
        if (p.P > kMaxWindow || p.Q > kMaxWindow)
            return fail(COVEST_ERR_UNSUPPORTED, "problem %lld: P, Q <= %d", (long long)i, kMaxWindow);
    }
    covest_plan *plan = new covest_plan();
    plan->opts = o;
    plan->count = count;
    st = build_batched(plan, problems, count, o, stream);
    if (st != COVEST_OK) {
        const std::string msg = g_err;
        free_plan(plan);
        return fail(st, "%s", msg.c_str());
    }
    *out = plan;
    return ok();
}

}  // namespace

// =================================================================== ABI ====
extern "C" {

int covest_version(void) { return COVEST_VERSION; }

const char *covest_last_error(void) { return g_err.c_str(); }

int covest_counts(int64_t N, int64_t M, int64_t P, int64_t Q, covest_counts_t *out)
{
    if (!out) return fail(COVEST_ERR_INVALID_ARG, "out is null");
    int st = check_shape(N, M, P, Q);
    if (st != COVEST_OK) return st;
    const Counts c = method_counts(N, M, P, Q);
    out->K = c.K;
    out->n_uc = c.n_uc;
    out->um = c.um;
    out->eta = c.eta;
    out->segments = c.segments;
    return ok();
}

int covest_workspace_size(int64_t N, int64_t M, int64_t P, int64_t Q, const covest_opts *opts,
                          size_t *bytes)
{
    if (!bytes) return fail(COVEST_ERR_INVALID_ARG, "bytes is null");
    const covest_opts o = resolve_opts(opts);
    int st = check_opts(o);
    if (st != COVEST_OK) return st;
    st = check_shape(N, M, P, Q);
    if (st != COVEST_OK) return st;
    if (use_recurrence(o)) {
        if (o.engine == COVEST_ENGINE_LANE) {
            st = lane_check((int)N, (int)M, (int)P, (int)Q, o);
            if (st != COVEST_OK) return st;
            *bytes = 0;
            return ok();
        }
        if (P > kMaxWindow || Q > kMaxWindow)
            return fail(COVEST_ERR_UNSUPPORTED, "the recurrence form supports P, Q <= %d", kMaxWindow);
        const int engine = pick_engine((int)N, (int)M, (int)P, (int)Q, o);
        if (engine == 0)
            return fail(COVEST_ERR_UNSUPPORTED, "the matrix-core engine cannot run this shape");
        *bytes = host_plan((int)N, (int)M, (int)P, (int)Q, o.ring_cols, o.ring_rows, engine)->ws_bytes;
        // AUTO falls back to the vector engine for inputs too large for
        // 32-bit offsets: cover both plans
        if (engine == 2 && o.engine == COVEST_ENGINE_AUTO)
            *bytes = std::max(*bytes, host_plan((int)N, (int)M, (int)P, (int)Q, 0, 0, 1)->ws_bytes);
        return ok();
    }
    const int prec = hankel_prec(o.prec);
    if (prec < 0) return fail(COVEST_ERR_UNSUPPORTED, "the matrix-core form has no FP64 precision");
    if (P > kMaxWindow || Q > kMaxWindow)
        return fail(COVEST_ERR_UNSUPPORTED, "the matrix-core form supports P, Q <= %d", kMaxWindow);
    *bytes = host_hankel_plan((int)N, (int)M, (int)P, (int)Q, prec)->ws_bytes;
    return ok();
}

int covest_forward_ex(const void *A, int64_t lda, int64_t N, int64_t M, int64_t P, int64_t Q, void *R,
                      int64_t ldr, const covest_opts *opts, void *ws, size_t ws_bytes,
                      hipStream_t stream)
{
    const covest_opts o = resolve_opts(opts);
    int st = check_opts(o);
    if (st != COVEST_OK) return st;
    st = check_shape(N, M, P, Q);
    if (st != COVEST_OK) return st;
    if (!A || !R) return fail(COVEST_ERR_INVALID_ARG, "A and R must be non-null device pointers");
    if (lda < M) return fail(COVEST_ERR_INVALID_ARG, "lda (%lld) < M (%lld)", (long long)lda, (long long)M);
    if (ldr < P * Q) return fail(COVEST_ERR_INVALID_ARG, "ldr (%lld) < PQ (%lld)", (long long)ldr, (long long)(P * Q));
    if (use_recurrence(o) && o.engine == COVEST_ENGINE_LANE)
        return lane_forward(A, lda, (int)N, (int)M, (int)P, (int)Q, R, ldr, o, stream);
    if (use_recurrence(o))
        return rec_forward(A, lda, (int)N, (int)M, (int)P, (int)Q, R, ldr, o, ws, ws_bytes, stream);
    return hankel_forward(A, lda, (int)N, (int)M, (int)P, (int)Q, R, ldr, o, ws, ws_bytes, stream);
}

int covest_forward(const void *A, int64_t N, int64_t M, int64_t P, int64_t Q, void *R,
                   const covest_opts *opts, void *ws, size_t ws_bytes, hipStream_t stream)
{
    return covest_forward_ex(A, M, N, M, P, Q, R, P * Q, opts, ws, ws_bytes, stream);
}

int covest_forward_noalloc(const void *A, int64_t lda, int64_t N, int64_t M, int64_t P, int64_t Q, void *R,
                           int64_t ldr, const covest_opts *opts, hipStream_t stream)
{
    const covest_opts o = resolve_opts(opts);
    int st = check_opts(o);
    if (st != COVEST_OK) return st;
    st = check_shape(N, M, P, Q);
    if (st != COVEST_OK) return st;
    if (!A || !R) return fail(COVEST_ERR_INVALID_ARG, "A and R must be non-null device pointers");
    if (lda < M) return fail(COVEST_ERR_INVALID_ARG, "lda (%lld) < M (%lld)", (long long)lda, (long long)M);
    if (ldr < P * Q) return fail(COVEST_ERR_INVALID_ARG, "ldr (%lld) < PQ (%lld)", (long long)ldr, (long long)(P * Q));
    if (!use_recurrence(o))
        return fail(COVEST_ERR_UNSUPPORTED, "the no-allocation entry point runs the recurrence form only");
    if (o.engine == COVEST_ENGINE_LANE)   // allocates nothing and uses no scratch
        return lane_forward(A, lda, (int)N, (int)M, (int)P, (int)Q, R, ldr, o, stream);
    return rec_forward_noalloc(A, lda, (int)N, (int)M, (int)P, (int)Q, R, ldr, o, stream);
}

int covest_backward_workspace_size(int64_t N, int64_t M, int64_t P, int64_t Q,
                                   const covest_opts *opts, size_t *bytes)
{
    if (!bytes) return fail(COVEST_ERR_INVALID_ARG, "bytes is null");
    const covest_opts o = resolve_opts(opts);
    int st = check_opts(o);
    if (st != COVEST_OK) return st;
    st = check_shape(N, M, P, Q);
    if (st != COVEST_OK) return st;
    if (P > kMaxWindow || Q > kMaxWindow)
        return fail(COVEST_ERR_UNSUPPORTED, "the adjoint supports P, Q <= %d", kMaxWindow);
    *bytes = adj_geometry((int)N, (int)M, (int)P, (int)Q).ws_bytes;
    return ok();
}

int covest_backward_ex(const void *A, int64_t lda, const void *dR, int64_t ldr, void *dA, int64_t ldda,
                       int64_t N, int64_t M, int64_t P, int64_t Q, const covest_opts *opts, void *ws,
                       size_t ws_bytes, hipStream_t stream)
{
    const covest_opts o = resolve_opts(opts);
    int st = check_opts(o);
    if (st != COVEST_OK) return st;
    st = check_shape(N, M, P, Q);
    if (st != COVEST_OK) return st;
    if (!A || !dR || !dA) return fail(COVEST_ERR_INVALID_ARG, "A, dR and dA must be non-null device pointers");
    if (lda < M || ldda < M)
        return fail(COVEST_ERR_INVALID_ARG, "lda (%lld) and ldda (%lld) must be >= M (%lld)", (long long)lda,
                    (long long)ldda, (long long)M);
    if (ldr < P * Q)
        return fail(COVEST_ERR_INVALID_ARG, "ldr (%lld) < PQ (%lld)", (long long)ldr, (long long)(P * Q));
    // element types: those of R under the same options (complex128 for FP64)
    const bool fp64 = o.prec == COVEST_PREC_FP64;
    const size_t ge = fp64 ? 16 : 8;
    auto span = [](const void *p, int64_t rows, int64_t ld, int64_t cols, size_t es) {
        const char *b = static_cast<const char *>(p);
        return std::make_pair(b, b + ((rows - 1) * ld + cols) * (int64_t)es);
    };
    auto overlap = [](std::pair<const char *, const char *> x, std::pair<const char *, const char *> y) {
        return x.first < y.second && y.first < x.second;
    };
    const auto sA = span(A, N, lda, M, 8), sG = span(dR, P * Q, ldr, P * Q, ge), sD = span(dA, N, ldda, M, ge);
    if (overlap(sD, sA) || overlap(sD, sG)) return fail(COVEST_ERR_INVALID_ARG, "dA must not overlap A or dR");
    if (P > kMaxWindow || Q > kMaxWindow)
        return fail(COVEST_ERR_UNSUPPORTED, "the adjoint supports P, Q <= %d", kMaxWindow);
    const AdjGeom g = adj_geometry((int)N, (int)M, (int)P, (int)Q);
    if (ws_bytes < g.ws_bytes || ws == nullptr)
        return fail(COVEST_ERR_WORKSPACE, "workspace of %zu bytes needed, %zu given", g.ws_bytes, ws_bytes);
    if (g.frame_jobs > INT32_MAX)
        return fail(COVEST_ERR_UNSUPPORTED, "the adjoint's border needs %lld jobs, more than one launch holds",
                    (long long)g.frame_jobs);
    AdjArgs aa{};
    aa.A = static_cast<const float2 *>(A);
    aa.lda = lda;
    aa.G = dR;
    aa.ldg = ldr;
    aa.dA = dA;
    aa.ldda = ldda;
    aa.g_fp64 = fp64 ? 1 : 0;
    aa.upper = o.fill == COVEST_FILL_UPPER ? 1 : 0;
    aa.N = (int)N;
    aa.M = (int)M;
    aa.P = (int)P;
    aa.Q = (int)Q;
    aa.Kr = (int)(N - P + 1);
    aa.Kc = (int)(M - Q + 1);
    aa.ir0 = g.ir0;
    aa.ir1 = g.ir1;
    aa.ic0 = g.ic0;
    aa.ic1 = g.ic1;
    aa.ndc = g.ndc;
    char *wsb = static_cast<char *>(ws);
    aa.tables = reinterpret_cast<double *>(wsb + g.off_tables);
    aa.hfull = reinterpret_cast<double *>(wsb + g.off_hfull);
    aa.wrows = reinterpret_cast<double *>(wsb + g.off_wrows);
    aa.wcols = reinterpret_cast<double *>(wsb + g.off_wcols);
    aa.normalize = o.normalize ? 1 : 0;
    if (g.mfma) {
        aa.ny = g.ny;
        aa.nx = g.nx;
        aa.mtiles = g.mtiles;
        aa.mranges = g.mranges;
        aa.bnd = reinterpret_cast<double *>(wsb + g.off_bnd);
        HIP_TRY(timed("adjoint", stream, [&] {
            return launch_adjoint_mfma(aa, g.n_lags, g.lds_tables, g.frame_jobs, g.lds_frame, stream);
        }));
        return finish_call(stream);
    }
    HIP_TRY(timed("adjoint", stream, [&] {
        return launch_adjoint(aa, g.n_lags, g.lds_tables, g.interior_blocks, g.lds_interior, g.frame_jobs, stream);
    }));
    return finish_call(stream);
}

int covest_backward(const void *A, const void *dR, void *dA, int64_t N, int64_t M, int64_t P, int64_t Q,
                    const covest_opts *opts, void *ws, size_t ws_bytes, hipStream_t stream)
{
    return covest_backward_ex(A, M, dR, P * Q, dA, M, N, M, P, Q, opts, ws, ws_bytes, stream);
}

int covest_plan_batched_create(covest_plan **out, const covest_problem *problems, int64_t count,
                               const covest_opts *opts, hipStream_t stream)
{
    if (!out || !problems || count < 1) return fail(COVEST_ERR_INVALID_ARG, "need out, problems and count >= 1");
    *out = nullptr;
    std::vector<covest_problem_ex> ex((size_t)count);
    for (int64_t i = 0; i < count; ++i) {
        const covest_problem &p = problems[i];
        ex[i] = covest_problem_ex{p.A, p.R, (int64_t)p.M, (int64_t)p.P * p.Q, p.N, p.M, p.P, p.Q};
    }
    return create_batched(out, ex.data(), count, opts, stream);
}

int covest_plan_batched_create_ex(covest_plan **out, const covest_problem_ex *problems, int64_t count,
                                  const covest_opts *opts, hipStream_t stream)
{
    if (!out || !problems || count < 1) return fail(COVEST_ERR_INVALID_ARG, "need out, problems and count >= 1");
    *out = nullptr;
    return create_batched(out, problems, count, opts, stream);
}

int covest_plan_apertures_create(covest_plan **out, const covest_aperture_grid *grid, int64_t P, int64_t Q,
                                 void *R, const covest_opts *opts, hipStream_t stream)
{
    if (!out || !grid || !grid->image || !R) return fail(COVEST_ERR_INVALID_ARG, "need out, grid, image and R");
    *out = nullptr;
    const covest_aperture_grid &g = *grid;
    if (g.H < 1 || g.W < 1 || g.ld < g.W)
        return fail(COVEST_ERR_INVALID_ARG, "image %lld x %lld with ld %lld", (long long)g.H, (long long)g.W,
                    (long long)g.ld);
    if (g.n_rows < 1 || g.n_cols < 1 || g.row_step < 1 || g.col_step < 1)
        return fail(COVEST_ERR_INVALID_ARG, "aperture counts and steps must be >= 1");
    if (g.ap_rows < 1 || g.ap_cols < 1 || g.ap_rows > g.H || g.ap_cols > g.W ||
        g.n_rows - 1 > (g.H - g.ap_rows) / g.row_step || g.n_cols - 1 > (g.W - g.ap_cols) / g.col_step)
        return fail(COVEST_ERR_SHAPE, "%lld x %lld apertures of %lld x %lld at steps %lld, %lld leave the %lld x %lld image",
                    (long long)g.n_rows, (long long)g.n_cols, (long long)g.ap_rows, (long long)g.ap_cols,
                    (long long)g.row_step, (long long)g.col_step, (long long)g.H, (long long)g.W);
    if (g.n_rows > INT32_MAX / g.n_cols) return fail(COVEST_ERR_SHAPE, "more than 2^31 - 1 apertures");
    int st = check_shape(g.ap_rows, g.ap_cols, P, Q);
    if (st != COVEST_OK) return st;
    if (P > kMaxWindow || Q > kMaxWindow)
        return fail(COVEST_ERR_UNSUPPORTED, "the recurrence form supports P, Q <= %d", kMaxWindow);
    const covest_opts o = resolve_opts(opts);
    st = check_opts(o);
    if (st != COVEST_OK) return st;
    const size_t esz = o.prec == COVEST_PREC_FP64 ? 16 : 8;
    const int64_t pq = P * Q, count = g.n_rows * g.n_cols;
    if (use_recurrence(o) && o.engine == COVEST_ENGINE_LANE) {
        st = lane_check((int)g.ap_rows, (int)g.ap_cols, (int)P, (int)Q, o);
        if (st != COVEST_OK) return st;
    }
    const bool lane_ok = use_recurrence(o) && (o.prec == COVEST_PREC_FP64 || o.prec == COVEST_PREC_FP32) &&
                         lane_fits((int)g.ap_rows, (int)g.ap_cols, (int)P, (int)Q);
    if (lane_ok && (o.engine == COVEST_ENGINE_LANE || o.engine == COVEST_ENGINE_AUTO)) {
        int dev = 0;
        HIP_TRY(hipGetDevice(&dev));
        const int cus = cus_of_device(dev);
        const bool lane = o.engine == COVEST_ENGINE_LANE || (count >= cus && o.ring_cols == 0 && o.ring_rows == 0);
        if (lane) {
            const int chain = lane_chain((int)g.ap_rows, (int)P, g.row_step, g.n_rows, g.n_cols, cus, true);
            covest_plan *plan = new covest_plan();
            plan->device = dev;
            plan->opts = o;
            plan->count = count;
            plan->lane = true;
            plan->lane_args = make_lane_args(g.image, g.ld, (int)g.ap_rows, (int)g.ap_cols, (int)P, (int)Q,
                                             g.row_step, g.col_step, g.n_rows, g.n_cols, chain, R, pq, pq * pq, o);
            const hipError_t e = prepare_lane_kernels();
            if (e != hipSuccess) {
                free_plan(plan);
                return fail(COVEST_ERR_HIP, "lane kernels: %s", hipGetErrorString(e));
            }
            *out = plan;
            return ok();
        }
    }
    std::vector<covest_problem_ex> ex((size_t)count);
    for (int64_t a = 0; a < g.n_rows; ++a)
        for (int64_t b = 0; b < g.n_cols; ++b) {
            const int64_t i = a * g.n_cols + b;
            ex[i].A = static_cast<const char *>(g.image) + 8 * (a * g.row_step * g.ld + b * g.col_step);
            ex[i].R = static_cast<char *>(R) + esz * (size_t)(i * pq * pq);
            ex[i].lda = g.ld;
            ex[i].ldr = pq;
            ex[i].N = (int32_t)g.ap_rows;
            ex[i].M = (int32_t)g.ap_cols;
            ex[i].P = (int32_t)P;
            ex[i].Q = (int32_t)Q;
        }
    return create_batched(out, ex.data(), count, opts, stream);
}

int covest_capon_workspace_size(int64_t count, int64_t P, int64_t Q, int64_t F1, size_t *bytes)
{
    if (!bytes) return fail(COVEST_ERR_INVALID_ARG, "bytes is null");
    if (count < 0 || P < 1 || Q < 1 || F1 < 1 || F1 > kCaponMaxGrid)
        return fail(COVEST_ERR_SHAPE, "need count >= 0, P, Q >= 1 and 1 <= F1 <= %d", kCaponMaxGrid);
    if (P * Q > kCaponMaxPQ) return fail(COVEST_ERR_UNSUPPORTED, "the spectrum supports PQ <= %d", kCaponMaxPQ);
    *bytes = (size_t)count * capon_ws_per_matrix((int)(P * Q), (int)Q, (int)F1);
    return ok();
}

int covest_capon_spectrum(const void *R, int64_t count, int64_t P, int64_t Q, int64_t F1, int64_t F2, double *S,
                          void *ws, size_t ws_bytes, hipStream_t stream)
{
    if (count < 0 || P < 1 || Q < 1 || F1 < 1 || F2 < 1 || F1 > kCaponMaxGrid || F2 > kCaponMaxGrid)
        return fail(COVEST_ERR_SHAPE, "need count >= 0, P, Q >= 1 and 1 <= F1, F2 <= %d", kCaponMaxGrid);
    if (P * Q > kCaponMaxPQ) return fail(COVEST_ERR_UNSUPPORTED, "the spectrum supports PQ <= %d", kCaponMaxPQ);
    if (count > INT32_MAX) return fail(COVEST_ERR_SHAPE, "count must be below 2^31");
    if (count == 0) return ok();
    if (!R || !S || !ws) return fail(COVEST_ERR_INVALID_ARG, "need R, S and ws");
    const int n = (int)(P * Q);
    const size_t per = capon_ws_per_matrix(n, (int)Q, (int)F1);
    if (ws_bytes < (size_t)count * per)
        return fail(COVEST_ERR_WORKSPACE, "workspace %zu bytes < %zu", ws_bytes, (size_t)count * per);
    CaponArgs ca{};
    ca.R = static_cast<const double2 *>(R);
    ca.S = S;
    ca.T = static_cast<double2 *>(ws);
    ca.F = reinterpret_cast<double2 *>(static_cast<char *>(ws) + (size_t)count * capon_t_bytes((int)Q, (int)F1));
    ca.n = n;
    ca.P = (int)P;
    ca.Q = (int)Q;
    ca.F1 = (int)F1;
    ca.F2 = (int)F2;
    HIP_TRY(timed("capon", stream, [&] { return launch_capon(ca, (int)count, stream); }));
    return finish_call(stream);
}

int covest_forward_batched(covest_plan *plan, hipStream_t stream)
{
    if (!plan || (!plan->exec && !plan->lane)) return fail(COVEST_ERR_INVALID_ARG, "invalid plan");
    int dev = -1;
    HIP_TRY(hipGetDevice(&dev));
    if (dev != plan->device)
        return fail(COVEST_ERR_PLAN_MISMATCH, "plan was built on device %d, current device is %d", plan->device, dev);
    if (plan->lane) return lane_run(plan->lane_args, stream);
    HIP_TRY(timed("batched_graph", stream, [&] { return hipGraphLaunch(plan->exec, stream); }));
    return finish_call(stream);
}

int covest_plan_destroy(covest_plan *plan)
{
    free_plan(plan);
    return ok();
}

static bool width_ok(int32_t w) { return w == 0 || w == 4 || w == 8 || w == 12 || w == 16; }

int covest_plan_info_get(int64_t N, int64_t M, int64_t P, int64_t Q, int32_t n_slots, int32_t w0,
                         int32_t w1, covest_plan_info *out)
{
    if (!out) return fail(COVEST_ERR_INVALID_ARG, "out is null");
    if (!width_ok(w0) || !width_ok(w1)) return fail(COVEST_ERR_INVALID_ARG, "ring widths are 0, 4, 8, 12 or 16");
    int st = check_shape(N, M, P, Q);
    if (st != COVEST_OK) return st;
    if (P > kMaxWindow || Q > kMaxWindow)
        return fail(COVEST_ERR_UNSUPPORTED, "the recurrence form supports P, Q <= %d", kMaxWindow);
    const ShapePlan sp = make_shape_plan((int)N, (int)M, (int)P, (int)Q, n_slots > 0 ? n_slots : 512, w0, w1);
    std::memset(out, 0, sizeof(*out));
    out->W0 = sp.W0;
    out->W1 = sp.W1;
    out->Rm0 = sp.Rm0;
    out->Rm1 = sp.Rm1;
    out->Cm0 = sp.Cm0;
    out->Cm1 = sp.Cm1;
    out->n_ir = sp.n_ir;
    out->n_ic = sp.n_ic;
    out->lag_stride = sp.lag_stride;
    out->bandw = sp.bandw;
    out->n_bulk = sp.n_bulk;
    out->n_jobs = (int32_t)sp.jobs.size();
    out->n_groups = (int32_t)sp.groups.size();
    out->n_items = (int32_t)sp.items.size();
    out->ws_bytes = (int64_t)sp.ws_bytes;
    out->lds_main = (int64_t)sp.lds_main;
    out->lds_fin = (int64_t)sp.lds_fin;
    out->main_products = sp.main_products;
    out->fin_products = sp.fin_products;
    return ok();
}

int covest_plan_tables(int64_t N, int64_t M, int64_t P, int64_t Q, int32_t n_slots, int32_t w0, int32_t w1,
                       int32_t *jobs, int32_t *groups, int32_t *items)
{
    if (!width_ok(w0) || !width_ok(w1)) return fail(COVEST_ERR_INVALID_ARG, "ring widths are 0, 4, 8, 12 or 16");
    int st = check_shape(N, M, P, Q);
    if (st != COVEST_OK) return st;
    if (P > kMaxWindow || Q > kMaxWindow)
        return fail(COVEST_ERR_UNSUPPORTED, "the recurrence form supports P, Q <= %d", kMaxWindow);
    const ShapePlan sp = make_shape_plan((int)N, (int)M, (int)P, (int)Q, n_slots > 0 ? n_slots : 512, w0, w1);
    if (jobs) {
        for (size_t k = 0; k < sp.jobs.size(); ++k) {
            const Job &j = sp.jobs[k];
            const int32_t row[12] = {j.mode, j.inst, j.group, j.out, j.u0, j.u1,
                                     j.x0, j.x1, j.c0, j.c1, j.tile_rows, j.tile_cols};
            std::memcpy(jobs + 12 * k, row, sizeof(row));
        }
    }
    if (groups) {
        for (size_t k = 0; k < sp.groups.size(); ++k) {
            const LagGroup &g = sp.groups[k];
            const int32_t row[14] = {g.orient, g.W, g.d1lo, g.d1hi, g.ch0, g.nch, g.v2lo, g.v2hi,
                                     g.lanes, g.slots, g.hr_lo, g.hr_hi, g.hc_lo, g.hc_hi};
            std::memcpy(groups + 14 * k, row, sizeof(row));
        }
    }
    if (items) {
        for (size_t k = 0; k < sp.items.size(); ++k) {
            const FinItem &it = sp.items[k];
            const int32_t row[5] = {it.inst, it.dr, it.dc, it.bulk0, it.bulk1};
            std::memcpy(items + 5 * k, row, sizeof(row));
        }
    }
    return ok();
}

int covest_timing_enable(int on)
{
    std::lock_guard<std::mutex> lk(g_tmu);
    g_timing = on != 0;
    return ok();
}

int covest_timing_reset(void)
{
    std::lock_guard<std::mutex> lk(g_tmu);
    for (Pending &p : g_pending) {
        (void)hipEventDestroy(p.a);
        (void)hipEventDestroy(p.b);
    }
    g_pending.clear();
    g_totals.clear();
    return ok();
}

int covest_timing_read(covest_timing_record *out, int cap)
{
    std::lock_guard<std::mutex> lk(g_tmu);
    for (Pending &p : g_pending) {
        hipError_t e = hipEventSynchronize(p.b);
        if (e != hipSuccess) return fail(COVEST_ERR_HIP, "hipEventSynchronize: %s", hipGetErrorString(e));
        float ms = 0.f;
        (void)hipEventElapsedTime(&ms, p.a, p.b);
        auto &t = g_totals[p.name];
        t.first += 1;
        t.second += ms;
        (void)hipEventDestroy(p.a);
        (void)hipEventDestroy(p.b);
    }
    g_pending.clear();
    int n = 0;
    for (auto &kv : g_totals) {
        if (out && n < cap) {
            std::memset(&out[n], 0, sizeof(out[n]));
            std::snprintf(out[n].name, sizeof(out[n].name), "%s", kv.first.c_str());
            out[n].launches = kv.second.first;
            out[n].total_ms = kv.second.second;
        }
        ++n;
    }
    g_err.clear();
    return n;
}

}  // extern "C"

extern "C" int covest_forward_stamped(const void *A, int64_t N, int64_t M, int64_t P, int64_t Q, void *R,
                                     const covest_opts *opts, void *ws, size_t ws_bytes, uint64_t *stamps,
                                     int64_t n_stamps, int32_t *items, hipStream_t stream)
{
    const covest_opts o = resolve_opts(opts);
    int st = check_opts(o);
    if (st != COVEST_OK) return st;
    st = check_shape(N, M, P, Q);
    if (st != COVEST_OK) return st;
    if (!A || !R || !stamps) return fail(COVEST_ERR_INVALID_ARG, "A, R and stamps must be non-null device pointers");
    if (!use_recurrence(o)) return fail(COVEST_ERR_UNSUPPORTED, "stamps are taken for the recurrence form only");
    st = rec_forward(A, M, (int)N, (int)M, (int)P, (int)Q, R, P * Q, o, ws, ws_bytes, stream,
                     reinterpret_cast<unsigned long long *>(stamps), n_stamps);
    if (st != COVEST_OK || !items) return st;
    // the items in stamp order (host copy of the finalize table of the plan just used)
    int engine = 0;
    st = rec_engine((int)N, (int)M, (int)P, (int)Q, M, o, &engine);
    if (st != COVEST_OK) return st;
    const auto sp = host_plan((int)N, (int)M, (int)P, (int)Q, o.ring_cols, o.ring_rows, engine);
    for (size_t i = 0; i < sp->items.size(); ++i) {
        const FinItem &x = sp->items[i];
        const int32_t row[5] = {x.inst, x.dr, x.dc, x.bulk0, x.bulk1};
        std::memcpy(items + 5 * i, row, sizeof(row));
    }
    return ok();
}

extern "C" int covest_hankel_plan_get(int64_t N, int64_t M, int64_t P, int64_t Q, int32_t prec, int32_t n_cu,
                                      covest_hankel_plan_info *out, int32_t *items, int32_t *tiles,
                                      int32_t *item_index)
{
    if (!out) return fail(COVEST_ERR_INVALID_ARG, "out is null");
    int st = check_shape(N, M, P, Q);
    if (st != COVEST_OK) return st;
    if (P > kMaxWindow || Q > kMaxWindow)
        return fail(COVEST_ERR_UNSUPPORTED, "the matrix-core form supports P, Q <= %d", kMaxWindow);
    if (prec < COVEST_PREC_FP64 || prec > COVEST_PREC_FP16) return fail(COVEST_ERR_INVALID_ARG, "unknown precision");
    const int hp_prec = hankel_prec((covest_precision)prec);
    if (hp_prec < 0 || hp_prec == kPrecF32)
        return fail(COVEST_ERR_UNSUPPORTED, "the 16-bit plan covers BF16X3, FP16X3, BF16 and FP16");
    const HankelPlan hp = make_hankel_plan((int)N, (int)M, (int)P, (int)Q, hp_prec, n_cu > 0 ? n_cu : 256);
    out->pb = hp.pb;
    out->qb = hp.qb;
    out->stride_a = hp.stride_a;
    out->stride_b = hp.stride_b;
    out->tm = hp.tm;
    out->tn = hp.tn;
    out->npl = hp.npl16;
    out->ldp = hp.ldp;
    out->n_items = (int32_t)hp.items.size();
    out->n_tiles = (int32_t)hp.tiles.size();
    out->n_index = (int32_t)hp.item_index.size();
    out->lds = (int64_t)hp.lds;
    out->ws_bytes = (int64_t)hp.ws_bytes;
    out->planes_bytes = (int64_t)hp.planes_bytes;
    if (items)
        for (size_t i = 0; i < hp.items.size(); ++i) {
            const HItem &x = hp.items[i];
            const int32_t row[6] = {x.tr, x.tc, x.p0, x.p1, x.q0, x.q1};
            std::memcpy(items + 6 * i, row, sizeof(row));
        }
    if (tiles)
        for (size_t t = 0; t < hp.tiles.size(); ++t) {
            const HTile &x = hp.tiles[t];
            const int32_t row[4] = {x.tr, x.tc, x.item0, x.item1};
            std::memcpy(tiles + 4 * t, row, sizeof(row));
        }
    if (item_index) std::memcpy(item_index, hp.item_index.data(), hp.item_index.size() * sizeof(int32_t));
    return ok();
}

extern "C" int covest_lane_plan_get(int64_t N, int64_t M, int64_t P, int64_t Q, int64_t row_step, int64_t n_rows,
                                    int64_t n_cols, int32_t n_cu, covest_lane_plan_info *out)
{
    if (!out) return fail(COVEST_ERR_INVALID_ARG, "out is null");
    int st = check_shape(N, M, P, Q);
    if (st != COVEST_OK) return st;
    if (row_step < 1 || n_rows < 1 || n_cols < 1 || n_rows > INT32_MAX / n_cols)
        return fail(COVEST_ERR_SHAPE, "need row_step, n_rows, n_cols >= 1 and fewer than 2^31 inputs");
    std::memset(out, 0, sizeof(*out));
    out->fits = lane_fits((int)N, (int)M, (int)P, (int)Q) ? 1 : 0;
    out->qmax = lane_qmax((int)Q);
    out->ring = lane_ring((int)P);
    out->gstride = lane_gstride((int)M, (int)Q);
    out->chunk = kLaneChunk;
    out->chain = lane_chain((int)N, (int)P, row_step, n_rows, n_cols, n_cu > 0 ? n_cu : 256, false);
    out->n_blocks = (int32_t)(n_cols * ((n_rows + out->chain - 1) / out->chain));
    out->threads = (lane_n_lags((int)P, (int)Q) + 63) / 64 * 64;
    out->lds = (int64_t)lane_lds_bytes((int)M, (int)P, (int)Q);
    return ok();
}

extern "C" int covest_engine_choice(int64_t N, int64_t M, int64_t P, int64_t Q, int32_t batch, int32_t *engine,
                                    int32_t *fits)
{
    if (!engine || !fits) return fail(COVEST_ERR_INVALID_ARG, "engine and fits must be non-null");
    int st = check_shape(N, M, P, Q);
    if (st != COVEST_OK) return st;
    if (P > kMaxWindow || Q > kMaxWindow)
        return fail(COVEST_ERR_UNSUPPORTED, "the recurrence form supports P, Q <= %d", kMaxWindow);
    *fits = mfma_fits((int)N, (int)M, (int)P, (int)Q) ? 1 : 0;
    *engine = mfma_preferred((int)N, (int)M, (int)P, (int)Q, batch != 0) ? COVEST_ENGINE_MATRIX
                                                                         : COVEST_ENGINE_VECTOR;
    return ok();
}

extern "C" int covest_mfma_plan_get(int64_t N, int64_t M, int64_t P, int64_t Q, int32_t n_cu,
                                    covest_mfma_plan_info *out, int32_t *jobs, int32_t *items)
{
    try {
        if (!out) return fail(COVEST_ERR_INVALID_ARG, "out is null");
        int st = check_shape(N, M, P, Q);
        if (st != COVEST_OK) return st;
        if (P > kMaxWindow || Q > kMaxWindow || !mfma_fits((int)N, (int)M, (int)P, (int)Q))
            return fail(COVEST_ERR_UNSUPPORTED, "the matrix-core engine cannot run this shape");
        const ShapePlan sp = make_mfma_plan((int)N, (int)M, (int)P, (int)Q, n_cu > 0 ? n_cu : 256);
        std::memset(out, 0, sizeof(*out));
        out->mt = sp.mt;
        out->nt = sp.nt;
        out->Rm0 = sp.Rm0;
        out->Rm1 = sp.Rm1;
        out->Cm0 = sp.Cm0;
        out->Cm1 = sp.Cm1;
        out->n_ir = sp.n_ir;
        out->n_ic = sp.n_ic;
        out->lag_stride = sp.lag_stride;
        out->n_bulk = sp.n_bulk;
        out->n_jobs = (int32_t)sp.mjobs.size();
        out->n_items = (int32_t)sp.items.size();
        out->zpieces = sp.zpieces;
        out->ws_bytes = (int64_t)sp.ws_bytes;
        out->lds_main = (int64_t)sp.lds_main;
        out->lds_fin = (int64_t)sp.lds_fin;
        out->main_products = sp.main_products;
        out->fin_products = sp.fin_products;
        if (jobs) {
            for (size_t k = 0; k < sp.mjobs.size(); ++k) {
                const MJob &j = sp.mjobs[k];
                const int32_t row[16] = {j.inst, j.orient, j.kind, j.out, j.line0, j.line_end, j.b0, j.kg0,
                                         j.b1, j.kg1, j.n_kg, j.pos_lo, j.pos_hi, j.k0, j.kin, 0};
                std::memcpy(jobs + 16 * k, row, sizeof(row));
            }
        }
        if (items) {
            for (size_t k = 0; k < sp.items.size(); ++k) {
                const FinItem &it = sp.items[k];
                const int32_t row[5] = {it.inst, it.dr, it.dc, it.bulk0, it.bulk1};
                std::memcpy(items + 5 * k, row, sizeof(row));
            }
        }
        return ok();
    } catch (const std::exception &e) {
        return fail(COVEST_ERR_INVALID_ARG, "%s", e.what());
    }
}
