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
#include <map>
#include <memory>
#include <mutex>
#include <string>
#include <tuple>
#include <vector>

#include "covest.h"
#include "covest_plan.h"
#include "adj_internal.hpp"
#include "launch.hpp"
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
    int xcd_remap = 0;
};

std::mutex g_pmu;
std::map<std::tuple<int, int, int, int, int>, std::unique_ptr<DevPlan>> g_plans;

int n_slots_for_device(int dev)
{
    int cus = 0;
    if (hipDeviceGetAttribute(&cus, hipDeviceAttributeMultiprocessorCount, dev) != hipSuccess || cus <= 0)
        cus = 256;
    return 2 * cus;
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

int get_plan(int N, int M, int P, int Q, DevPlan **out)
{
    int dev = 0;
    HIP_TRY(hipGetDevice(&dev));
    auto key = std::make_tuple(dev, N, M, P, Q);
    std::lock_guard<std::mutex> lk(g_pmu);
    auto it = g_plans.find(key);
    if (it != g_plans.end()) {
        *out = it->second.get();
        return COVEST_OK;
    }
    auto dp = std::make_unique<DevPlan>();
    dp->sp = make_shape_plan(N, M, P, Q, n_slots_for_device(dev));
    HIP_TRY(upload(&dp->d_jobs, dp->sp.jobs));
    HIP_TRY(upload(&dp->d_groups, dp->sp.groups));
    HIP_TRY(upload(&dp->d_items, dp->sp.items));
    dp->xcd_remap = dp->sp.jobs.empty() ? 0 : 1;
    *out = dp.get();
    g_plans.emplace(key, std::move(dp));
    return COVEST_OK;
}

std::mutex g_hmu;
std::map<std::tuple<int, int, int, int, int>, std::shared_ptr<const ShapePlan>> g_host_plans;

// Host-only planning, cached (workspace queries must work without a device).
std::shared_ptr<const ShapePlan> host_plan(int N, int M, int P, int Q)
{
    int dev = 0, slots = 512;
    if (hipGetDevice(&dev) == hipSuccess) slots = n_slots_for_device(dev);
    auto key = std::make_tuple(slots, N, M, P, Q);
    std::lock_guard<std::mutex> lk(g_hmu);
    auto it = g_host_plans.find(key);
    if (it != g_host_plans.end()) return it->second;
    auto sp = std::make_shared<const ShapePlan>(make_shape_plan(N, M, P, Q, slots));
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
    in.zc = in.zr + (size_t)2 * sp.lag_stride * sp.n_ir;
    in.out_fp64 = o.prec == COVEST_PREC_FP64 ? 1 : 0;
    in.fill_full = o.fill == COVEST_FILL_FULL ? 1 : 0;
    in.normalize = o.normalize ? 1 : 0;
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

int rec_forward(const void *A, int64_t lda, int N, int M, int P, int Q, void *R, int64_t ldr,
                const covest_opts &o, void *ws, size_t ws_bytes, hipStream_t stream)
{
    if (P > kMaxWindow || Q > kMaxWindow)
        return fail(COVEST_ERR_UNSUPPORTED, "the recurrence form supports P, Q <= %d", kMaxWindow);
    if (o.prec != COVEST_PREC_FP64 && o.prec != COVEST_PREC_FP32)
        return fail(COVEST_ERR_UNSUPPORTED, "the recurrence form computes in FP64 (prec FP64 or FP32 output)");
    DevPlan *dp = nullptr;
    int st = get_plan(N, M, P, Q, &dp);
    if (st != COVEST_OK) return st;
    const ShapePlan &sp = dp->sp;
    if (ws_bytes < sp.ws_bytes || (sp.ws_bytes > 0 && ws == nullptr))
        return fail(COVEST_ERR_WORKSPACE, "workspace of %zu bytes needed, %zu given", sp.ws_bytes, ws_bytes);
    const Inst in = make_inst(sp, A, lda, R, ldr, ws, o);
    if (!sp.jobs.empty()) {
        MainArgs ma{};
        ma.jobs = dp->d_jobs;
        ma.groups = dp->d_groups;
        ma.insts = nullptr;
        ma.n_jobs = (int)sp.jobs.size();
        ma.xcd_remap = dp->xcd_remap;
        ma.use_inline = 1;
        ma.inst_inline = in;
        HIP_TRY(timed("rec_main", stream, [&] {
            return launch_rec_main(ma, (int)sp.jobs.size(), sp.lds_main, stream);
        }));
    }
    FinArgs fa{};
    fa.items = dp->d_items;
    fa.insts = nullptr;
    fa.n_items = (int)sp.items.size();
    fa.use_inline = 1;
    fa.inst_inline = in;
    HIP_TRY(timed("rec_finalize", stream, [&] {
        return launch_rec_finalize(fa, (int)sp.items.size(), sp.lds_fin, sp.fin_table, stream);
    }));
    return finish_call(stream);
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
    ha.partial = static_cast<double *>(ws);
    ha.R = R;
    ha.ldr = ldr;
    ha.fill_full = o.fill == COVEST_FILL_FULL ? 1 : 0;
    ha.normalize = o.normalize ? 1 : 0;
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
    int64_t n_frame;
    size_t lds_tables, lds_interior, ws_bytes;
};

AdjGeom adj_geometry(int N, int M, int P, int Q)
{
    AdjGeom g{};
    const int Kr = N - P + 1, Kc = M - Q + 1;
    g.n_lags = (2 * P - 1) * (2 * Q - 1);
    g.ndc = ((2 * Q - 1 + 15) / 16) * 16;
    g.lds_tables = (size_t)(P + 1) * (Q + 1) * 16;
    const int rows = kAdjTR + 2 * (P - 1);
    const int stride = (kAdjTC + g.ndc) | 1;
    g.lds_interior = std::max((size_t)(2 * P - 1) * g.ndc * 16 + (size_t)rows * stride * 8,
                              (size_t)256 * 16 * 16);
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
    g.n_frame = (int64_t)N * M - (int64_t)(g.ir1 - g.ir0) * (g.ic1 - g.ic0);
    g.ws_bytes = (size_t)g.n_lags * (P + 1) * (Q + 1) * 16 + (size_t)g.n_lags * 16;
    return g;
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
        if (P > kMaxWindow || Q > kMaxWindow)
            return fail(COVEST_ERR_UNSUPPORTED, "the recurrence form supports P, Q <= %d", kMaxWindow);
        *bytes = host_plan((int)N, (int)M, (int)P, (int)Q)->ws_bytes;
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
    if (use_recurrence(o))
        return rec_forward(A, lda, (int)N, (int)M, (int)P, (int)Q, R, ldr, o, ws, ws_bytes, stream);
    return hankel_forward(A, lda, (int)N, (int)M, (int)P, (int)Q, R, ldr, o, ws, ws_bytes, stream);
}

int covest_forward(const void *A, int64_t N, int64_t M, int64_t P, int64_t Q, void *R,
                   const covest_opts *opts, void *ws, size_t ws_bytes, hipStream_t stream)
{
    return covest_forward_ex(A, M, N, M, P, Q, R, P * Q, opts, ws, ws_bytes, stream);
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

int covest_backward(const void *A, const void *dR, void *dA, int64_t N, int64_t M, int64_t P, int64_t Q,
                    const covest_opts *opts, void *ws, size_t ws_bytes, hipStream_t stream)
{
    const covest_opts o = resolve_opts(opts);
    int st = check_opts(o);
    if (st != COVEST_OK) return st;
    st = check_shape(N, M, P, Q);
    if (st != COVEST_OK) return st;
    if (!A || !dR || !dA) return fail(COVEST_ERR_INVALID_ARG, "A, dR and dA must be non-null device pointers");
    if (dA == A || dA == dR) return fail(COVEST_ERR_INVALID_ARG, "dA must not alias A or dR");
    if (P > kMaxWindow || Q > kMaxWindow)
        return fail(COVEST_ERR_UNSUPPORTED, "the adjoint supports P, Q <= %d", kMaxWindow);
    const AdjGeom g = adj_geometry((int)N, (int)M, (int)P, (int)Q);
    if (ws_bytes < g.ws_bytes || ws == nullptr)
        return fail(COVEST_ERR_WORKSPACE, "workspace of %zu bytes needed, %zu given", g.ws_bytes, ws_bytes);
    AdjArgs aa{};
    aa.A = static_cast<const float2 *>(A);
    aa.lda = M;
    aa.G = static_cast<const float2 *>(dR);
    aa.ldg = P * Q;
    aa.dA = static_cast<float2 *>(dA);
    aa.ldda = M;
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
    aa.n_frame = g.n_frame;
    aa.tables = static_cast<double *>(ws);
    aa.hfull = aa.tables + (size_t)2 * g.n_lags * (P + 1) * (Q + 1);
    aa.normalize = o.normalize ? 1 : 0;
    HIP_TRY(timed("adjoint", stream, [&] {
        return launch_adjoint(aa, g.n_lags, g.lds_tables, g.interior_blocks, g.lds_interior, g.n_frame, stream);
    }));
    return finish_call(stream);
}

int covest_plan_batched_create(covest_plan **out, const covest_problem *problems, int64_t count,
                               const covest_opts *opts, hipStream_t stream)
{
    (void)out; (void)problems; (void)count; (void)opts; (void)stream;
    return fail(COVEST_ERR_UNSUPPORTED, "batched plans are not available in this build");
}

int covest_forward_batched(covest_plan *plan, hipStream_t stream)
{
    (void)plan; (void)stream;
    return fail(COVEST_ERR_UNSUPPORTED, "batched plans are not available in this build");
}

int covest_plan_destroy(covest_plan *plan)
{
    (void)plan;
    return ok();
}

int covest_plan_info_get(int64_t N, int64_t M, int64_t P, int64_t Q, int32_t n_slots,
                         covest_plan_info *out)
{
    if (!out) return fail(COVEST_ERR_INVALID_ARG, "out is null");
    int st = check_shape(N, M, P, Q);
    if (st != COVEST_OK) return st;
    if (P > kMaxWindow || Q > kMaxWindow)
        return fail(COVEST_ERR_UNSUPPORTED, "the recurrence form supports P, Q <= %d", kMaxWindow);
    const ShapePlan sp = make_shape_plan((int)N, (int)M, (int)P, (int)Q, n_slots > 0 ? n_slots : 512);
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

int covest_plan_tables(int64_t N, int64_t M, int64_t P, int64_t Q, int32_t n_slots, int32_t *jobs,
                       int32_t *groups, int32_t *items)
{
    int st = check_shape(N, M, P, Q);
    if (st != COVEST_OK) return st;
    if (P > kMaxWindow || Q > kMaxWindow)
        return fail(COVEST_ERR_UNSUPPORTED, "the recurrence form supports P, Q <= %d", kMaxWindow);
    const ShapePlan sp = make_shape_plan((int)N, (int)M, (int)P, (int)Q, n_slots > 0 ? n_slots : 512);
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
