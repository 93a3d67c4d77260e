// sc_api.cpp -- host runtime behind the C ABI declared in include/sc.h:
// contexts, problems, argument validation, device memory, launch shapes,
// the batched persistent launch, timing and the autotuner.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <chrono>
#include <cmath>
#include <cstdarg>
#include <cstdio>
#include <cstring>
#include <fstream>
#include <map>
#include <mutex>
#include <new>
#include <sstream>
#include <string>
#include <tuple>
#include <vector>

#include "sc_host.h"

using namespace sc;

// ===================================================================== errors

static thread_local std::string g_err;

sc_status sc::fail(sc_status st, const char *fmt, ...)
{
    char buf[512];
    va_list ap;
    va_start(ap, fmt);
    vsnprintf(buf, sizeof buf, fmt, ap);
    va_end(ap);
    g_err = buf;
    return st;
}

extern "C" const char *sc_last_error(void) { return g_err.c_str(); }
extern "C" const char *sc_version(void) { return "sc-mi355x 0.1 (gfx950)"; }

bool sc::debug_fail_this_alloc()
{
    static std::mutex mu;
    static long count = 0;
    static long fail_at = -2;
    std::lock_guard<std::mutex> lk(mu);
    if (fail_at == -2) {
        const char *s = getenv("SC_DEBUG_FAIL_ALLOC");
        fail_at = s ? atol(s) : -1;
    }
    ++count;
    return fail_at > 0 && count == fail_at;
}

static sc_status scratch_init(int device);

extern "C" sc_status sc_ctx_create(int device, void *stream, sc_ctx **out)
{
    if (!out) return fail(SC_E_INVAL, "sc_ctx_create: out is NULL");
    *out = nullptr;
    int n = 0;
    HIP_TRY(hipGetDeviceCount(&n));
    if (device < 0 || device >= n) return fail(SC_E_INVAL, "sc_ctx_create: device %d not in [0, %d)", device, n);
    DeviceGuard g(device);
    sc_ctx *c = new (std::nothrow) sc_ctx();
    if (!c) return fail(SC_E_NOMEM, "sc_ctx_create: out of host memory");
    c->device = device;
    hipDeviceProp_t prop;
    if (hipGetDeviceProperties(&prop, device) == hipSuccess && prop.multiProcessorCount > 0)
        c->n_cu = prop.multiProcessorCount;
    if (stream) {
        c->stream = (hipStream_t)stream;
    } else {
        if (hipStreamCreateWithFlags(&c->stream, hipStreamNonBlocking) != hipSuccess) {
            delete c;
            return fail(SC_E_DEVICE, "sc_ctx_create: hipStreamCreate failed");
        }
        c->own_stream = true;
    }
    static_assert(QUAD_SEGMENTS * sizeof(unsigned int) <= 256, "work counters must fit the counter buffer");
    sc_status st = scratch_init(device);
    if (st == SC_OK) st = c->counter.reserve(256);
    if (st == SC_OK && hipEventCreateWithFlags(&c->upload_done, hipEventDisableTiming) != hipSuccess)
        st = fail(SC_E_DEVICE, "sc_ctx_create: hipEventCreate failed");
    if (st != SC_OK) {
        if (c->own_stream) (void)hipStreamDestroy(c->stream);
        delete c;
        return st;
    }
    *out = c;
    return SC_OK;
}

extern "C" sc_status sc_ctx_destroy(sc_ctx *c)
{
    if (!c) return SC_OK;
    if (c->n_probs > 0)
        return fail(SC_E_STATE, "sc_ctx_destroy: %d problem(s) still alive on this context", c->n_probs.load());
    DeviceGuard g(c->device);
    (void)hipStreamSynchronize(c->stream);
    if (c->upload_done) (void)hipEventDestroy(c->upload_done);
    c->counter.release();
    c->jobs.release();
    if (c->own_stream) (void)hipStreamDestroy(c->stream);
    delete c;
    return SC_OK;
}

extern "C" sc_status sc_ctx_synchronize(sc_ctx *c)
{
    if (!c) return fail(SC_E_INVAL, "sc_ctx_synchronize: ctx is NULL");
    DeviceGuard g(c->device);
    HIP_TRY(hipStreamSynchronize(c->stream));
    return SC_OK;
}

extern "C" sc_status sc_ctx_set_profiling(sc_ctx *c, int enable)
{
    if (!c) return fail(SC_E_INVAL, "sc_ctx_set_profiling: ctx is NULL");
    c->profiling = enable ? 1 : 0;
    return SC_OK;
}

// ================================================================== problem

static size_t round_up(size_t v, size_t m) { return (v + m - 1) / m * m; }

static int log2_bucket(int64_t v)
{
    int b = 0;
    while (v > 1) {
        v >>= 1;
        ++b;
    }
    return b;
}

extern "C" sc_status sc_prob_create(sc_ctx *ctx, sc_prob **out)
{
    if (!ctx || !out) return fail(SC_E_INVAL, "sc_prob_create: NULL argument");
    *out = nullptr;
    DeviceGuard g(ctx->device);
    sc_prob *p = new (std::nothrow) sc_prob();
    if (!p) return fail(SC_E_NOMEM, "sc_prob_create: out of host memory");
    p->ctx = ctx;
    ctx->n_probs++;
    for (int i = 0; i < EV_N; ++i) {
        if (hipEventCreate(&p->ev[i]) != hipSuccess) {
            for (int j = 0; j < i; ++j) (void)hipEventDestroy(p->ev[j]);
            ctx->n_probs--;
            delete p;
            return fail(SC_E_DEVICE, "sc_prob_create: hipEventCreate failed");
        }
    }
    *out = p;
    return SC_OK;
}

extern "C" sc_status sc_prob_destroy(sc_prob *p)
{
    if (!p) return SC_OK;
    DeviceGuard g(p->ctx->device);
    // buffers from the stream-ordered allocator are freed behind the work queued on their stream; the
    // others need the problem's work finished first
    if (!p->alloc_stream) (void)hipStreamSynchronize(p->ctx->stream);
    for (int i = 0; i < EV_N; ++i)
        if (p->ev[i]) (void)hipEventDestroy(p->ev[i]);
    if (p->stage_ev) (void)hipEventDestroy(p->stage_ev);
    if (p->fact_ev) (void)hipEventDestroy(p->fact_ev);
    p->ctx->n_probs--;
    delete p;   // DevBufs free themselves
    return SC_OK;
}

// The staging vectors of a problem are rewritten only after the last copy from them has run.
static sc_status staging_wait(sc_prob *p)
{
    if (p->stage_pending) {
        HIP_TRY(hipEventSynchronize(p->stage_ev));
        p->stage_pending = false;
    }
    return SC_OK;
}

static sc_status staging_mark(sc_prob *p)
{
    if (!p->stage_ev) HIP_TRY(hipEventCreateWithFlags(&p->stage_ev, hipEventDisableTiming));
    HIP_TRY(hipEventRecord(p->stage_ev, p->ctx->stream));
    p->stage_pending = true;
    return SC_OK;
}

// Host memory for an upload of n doubles: a slice of the problem's pinned area when it has one with
// room left (*in_ext = true), else the staging vector `vec` (after its last upload has run); in that
// case staging_mark follows the copies.
static sc_status stage_area(sc_prob *p, std::vector<double> &vec, size_t n, double **out, bool *in_ext)
{
    const size_t bytes = (sizeof(double) * n + 63) & ~size_t(63);
    if (p->stage_ext && p->stage_ext_off + bytes <= p->stage_ext_cap) {
        *out = (double *)(p->stage_ext + p->stage_ext_off);
        p->stage_ext_off += bytes;
        *in_ext = true;
        return SC_OK;
    }
    SC_TRY(staging_wait(p));
    vec.resize(n);
    *out = vec.data();
    *in_ext = false;
    return SC_OK;
}

// Gauss-Legendre rules are computed once per order and kept by the context.
static void gauss_rule_cached(sc_ctx *c, int n, const std::vector<double> *out[2])
{
    auto it = c->gauss.find(n);
    if (it == c->gauss.end()) {
        std::pair<std::vector<double>, std::vector<double>> r;
        gauss_legendre_rule(n, r.first, r.second);
        it = c->gauss.emplace(n, std::move(r)).first;
    }
    out[0] = &it->second.first;
    out[1] = &it->second.second;
}

static void invalidate_tables(sc_prob *p)
{
    p->has_tab = p->tab32_ok = p->tab32n_ok = p->has_tab64 = p->has_power = false;
    p->fact_checked = p->fact_ok = p->fact64_ok = p->tie_ok = p->tie64_ok = false;
    p->fact32_built = p->fact64_built = false;
    p->fact_pending = p->cast_pending = false;   // a flag still on its way belongs to the old tables
    p->res_prec = -1;
}

// Relative tolerances of the factoring test (residual of the current off its direction u, over the
// node's largest |Jt|): the built-in beams whose current keeps one real direction factor to rounding
// (~1e-16); the longitudinal magnetic term of the curl-consistent linear beam turns the current by
// O(1/(k w0)) and is rejected.  FP64 evaluation, accurate to ~1e-13, takes the factored tables only
// when the residual is below 1e-14.  The same tolerances, against the node's largest |rho_t|,
// decide whether the charge is tied to the current (rho_t = -i beta s / k): it is, to rounding, for
// the beams whose E and B share one complex amplitude.
constexpr double FACTOR_TOL = 1e-10;
constexpr double FACTOR_TOL_FP64 = 1e-14;

// The outcome of the factoring test (bit 0: the FP32 split tolerance failed, bit 1: the FP64
// one; bits 2 and 3 the same for the tied charge): which factored tables exist now, and the ones
// that will not be used are released.
static void apply_factoring_flag(sc_prob *p, unsigned int bad, bool need32, bool need64)
{
    p->fact_checked = true;
    p->fact_ok = (bad & 1u) == 0;
    p->fact64_ok = p->fact_ok && (bad & 2u) == 0;
    p->tie_ok = p->fact_ok && (bad & 4u) == 0;
    p->tie64_ok = p->fact64_ok && (bad & 8u) == 0;
    p->fact32_built = p->fact32_built || (need32 && p->fact_ok);
    p->fact64_built = p->fact64_built || (need64 && p->fact64_ok);
    if (!p->fact_ok) {
        p->tabf.release();
        p->posf.release();
        p->betaf.release();
        p->tabp.release();
    }
    if (!p->fact64_ok) {
        p->tabf64.release();
        p->posf64.release();
        p->betaf64.release();
    }
}

static sc_status drop_fp64_tables(sc_prob *p, bool cast);

sc_status sc::resolve_factoring(sc_prob *p, bool block, bool *ready)
{
    if (ready) *ready = true;
    if (!p->fact_pending) return SC_OK;
    if (block) {
        HIP_TRY(hipEventSynchronize(p->fact_ev));
    } else {
        const hipError_t e = hipEventQuery(p->fact_ev);
        if (e == hipErrorNotReady) {
            (void)hipGetLastError();
            if (ready) *ready = false;
            return SC_OK;
        }
        HIP_TRY(e);
    }
    p->fact_pending = false;
    apply_factoring_flag(p, *p->fact_flag_host, p->fact_req32, p->fact_req64);
    if (p->cast_pending) {
        p->cast_pending = false;
        const bool cast = !(p->allow_fact && p->fact_ok);
        // without a cast the factoring kernel, finished now, was the FP64 tables' last user
        if (!cast && p->free_stream && p->tab64.stream) p->tab64.stream = p->free_stream;
        SC_TRY(drop_fp64_tables(p, cast));
    }
    return SC_OK;
}

// A problem's factoring state is read only after a deferred test has completed.
static sc_status settle_factoring(sc_prob *p) { return resolve_factoring(p, true, nullptr); }

// Factored tables from the FP64 tables: the test runs once per table set (one flag read back); the
// FP32 split (need32) and FP64 (need64) tables are built when asked for and the test passed at that
// precision's tolerance (otherwise the general tables are used).  With fact_flag_host set, the flag
// is not waited for: the test completes in resolve_factoring.
static sc_status ensure_factored(sc_prob *p, bool need32, bool need64)
{
    if (!p->allow_fact || !p->has_tab64) return SC_OK;
    SC_TRY(settle_factoring(p));
    if (p->fact_checked) {
        need32 = need32 && p->fact_ok && !p->fact32_built;
        need64 = need64 && p->fact64_ok && !p->fact64_built;
        if (!need32 && !need64) return SC_OK;
    }
    hipStream_t st = p->ctx->stream;
    const int n_k = (int)p->k.size();
    const size_t nrec = (size_t)n_k * p->n_tot;
    if (need32) {
        SC_TRY(p->tabf.reserve(sizeof(float) * 4 * nrec, p->alloc_stream));
        SC_TRY(p->posf.reserve(sizeof(float) * 8 * (size_t)p->n_tot, p->alloc_stream));
        SC_TRY(p->betaf.reserve(sizeof(float) * (size_t)p->n_tot, p->alloc_stream));
        SC_TRY(p->tabp.reserve(sizeof(float) * 2 * nrec, p->alloc_stream));
    }
    if (need64) {
        SC_TRY(p->tabf64.reserve(sizeof(double) * 4 * nrec, p->alloc_stream));
        SC_TRY(p->posf64.reserve(sizeof(double) * 8 * (size_t)p->n_tot, p->alloc_stream));
        SC_TRY(p->betaf64.reserve(sizeof(double) * (size_t)p->n_tot, p->alloc_stream));
    }
    SC_TRY(p->fact_flag.reserve(sizeof(unsigned int), p->alloc_stream));
    HIP_TRY(launch_fill_u32(st, p->fact_flag.as<unsigned int>(), 0u, 1));
    HIP_TRY(launch_tables_factor(st, n_k, p->n_tot, p->d_k.as<double>(), p->tab64.as<double>(),
                                 p->pos32.as<float>(), p->pos64.as<double>(), FACTOR_TOL, FACTOR_TOL_FP64,
                                 need32 ? p->tabf.as<float>() : nullptr, need32 ? p->posf.as<float>() : nullptr,
                                 need32 ? p->betaf.as<float>() : nullptr, need32 ? p->tabp.as<float>() : nullptr,
                                 need64 ? p->tabf64.as<double>() : nullptr,
                                 need64 ? p->posf64.as<double>() : nullptr,
                                 need64 ? p->betaf64.as<double>() : nullptr, p->fact_flag.as<unsigned int>()));
    if (p->fact_checked) {
        p->fact32_built = p->fact32_built || need32;
        p->fact64_built = p->fact64_built || need64;
        return SC_OK;
    }
    if (p->fact_flag_host) {
        HIP_TRY(hipMemcpyAsync(p->fact_flag_host, p->fact_flag.p, sizeof(unsigned int), hipMemcpyDeviceToHost, st));
        if (!p->fact_ev) HIP_TRY(hipEventCreateWithFlags(&p->fact_ev, hipEventDisableTiming));
        HIP_TRY(hipEventRecord(p->fact_ev, st));
        p->fact_pending = true;
        p->fact_req32 = need32;
        p->fact_req64 = need64;
        return SC_OK;
    }
    unsigned int bad = 15;
    HIP_TRY(hipMemcpyAsync(&bad, p->fact_flag.p, sizeof(bad), hipMemcpyDeviceToHost, st));
    HIP_TRY(hipStreamSynchronize(st));
    apply_factoring_flag(p, bad, need32, need64);
    return SC_OK;
}

static sc_status reserve_power(sc_prob *p)
{
    const size_t n = p->k.size() + (size_t)power_partial_count((int)p->k.size());
    return p->d_power.reserve(sizeof(double) * n, p->alloc_stream);
}

// After tab64 was (re)built: with keep_fp64 off, cast to the FP32 split tables now and release tab64.
static sc_status finish_tables(sc_prob *p)
{
    p->has_tab = true;
    p->has_tab64 = true;
    // the factoring test (and the factored tables of the expected precision) now, so that the table
    // layout, and with it the launch shape, is known before the first evaluation; it needs the FP64
    // tables
    SC_TRY(ensure_factored(p, p->eager_prec == SC_FP32_SPLIT, p->eager_prec == SC_FP64 && p->keep_fp64));
    if (p->keep_fp64) return SC_OK;
    if (p->fact_pending) {   // the general FP32 tables only if the current does not factor
        p->cast_pending = true;
        return SC_OK;
    }
    return drop_fp64_tables(p, true);
}

// FP32-only storage: the general FP32 tables cast from the FP64 ones (when `cast`), then the FP64
// tables and their factored copy released.
static sc_status drop_fp64_tables(sc_prob *p, bool cast)
{
    if (cast) {
        const size_t nrec = p->k.size() * (size_t)p->n_tot;
        SC_TRY(p->tab32.reserve(sizeof(float) * 8 * nrec, p->alloc_stream));
        HIP_TRY(launch_tables_cast(p->ctx->stream, (int)p->k.size(), p->n_tot, p->d_k.as<double>(),
                                   p->pos64.as<double>(), p->tab64.as<double>(), nullptr, p->tab32.as<float>(), 0));
        p->tab32_ok = true;
    }
    // a stream-ordered free runs after the cast; a plain hipFree needs the cast to have finished
    if (!p->tab64.stream) HIP_TRY(hipStreamSynchronize(p->ctx->stream));
    p->tab64.release();
    p->has_tab64 = false;
    // without the FP64 tables there is no FP64 evaluation, so its factored tables go too
    p->tabf64.release();
    p->posf64.release();
    p->betaf64.release();
    p->fact64_built = false;
    return SC_OK;
}

extern "C" sc_status sc_set_table_storage(sc_prob *p, int keep_fp64)
{
    if (!p) return fail(SC_E_INVAL, "sc_set_table_storage: prob is NULL");
    DeviceGuard g(p->ctx->device);
    p->keep_fp64 = keep_fp64 != 0;
    if (!p->keep_fp64 && p->has_tab64) return finish_tables(p);
    return SC_OK;
}

extern "C" sc_status sc_set_factoring(sc_prob *p, int enable)
{
    if (!p) return fail(SC_E_INVAL, "sc_set_factoring: prob is NULL");
    if (enable < 0 || enable > 2) return fail(SC_E_INVAL, "sc_set_factoring: enable must be 0, 1 or 2");
    p->allow_fact = enable != 0;
    p->allow_tie = enable == 1;
    return SC_OK;
}

extern "C" sc_status sc_get_factoring_for(sc_prob *p, sc_precision prec, int *active)
{
    if (!p || !active) return fail(SC_E_INVAL, "sc_get_factoring: NULL argument");
    if (prec != SC_FP64 && prec != SC_FP32_SPLIT && prec != SC_FP32)
        return fail(SC_E_INVAL, "sc_get_factoring: unknown precision %d", (int)prec);
    if (!p->has_tab) return fail(SC_E_STATE, "sc_get_factoring: no incident field set");
    DeviceGuard g(p->ctx->device);
    SC_TRY(ensure_factored(p, false, false));   // runs the test if it has not run yet
    if (prec == SC_FP32_SPLIT) *active = p->allow_fact && p->fact_ok ? (p->allow_tie && p->tie_ok ? 2 : 1) : 0;
    else if (prec == SC_FP64)
        *active = p->allow_fact && p->fact64_ok && p->has_tab64 ? (p->allow_tie && p->tie64_ok ? 2 : 1) : 0;
    else *active = 0;
    return SC_OK;
}

extern "C" sc_status sc_get_factoring(sc_prob *p, int *active)
{
    return sc_get_factoring_for(p, SC_FP32_SPLIT, active);
}

extern "C" sc_status sc_set_mirror(sc_prob *p, double f, double r_max, int n_r, int n_phi)
{
    if (!p) return fail(SC_E_INVAL, "sc_set_mirror: prob is NULL");
    if (!(f > 0.0) || !std::isfinite(f)) return fail(SC_E_INVAL, "sc_set_mirror: f must be > 0 (got %g)", f);
    if (!(r_max > 0.0) || !std::isfinite(r_max)) return fail(SC_E_INVAL, "sc_set_mirror: r_max must be > 0");
    if (n_r < 1 || n_phi < 1) return fail(SC_E_INVAL, "sc_set_mirror: n_r, n_phi must be >= 1");
    if ((int64_t)(n_r + 1) * n_phi >= (1LL << 31))
        return fail(SC_E_INVAL, "sc_set_mirror: (n_r+1)*n_phi must be < 2^31");
    DeviceGuard g(p->ctx->device);
    hipStream_t st = p->ctx->stream;
    const std::vector<double> *xw[2];
    gauss_rule_cached(p->ctx, n_r, xw);
    const std::vector<double> &x = *xw[0], &w = *xw[1];
    // staging layout: r [n_r + 1], w_r [n_r], cos phi [n_phi], sin phi [n_phi]
    double *r = nullptr;
    bool ext = false;
    SC_TRY(stage_area(p, p->h_stage_rule, (size_t)2 * n_r + 1 + 2 * (size_t)n_phi, &r, &ext));
    double *wr = r + n_r + 1, *c = wr + n_r, *s = c + n_phi;
    for (int i = 0; i < n_r; ++i) {
        r[i] = r_max * (1.0 + x[i]) / 2.0;
        wr[i] = r_max * w[i] / 2.0;
    }
    r[n_r] = r_max;
    for (int j = 0; j < n_phi; ++j) {
        double phi = 2.0 * M_PI * (double)j / (double)n_phi;
        sincos(phi, &s[j], &c[j]);   // libm sincos: one correctly paired evaluation
    }
    const int n_tot = (n_r + 1) * n_phi;
    invalidate_tables(p);
    p->has_mirror = false;
    SC_TRY(p->d_r.reserve(sizeof(double) * (n_r + 1), p->alloc_stream));
    SC_TRY(p->d_wr.reserve(sizeof(double) * n_r, p->alloc_stream));
    SC_TRY(p->d_c.reserve(sizeof(double) * n_phi, p->alloc_stream));
    SC_TRY(p->d_s.reserve(sizeof(double) * n_phi, p->alloc_stream));
    SC_TRY(p->pos64.reserve(sizeof(double) * 4 * n_tot, p->alloc_stream));
    SC_TRY(p->pos32.reserve(sizeof(float) * 4 * n_tot, p->alloc_stream));
    SC_TRY(p->nrm.reserve(sizeof(double) * 3 * n_tot, p->alloc_stream));
    SC_TRY(p->wgt.reserve(sizeof(double) * n_tot, p->alloc_stream));
    SC_TRY(p->tan.reserve(sizeof(double) * 3 * n_phi, p->alloc_stream));
    HIP_TRY(hipMemcpyAsync(p->d_r.p, r, sizeof(double) * (n_r + 1), hipMemcpyHostToDevice, st));
    HIP_TRY(hipMemcpyAsync(p->d_wr.p, wr, sizeof(double) * n_r, hipMemcpyHostToDevice, st));
    HIP_TRY(hipMemcpyAsync(p->d_c.p, c, sizeof(double) * n_phi, hipMemcpyHostToDevice, st));
    HIP_TRY(hipMemcpyAsync(p->d_s.p, s, sizeof(double) * n_phi, hipMemcpyHostToDevice, st));
    if (!ext) SC_TRY(staging_mark(p));
    HIP_TRY(launch_node_tables(st, n_r, n_phi, f, p->d_r.as<double>(), p->d_wr.as<double>(), p->d_c.as<double>(),
                               p->d_s.as<double>(), 2.0 * M_PI / (double)n_phi, p->pos64.as<double>(),
                               p->pos32.as<float>(), p->nrm.as<double>(), p->wgt.as<double>(), p->tan.as<double>()));
    SC_TRY(p->hinv64.reserve(sizeof(double) * n_tot, p->alloc_stream));
    SC_TRY(p->hinv32.reserve(sizeof(float) * n_tot, p->alloc_stream));
    HIP_TRY(launch_node_half_inverse(st, n_tot, p->pos64.as<double>(), p->hinv64.as<double>(),
                                     p->hinv32.as<float>()));
    p->f = f;
    p->a = r_max;
    p->rs_min = f;   // |r_s| = r^2 / 4f + f on the paraboloid (distance to the focus)
    p->n_r = n_r;
    p->n_phi = n_phi;
    p->n_surf = n_r * n_phi;
    p->n_rim = n_phi;
    p->n_tot = n_tot;
    p->has_mirror = true;
    return SC_OK;
}

extern "C" sc_status sc_set_surface(sc_prob *p, int n_surf, const double *xyz, const double *ndS, int n_rim,
                                    const double *rim_xyz, const double *rim_n, const double *rim_dl)
{
    if (!p || !xyz || !ndS) return fail(SC_E_INVAL, "sc_set_surface: NULL argument");
    if (n_surf < 1 || n_rim < 0) return fail(SC_E_INVAL, "sc_set_surface: need n_surf >= 1 and n_rim >= 0");
    if (n_rim > 0 && (!rim_xyz || !rim_n || !rim_dl)) return fail(SC_E_INVAL, "sc_set_surface: NULL rim array");
    if ((int64_t)n_surf + n_rim >= (1LL << 31)) return fail(SC_E_INVAL, "sc_set_surface: too many nodes");
    for (int64_t i = 0; i < 3LL * n_surf; ++i)
        if (!std::isfinite(xyz[i]) || !std::isfinite(ndS[i]))
            return fail(SC_E_INVAL, "sc_set_surface: surface node %lld is not finite", (long long)(i / 3));
    for (int64_t i = 0; i < 3LL * n_rim; ++i)
        if (!std::isfinite(rim_xyz[i]) || !std::isfinite(rim_n[i]) || !std::isfinite(rim_dl[i]))
            return fail(SC_E_INVAL, "sc_set_surface: rim node %lld is not finite", (long long)(i / 3));
    for (int j = 0; j < n_rim; ++j)
        if (!(rim_n[3 * j] * rim_n[3 * j] + rim_n[3 * j + 1] * rim_n[3 * j + 1] + rim_n[3 * j + 2] * rim_n[3 * j + 2] >
              0.0))
            return fail(SC_E_INVAL, "sc_set_surface: rim normal %d is zero", j);
    DeviceGuard g(p->ctx->device);
    hipStream_t st = p->ctx->stream;
    const int n_tot = n_surf + n_rim;
    invalidate_tables(p);
    p->has_mirror = false;
    DevBuf d_xyz, d_nds, d_rx, d_rn, d_rdl;
    SC_TRY(d_xyz.reserve(sizeof(double) * 3 * n_surf, p->alloc_stream));
    SC_TRY(d_nds.reserve(sizeof(double) * 3 * n_surf, p->alloc_stream));
    SC_TRY(d_rx.reserve(sizeof(double) * 3 * std::max(n_rim, 1), p->alloc_stream));
    SC_TRY(d_rn.reserve(sizeof(double) * 3 * std::max(n_rim, 1), p->alloc_stream));
    SC_TRY(d_rdl.reserve(sizeof(double) * 3 * std::max(n_rim, 1), p->alloc_stream));
    SC_TRY(p->pos64.reserve(sizeof(double) * 4 * n_tot, p->alloc_stream));
    SC_TRY(p->pos32.reserve(sizeof(float) * 4 * n_tot, p->alloc_stream));
    SC_TRY(p->nrm.reserve(sizeof(double) * 3 * n_tot, p->alloc_stream));
    SC_TRY(p->wgt.reserve(sizeof(double) * n_tot, p->alloc_stream));
    SC_TRY(p->tan.reserve(sizeof(double) * 3 * std::max(n_rim, 1), p->alloc_stream));
    HIP_TRY(hipMemcpyAsync(d_xyz.p, xyz, sizeof(double) * 3 * n_surf, hipMemcpyHostToDevice, st));
    HIP_TRY(hipMemcpyAsync(d_nds.p, ndS, sizeof(double) * 3 * n_surf, hipMemcpyHostToDevice, st));
    if (n_rim > 0) {
        HIP_TRY(hipMemcpyAsync(d_rx.p, rim_xyz, sizeof(double) * 3 * n_rim, hipMemcpyHostToDevice, st));
        HIP_TRY(hipMemcpyAsync(d_rn.p, rim_n, sizeof(double) * 3 * n_rim, hipMemcpyHostToDevice, st));
        HIP_TRY(hipMemcpyAsync(d_rdl.p, rim_dl, sizeof(double) * 3 * n_rim, hipMemcpyHostToDevice, st));
    }
    HIP_TRY(launch_surface_records(st, n_surf, n_rim, d_xyz.as<double>(), d_nds.as<double>(), d_rx.as<double>(),
                                   d_rn.as<double>(), d_rdl.as<double>(), p->pos64.as<double>(), p->pos32.as<float>(),
                                   p->nrm.as<double>(), p->wgt.as<double>(), p->tan.as<double>()));
    SC_TRY(p->hinv64.reserve(sizeof(double) * n_tot, p->alloc_stream));
    SC_TRY(p->hinv32.reserve(sizeof(float) * n_tot, p->alloc_stream));
    HIP_TRY(launch_node_half_inverse(st, n_tot, p->pos64.as<double>(), p->hinv64.as<double>(),
                                     p->hinv32.as<float>()));
    HIP_TRY(hipStreamSynchronize(st));   // staging buffers are freed on return
    double rs2 = INFINITY;
    for (int i = 0; i < n_surf; ++i)
        rs2 = std::min(rs2, xyz[3 * i] * xyz[3 * i] + xyz[3 * i + 1] * xyz[3 * i + 1] + xyz[3 * i + 2] * xyz[3 * i + 2]);
    for (int j = 0; j < n_rim; ++j)
        rs2 = std::min(rs2, rim_xyz[3 * j] * rim_xyz[3 * j] + rim_xyz[3 * j + 1] * rim_xyz[3 * j + 1] +
                                rim_xyz[3 * j + 2] * rim_xyz[3 * j + 2]);
    p->rs_min = std::sqrt(rs2);
    p->f = p->a = 0.0;
    p->n_r = p->n_phi = 0;
    p->n_surf = n_surf;
    p->n_rim = n_rim;
    p->n_tot = n_tot;
    p->has_mirror = true;
    return SC_OK;
}

extern "C" sc_status sc_get_num_nodes(const sc_prob *p, int *n_surface, int *n_rim)
{
    if (!p) return fail(SC_E_INVAL, "sc_get_num_nodes: prob is NULL");
    if (!p->has_mirror) return fail(SC_E_STATE, "sc_get_num_nodes: no mirror set");
    if (n_surface) *n_surface = p->n_surf;
    if (n_rim) *n_rim = p->n_rim;
    return SC_OK;
}

extern "C" sc_status sc_get_nodes(const sc_prob *p, double *xyz, double *normal, double *weight)
{
    if (!p) return fail(SC_E_INVAL, "sc_get_nodes: prob is NULL");
    if (!p->has_mirror) return fail(SC_E_STATE, "sc_get_nodes: no mirror set");
    DeviceGuard g(p->ctx->device);
    hipStream_t st = p->ctx->stream;
    HIP_TRY(hipStreamSynchronize(st));
    if (xyz) {
        std::vector<double> tmp((size_t)4 * p->n_tot);
        HIP_TRY(hipMemcpy(tmp.data(), p->pos64.p, sizeof(double) * 4 * p->n_tot, hipMemcpyDeviceToHost));
        for (int q = 0; q < p->n_tot; ++q)
            for (int c = 0; c < 3; ++c) xyz[3 * (size_t)q + c] = tmp[4 * (size_t)q + c];
    }
    if (normal) HIP_TRY(hipMemcpy(normal, p->nrm.p, sizeof(double) * 3 * p->n_tot, hipMemcpyDeviceToHost));
    if (weight) HIP_TRY(hipMemcpy(weight, p->wgt.p, sizeof(double) * p->n_tot, hipMemcpyDeviceToHost));
    return SC_OK;
}

extern "C" sc_status sc_set_frequencies(sc_prob *p, const double *k, int n_k)
{
    if (!p) return fail(SC_E_INVAL, "sc_set_frequencies: prob is NULL");
    if (!k || n_k < 1) return fail(SC_E_INVAL, "sc_set_frequencies: need n_k >= 1 wavenumbers");
    if (n_k > SC_MAX_FREQUENCIES)
        return fail(SC_E_INVAL, "sc_set_frequencies: at most %d wavenumbers per problem", SC_MAX_FREQUENCIES);
    for (int i = 0; i < n_k; ++i)
        if (!(k[i] > 0.0) || !std::isfinite(k[i]))
            return fail(SC_E_INVAL, "sc_set_frequencies: k[%d] = %g is not a positive wavenumber", i, k[i]);
    DeviceGuard g(p->ctx->device);
    invalidate_tables(p);
    p->k.assign(k, k + n_k);
    SC_TRY(p->d_k.reserve(sizeof(double) * n_k, p->alloc_stream));
    if (p->stage_ext) {   // p->k is pageable: copy from the pinned area when there is one
        double *h = nullptr;
        bool ext = false;
        SC_TRY(stage_area(p, p->h_stage_spec, (size_t)n_k, &h, &ext));
        if (ext) {
            std::copy(k, k + n_k, h);
            HIP_TRY(hipMemcpyAsync(p->d_k.p, h, sizeof(double) * n_k, hipMemcpyHostToDevice, p->ctx->stream));
            return SC_OK;
        }
    }
    HIP_TRY(hipMemcpyAsync(p->d_k.p, p->k.data(), sizeof(double) * n_k, hipMemcpyHostToDevice, p->ctx->stream));
    return SC_OK;
}

static void ev_record(sc_prob *p, int which)
{
    if (p->ctx->profiling) (void)hipEventRecord(p->ev[which], p->ctx->stream);
}

extern "C" sc_status sc_set_incident(sc_prob *p, const double *E, const double *B, int on_device)
{
    if (!p || !E || !B) return fail(SC_E_INVAL, "sc_set_incident: NULL argument");
    if (!p->has_mirror || p->k.empty()) return fail(SC_E_STATE, "sc_set_incident: set mirror and frequencies first");
    DeviceGuard g(p->ctx->device);
    hipStream_t st = p->ctx->stream;
    const int n_k = (int)p->k.size();
    const size_t nrec = (size_t)n_k * p->n_tot;
    invalidate_tables(p);
    SC_TRY(p->tab64.reserve(sizeof(double) * 8 * nrec, p->alloc_stream));
    DevBuf stageE, stageB;
    const double *dE = E, *dB = B;
    if (!on_device) {
        SC_TRY(stageE.reserve(sizeof(double) * 6 * nrec, p->alloc_stream));
        SC_TRY(stageB.reserve(sizeof(double) * 6 * nrec, p->alloc_stream));
        HIP_TRY(hipMemcpyAsync(stageE.p, E, sizeof(double) * 6 * nrec, hipMemcpyHostToDevice, st));
        HIP_TRY(hipMemcpyAsync(stageB.p, B, sizeof(double) * 6 * nrec, hipMemcpyHostToDevice, st));
        dE = stageE.as<double>();
        dB = stageB.as<double>();
    }
    ev_record(p, EV_PREP0);
    HIP_TRY(launch_tables_from_fields(st, n_k, p->n_surf, p->n_tot, p->d_k.as<double>(), p->pos64.as<double>(),
                                      p->nrm.as<double>(), p->wgt.as<double>(), p->tan.as<double>(), dE, dB,
                                      p->tab64.as<double>()));
    SC_TRY(reserve_power(p));
    HIP_TRY(launch_power_fields(st, n_k, p->n_surf, p->n_tot, p->nrm.as<double>(), p->wgt.as<double>(), dE, dB,
                                p->d_power.as<double>() + n_k, p->d_power.as<double>()));
    p->has_power = true;
    ev_record(p, EV_PREP1);
    p->ev_prep = p->ctx->profiling;
    if (!on_device) HIP_TRY(hipStreamSynchronize(st));   // staging buffers are freed on return
    return finish_tables(p);
}

// Tables and aperture power of a built-in beam (beam 3: the Laguerre-Gauss modes already in d_modes).
static sc_status set_incident_builtin(sc_prob *p, int beam, double w0, double pol_angle, const double *spectrum,
                                      int consistent, int n_modes, const char *who)
{
    if (!p->has_mirror || p->k.empty()) return fail(SC_E_STATE, "%s: set mirror and frequencies first", who);
    if (spectrum)
        for (size_t i = 0; i < 2 * p->k.size(); ++i)
            if (!std::isfinite(spectrum[i])) return fail(SC_E_INVAL, "%s: spectrum[%zu] is not finite", who, i / 2);
    hipStream_t st = p->ctx->stream;
    const int n_k = (int)p->k.size();
    invalidate_tables(p);
    SC_TRY(p->tab64.reserve(sizeof(double) * 8 * (size_t)n_k * p->n_tot, p->alloc_stream));
    const double *dspec = nullptr;
    if (spectrum) {
        double *h = nullptr;
        bool ext = false;
        SC_TRY(stage_area(p, p->h_stage_spec, 2 * (size_t)n_k, &h, &ext));
        std::copy(spectrum, spectrum + 2 * (size_t)n_k, h);
        SC_TRY(p->d_spec.reserve(sizeof(double) * 2 * n_k, p->alloc_stream));
        HIP_TRY(hipMemcpyAsync(p->d_spec.p, h, sizeof(double) * 2 * n_k, hipMemcpyHostToDevice, st));
        if (!ext) SC_TRY(staging_mark(p));
        dspec = p->d_spec.as<double>();
    }
    const double *modes = beam == 3 ? p->d_modes.as<double>() : nullptr;
    ev_record(p, EV_PREP0);
    HIP_TRY(launch_tables_gaussian(st, n_k, p->n_surf, p->n_tot, p->d_k.as<double>(), p->pos64.as<double>(),
                                   p->nrm.as<double>(), p->wgt.as<double>(), p->tan.as<double>(), beam, w0, pol_angle,
                                   dspec, consistent ? 1 : 0, modes, n_modes, p->tab64.as<double>()));
    SC_TRY(reserve_power(p));
    HIP_TRY(launch_power_gaussian(st, n_k, p->n_surf, p->d_k.as<double>(), p->pos64.as<double>(),
                                  p->nrm.as<double>(), p->wgt.as<double>(), beam, w0, pol_angle, dspec,
                                  consistent ? 1 : 0, modes, n_modes, p->d_power.as<double>() + n_k,
                                  p->d_power.as<double>()));
    p->has_power = true;
    ev_record(p, EV_PREP1);
    p->ev_prep = p->ctx->profiling;
    return finish_tables(p);
}

extern "C" sc_status sc_set_incident_beam(sc_prob *p, int beam, double w0, double pol_angle, const double *spectrum,
                                          int consistent)
{
    if (!p) return fail(SC_E_INVAL, "sc_set_incident_beam: prob is NULL");
    if (beam != SC_BEAM_LINEAR && beam != SC_BEAM_RADIAL && beam != SC_BEAM_AZIMUTHAL)
        return fail(SC_E_INVAL, "sc_set_incident_beam: unknown beam %d", beam);
    if (!(w0 > 0.0)) return fail(SC_E_INVAL, "sc_set_incident_beam: w0 must be > 0");
    if (beam != SC_BEAM_LINEAR && !std::isfinite(w0))
        return fail(SC_E_INVAL, "sc_set_incident_beam: a radially or azimuthally polarised beam needs a finite w0");
    if (!std::isfinite(pol_angle)) return fail(SC_E_INVAL, "sc_set_incident_beam: bad polarisation angle");
    DeviceGuard g(p->ctx->device);
    return set_incident_builtin(p, beam, w0, pol_angle, spectrum, consistent, 0, "sc_set_incident_beam");
}

extern "C" sc_status sc_set_incident_lg(sc_prob *p, const sc_lg_mode *modes, int n_modes, double w0,
                                        const double *spectrum)
{
    if (!p || !modes) return fail(SC_E_INVAL, "sc_set_incident_lg: NULL argument");
    if (n_modes < 1 || n_modes > SC_MAX_LG_MODES)
        return fail(SC_E_INVAL, "sc_set_incident_lg: need 1 <= n_modes <= %d", SC_MAX_LG_MODES);
    if (!(w0 > 0.0) || !std::isfinite(w0)) return fail(SC_E_INVAL, "sc_set_incident_lg: w0 must be finite and > 0");
    for (int m = 0; m < n_modes; ++m) {
        const sc_lg_mode &md = modes[m];
        if (md.p < 0 || md.p > SC_MAX_LG_INDEX || md.l < -SC_MAX_LG_INDEX || md.l > SC_MAX_LG_INDEX)
            return fail(SC_E_INVAL, "sc_set_incident_lg: mode %d: need 0 <= p <= %d and |l| <= %d", m,
                        SC_MAX_LG_INDEX, SC_MAX_LG_INDEX);
        if (!std::isfinite(md.ex[0]) || !std::isfinite(md.ex[1]) || !std::isfinite(md.ey[0]) ||
            !std::isfinite(md.ey[1]))
            return fail(SC_E_INVAL, "sc_set_incident_lg: mode %d: amplitudes must be finite", m);
    }
    if (!p->has_mirror || p->k.empty()) return fail(SC_E_STATE, "sc_set_incident_lg: set mirror and frequencies first");
    DeviceGuard g(p->ctx->device);
    // per mode: p, l, ex (re, im), ey (re, im) and the normalisation
    // C = sqrt(2 p! / (pi (p + |l|)!)) / w0, which does not depend on the position
    double *h = nullptr;
    bool ext = false;
    SC_TRY(stage_area(p, p->h_stage_modes, SC_LG_RECORD * (size_t)n_modes, &h, &ext));
    for (int m = 0; m < n_modes; ++m) {
        double *d = h + SC_LG_RECORD * m;
        const int al = modes[m].l < 0 ? -modes[m].l : modes[m].l;
        d[0] = modes[m].p;
        d[1] = modes[m].l;
        d[2] = modes[m].ex[0];
        d[3] = modes[m].ex[1];
        d[4] = modes[m].ey[0];
        d[5] = modes[m].ey[1];
        d[6] = std::sqrt(2.0 * std::exp(std::lgamma(modes[m].p + 1.0) - std::lgamma(modes[m].p + al + 1.0)) / M_PI) / w0;
        d[7] = 0.0;
    }
    SC_TRY(p->d_modes.reserve(sizeof(double) * SC_LG_RECORD * (size_t)n_modes, p->alloc_stream));
    HIP_TRY(hipMemcpyAsync(p->d_modes.p, h, sizeof(double) * SC_LG_RECORD * (size_t)n_modes, hipMemcpyHostToDevice,
                           p->ctx->stream));
    if (!ext) SC_TRY(staging_mark(p));
    return set_incident_builtin(p, 3, w0, 0.0, spectrum, 0, n_modes, "sc_set_incident_lg");
}

extern "C" sc_status sc_set_incident_gaussian(sc_prob *p, double w0, double pol_angle, const double *spectrum,
                                              int consistent)
{
    return sc_set_incident_beam(p, SC_BEAM_LINEAR, w0, pol_angle, spectrum, consistent);
}

extern "C" sc_status sc_get_incident_power(const sc_prob *p, double *P)
{
    if (!p || !P) return fail(SC_E_INVAL, "sc_get_incident_power: NULL argument");
    if (!p->has_power) return fail(SC_E_STATE, "sc_get_incident_power: no incident field set");
    DeviceGuard g(p->ctx->device);
    HIP_TRY(hipStreamSynchronize(p->ctx->stream));
    HIP_TRY(hipMemcpy(P, p->d_power.p, sizeof(double) * p->k.size(), hipMemcpyDeviceToHost));
    return SC_OK;
}

// Multiply frequency n of the tables by fac[n] (complex, host) and its power by |fac[n]|^2.
static sc_status scale_tables(sc_prob *p, const std::vector<double> &fac)
{
    SC_TRY(settle_factoring(p));
    hipStream_t st = p->ctx->stream;
    const int n_k = (int)p->k.size();
    DevBuf dfac;
    SC_TRY(dfac.reserve(sizeof(double) * 2 * n_k, p->alloc_stream));
    HIP_TRY(hipMemcpyAsync(dfac.p, fac.data(), sizeof(double) * 2 * n_k, hipMemcpyHostToDevice, st));
    if (p->has_tab64) {
        HIP_TRY(launch_tables_scale(st, n_k, p->n_tot, 4, dfac.as<double>(), p->tab64.as<double>(), nullptr));
        p->tab32_ok = false;   // rebuilt from the scaled FP64 tables when needed
        p->fact_checked = p->fact_ok = p->fact64_ok = p->tie_ok = p->tie64_ok = false;
        p->fact32_built = p->fact64_built = false;
        p->fact_pending = false;
    } else {
        if (p->tab32_ok)
            HIP_TRY(launch_tables_scale(st, n_k, p->n_tot, 4, dfac.as<double>(), nullptr, p->tab32.as<float>()));
        if (p->fact32_built) {   // a factor per frequency keeps the direction: scale s and rho_t
            HIP_TRY(launch_tables_scale(st, n_k, p->n_tot, 2, dfac.as<double>(), nullptr, p->tabf.as<float>()));
            HIP_TRY(launch_tables_polar(st, (int64_t)n_k * p->n_tot, p->tabf.as<float>(), p->tabp.as<float>()));
        }
    }
    p->tab32n_ok = false;
    p->res_prec = -1;
    std::vector<double> P(n_k);
    HIP_TRY(hipMemcpyAsync(P.data(), p->d_power.p, sizeof(double) * n_k, hipMemcpyDeviceToHost, st));
    HIP_TRY(hipStreamSynchronize(st));   // fac and P are host memory, dfac is freed on return
    for (int i = 0; i < n_k; ++i) P[i] *= fac[2 * i] * fac[2 * i] + fac[2 * i + 1] * fac[2 * i + 1];
    HIP_TRY(hipMemcpy(p->d_power.p, P.data(), sizeof(double) * n_k, hipMemcpyHostToDevice));
    return SC_OK;
}

extern "C" sc_status sc_scale_spectrum(sc_prob *p, const double *factor)
{
    if (!p || !factor) return fail(SC_E_INVAL, "sc_scale_spectrum: NULL argument");
    if (!p->has_tab || !p->has_power) return fail(SC_E_STATE, "sc_scale_spectrum: set the incident field first");
    const int n_k = (int)p->k.size();
    for (int i = 0; i < 2 * n_k; ++i)
        if (!std::isfinite(factor[i])) return fail(SC_E_INVAL, "sc_scale_spectrum: factor[%d] is not finite", i / 2);
    DeviceGuard g(p->ctx->device);
    return scale_tables(p, std::vector<double>(factor, factor + 2 * n_k));
}

extern "C" sc_status sc_normalize_energy(sc_prob *p, const double *eps, double e_tot, double dk)
{
    if (!p || !eps) return fail(SC_E_INVAL, "sc_normalize_energy: NULL argument");
    if (!p->has_tab || !p->has_power) return fail(SC_E_STATE, "sc_normalize_energy: set the incident field first");
    const int n_k = (int)p->k.size();
    if (!std::isfinite(e_tot) || e_tot < 0.0) return fail(SC_E_INVAL, "sc_normalize_energy: e_tot must be >= 0");
    if (e_tot > 0.0 && !(dk > 0.0 && std::isfinite(dk)))
        return fail(SC_E_INVAL, "sc_normalize_energy: dk must be > 0 when e_tot is given");
    double sum = 0.0;
    for (int i = 0; i < n_k; ++i) {
        if (!(eps[i] >= 0.0) || !std::isfinite(eps[i]))
            return fail(SC_E_INVAL, "sc_normalize_energy: eps[%d] = %g is not a power (>= 0)", i, eps[i]);
        sum += eps[i];
    }
    if (e_tot > 0.0 && !(sum > 0.0)) return fail(SC_E_INVAL, "sc_normalize_energy: eps is zero everywhere");
    const double scale = e_tot > 0.0 ? e_tot / (sum * dk) : 1.0;   // sum_n eps_n dk = e_tot
    DeviceGuard g(p->ctx->device);
    std::vector<double> P(n_k);
    HIP_TRY(hipStreamSynchronize(p->ctx->stream));
    HIP_TRY(hipMemcpy(P.data(), p->d_power.p, sizeof(double) * n_k, hipMemcpyDeviceToHost));
    std::vector<double> fac(2 * (size_t)n_k, 0.0);
    for (int i = 0; i < n_k; ++i) {
        const double target = eps[i] * scale;
        if (target == 0.0) continue;   // a component with no energy is removed
        if (!(P[i] > 0.0))
            return fail(SC_E_INVAL, "sc_normalize_energy: the incident field carries no power at k[%d]", i);
        fac[2 * i] = std::sqrt(target / P[i]);   // E_0^n, eq. normalizationAmplitude
    }
    return scale_tables(p, fac);
}

extern "C" sc_status sc_set_observation(sc_prob *p, const double *xyz, int n_obs, int on_device)
{
    if (!p || !xyz) return fail(SC_E_INVAL, "sc_set_observation: NULL argument");
    if (n_obs < 1) return fail(SC_E_INVAL, "sc_set_observation: n_obs must be >= 1");
    if (!on_device) {
        for (int o = 0; o < n_obs; ++o)
            for (int c = 0; c < 3; ++c)
                if (!std::isfinite(xyz[3 * (size_t)o + c]))
                    return fail(SC_E_INVAL, "sc_set_observation: point %d is not finite", o);
    }
    DeviceGuard g(p->ctx->device);
    hipStream_t st = p->ctx->stream;
    const int pad = (int)round_up((size_t)n_obs, OBS_PAD);
    p->res_prec = -1;
    SC_TRY(p->obs64.reserve(sizeof(double) * 4 * pad, p->alloc_stream));
    SC_TRY(p->obs32.reserve(sizeof(float) * 4 * pad, p->alloc_stream));
    const double *d = xyz;
    p->obs_r2max = -1.0;
    double r2max = -1.0;
    if (!on_device) {
        for (int o = 0; o < n_obs; ++o) {
            const double *q = xyz + 3 * (size_t)o;
            r2max = std::max(r2max, q[0] * q[0] + q[1] * q[1] + q[2] * q[2]);
        }
        double *h = nullptr;
        bool ext = false;
        SC_TRY(stage_area(p, p->h_stage_obs, 3 * (size_t)n_obs, &h, &ext));
        std::copy(xyz, xyz + 3 * (size_t)n_obs, h);
        SC_TRY(p->d_obs_in.reserve(sizeof(double) * 3 * n_obs, p->alloc_stream));
        HIP_TRY(hipMemcpyAsync(p->d_obs_in.p, h, sizeof(double) * 3 * n_obs, hipMemcpyHostToDevice, st));
        if (!ext) SC_TRY(staging_mark(p));
        d = p->d_obs_in.as<double>();
    }
    HIP_TRY(launch_obs_prep(st, d, n_obs, pad, p->obs64.as<double>(), p->obs32.as<float>()));
    p->obs_r2max = r2max;
    p->n_obs = n_obs;
    p->n_obs_pad = pad;
    return SC_OK;
}

// ============================================================ launch shapes

// The library's launch: one point per lane, frequencies per lane by table layout (0 here, settled in
// resolve_launch), 4 waves per workgroup, node chunks of 2048, as many workgroups as fit.
static sc_launch default_launch(sc_precision prec)
{
    (void)prec;
    sc_launch l{};
    l.obs_per_lane = 1;
    l.freq_per_lane = 0;
    l.waves_per_block = 4;
    l.chunk = 2048;
    l.blocks_per_cu = 0;   // 0 = occupancy limit
    return l;
}

// Whether an evaluation of p in prec reads the factored tables, as far as the problem knows now
// (the factoring test runs when the incident field is set).
static bool uses_factored(const sc_prob *p, sc_precision prec)
{
    if (!p->allow_fact || !p->fact_checked) return false;
    if (prec == SC_FP32_SPLIT) return p->fact_ok;
    if (prec == SC_FP64) return p->fact64_ok;
    return false;
}

// The same for the factored layout with the charge tied to the current.
static bool uses_tied(const sc_prob *p, sc_precision prec)
{
    if (!uses_factored(p, prec) || !p->allow_tie) return false;
    return prec == SC_FP64 ? p->tie64_ok : p->tie_ok;
}

// Frequencies per lane by table layout: with the factored current a frequency costs 37 vector
// instructions against the 30 of the geometry it shares, so four per lane (at five waves per SIMD)
// beat two; the general tables' longer per-frequency work does not pay for the registers.
static int auto_freq_per_lane(sc_precision prec, bool fact) { return prec != SC_FP64 && fact ? 4 : 2; }

static TuneKey tune_key(const sc_prob *p, sc_precision prec)
{
    return {(int)prec, uses_tied(p, prec) ? 2 : uses_factored(p, prec) ? 1 : 0, log2_bucket(p->n_obs),
            log2_bucket((int64_t)p->k.size()), log2_bucket(p->n_tot)};
}

sc_status sc::check_launch(const sc_launch &l)
{
    if (l.obs_per_lane != 1 && l.obs_per_lane != 2) return fail(SC_E_INVAL, "launch: obs_per_lane must be 1 or 2");
    if (l.freq_per_lane != 1 && l.freq_per_lane != 2 && l.freq_per_lane != 4)
        return fail(SC_E_INVAL, "launch: freq_per_lane must be 1, 2 or 4");
    if (l.obs_per_lane * l.freq_per_lane > 4 || (l.obs_per_lane == 2 && l.freq_per_lane == 4))
        return fail(SC_E_INVAL, "launch: obs_per_lane x freq_per_lane must be 1, 2 or 4 (not 2 x 4)");
    if (l.waves_per_block != 1 && l.waves_per_block != 2 && l.waves_per_block != 4)
        return fail(SC_E_INVAL, "launch: waves_per_block must be 1, 2 or 4");
    if (l.chunk < 64 || l.chunk % 64 != 0) return fail(SC_E_INVAL, "launch: chunk must be a positive multiple of 64");
    if (l.blocks_per_cu < 0 || l.blocks_per_cu > 64) return fail(SC_E_INVAL, "launch: blocks_per_cu out of range");
    return SC_OK;
}

sc_launch sc::resolve_launch(const sc_prob *p, sc_precision prec)
{
    sc_launch l = default_launch(prec);
    auto it = p->ctx->tune.find(tune_key(p, prec));
    if (it != p->ctx->tune.end()) l = it->second;
    if (p->has_launch) {
        if (p->launch.obs_per_lane) l.obs_per_lane = p->launch.obs_per_lane;
        if (p->launch.waves_per_block) l.waves_per_block = p->launch.waves_per_block;
        if (p->launch.chunk) l.chunk = p->launch.chunk;
        if (p->launch.blocks_per_cu) l.blocks_per_cu = p->launch.blocks_per_cu;
        if (p->launch.freq_per_lane) l.freq_per_lane = p->launch.freq_per_lane;
    }
    if (l.freq_per_lane == 0) l.freq_per_lane = auto_freq_per_lane(prec, uses_factored(p, prec));
    if (l.obs_per_lane * l.freq_per_lane > 4 || (l.obs_per_lane == 2 && l.freq_per_lane == 4))
        l.freq_per_lane = 4 / (2 * l.obs_per_lane);   // 2 points per lane: at most 2 frequencies
    return l;
}

extern "C" sc_status sc_set_launch(sc_prob *p, const sc_launch *l)
{
    if (!p) return fail(SC_E_INVAL, "sc_set_launch: prob is NULL");
    if (!l) {
        p->has_launch = false;
        return SC_OK;
    }
    sc_launch full = default_launch(SC_FP32_SPLIT);
    full.freq_per_lane = 1;   // a shape left to the library is always valid: check the rest with 1
    if (l->obs_per_lane) full.obs_per_lane = l->obs_per_lane;
    if (l->waves_per_block) full.waves_per_block = l->waves_per_block;
    if (l->chunk) full.chunk = l->chunk;
    if (l->freq_per_lane) full.freq_per_lane = l->freq_per_lane;
    full.blocks_per_cu = l->blocks_per_cu;
    SC_TRY(check_launch(full));
    p->launch = *l;
    p->has_launch = true;
    return SC_OK;
}

extern "C" sc_status sc_get_launch(const sc_prob *p, sc_precision prec, sc_launch *out)
{
    if (!p || !out) return fail(SC_E_INVAL, "sc_get_launch: NULL argument");
    if (prec != SC_FP64 && prec != SC_FP32_SPLIT && prec != SC_FP32)
        return fail(SC_E_INVAL, "sc_get_launch: unknown precision %d", (int)prec);
    {
        DeviceGuard g(p->ctx->device);
        SC_TRY(settle_factoring(const_cast<sc_prob *>(p)));   // the layout decides the default shape
    }
    *out = resolve_launch(p, prec);
    return SC_OK;
}

// ====================================================================== evaluate

int sc::mode_of(sc_precision prec)
{
    return prec == SC_FP64 ? MODE_FP64 : (prec == SC_FP32_SPLIT ? MODE_SPLIT : MODE_NAIVE);
}

size_t sc::real_size(sc_precision prec) { return prec == SC_FP64 ? sizeof(double) : sizeof(float); }

// The tables an evaluation in `prec` reads: with `build`, built first where missing (which may
// allocate); without, SC_E_STATE if they are not there yet.  *fact: the factored layout.
static sc_status select_tables(sc_prob *p, sc_precision prec, bool build, const void **tab, bool *fact)
{
    if (prec != SC_FP64 && prec != SC_FP32_SPLIT && prec != SC_FP32)
        return fail(SC_E_INVAL, "evaluate: unknown precision %d", (int)prec);
    if (!p->has_mirror || p->k.empty() || !p->has_tab || p->n_obs < 1)
        return fail(SC_E_STATE, "evaluate: mirror, frequencies, incident field and observation points are required");
    if (prec == SC_FP64 && !p->has_tab64)
        return fail(SC_E_STATE, "evaluate: FP64 tables were not kept (sc_set_table_storage(p, 0))");
    if (prec != SC_FP64 && !p->tab32_ok && !p->has_tab64 &&
        !(prec == SC_FP32_SPLIT && p->allow_fact && p->fact32_built))
        return fail(SC_E_STATE, "evaluate: no tables to build the FP32 tables from");
    static const char *not_built = "evaluate without allocation: the tables of this precision are not built yet "
                                   "(evaluate the problem once with sc_evaluate first)";
    hipStream_t st = p->ctx->stream;
    const int n_k = (int)p->k.size();
    const size_t nrec = (size_t)n_k * p->n_tot;
    *fact = false;
    if ((prec == SC_FP32_SPLIT || prec == SC_FP64) && p->allow_fact) {
        const bool is64 = prec == SC_FP64;
        if (build) {
            SC_TRY(ensure_factored(p, !is64, is64));
        } else if (p->has_tab64 && !(p->fact_checked && (is64 ? (!p->fact64_ok || p->fact64_built)
                                                              : (!p->fact_ok || p->fact32_built)))) {
            return fail(SC_E_STATE, "%s", not_built);
        }
        *fact = is64 ? p->fact64_built : p->fact32_built;
    }
    if (*fact) {
        *tab = prec == SC_FP64 ? p->tabf64.p : p->tabf.p;
    } else if (prec == SC_FP32_SPLIT) {
        if (!p->tab32_ok) {
            if (!build) return fail(SC_E_STATE, "%s", not_built);
            SC_TRY(p->tab32.reserve(sizeof(float) * 8 * nrec, p->alloc_stream));
            HIP_TRY(launch_tables_cast(st, n_k, p->n_tot, p->d_k.as<double>(), p->pos64.as<double>(),
                                       p->tab64.as<double>(), nullptr, p->tab32.as<float>(), 0));
            p->tab32_ok = true;
        }
        *tab = p->tab32.p;
    } else if (prec == SC_FP32) {
        if (!p->tab32n_ok) {
            if (!build) return fail(SC_E_STATE, "%s", not_built);
            SC_TRY(p->tab32n.reserve(sizeof(float) * 8 * nrec, p->alloc_stream));
            HIP_TRY(launch_tables_cast(st, n_k, p->n_tot, p->d_k.as<double>(), p->pos64.as<double>(),
                                       p->has_tab64 ? p->tab64.as<double>() : nullptr, p->tab32.as<float>(),
                                       p->tab32n.as<float>(), 1));
            p->tab32n_ok = true;
        }
        *tab = p->tab32n.p;
    } else {
        *tab = p->tab64.p;
    }
    return SC_OK;
}

// The quadrature job of one problem (no allocation): tables `tab` of the chosen layout, split-K
// partials in `partial` ([n_chunks][n_k][12][n_obs_pad] reals of the precision).
static void fill_job(const sc_prob *p, sc_precision prec, const sc_launch &l, const void *tab, bool fact,
                     void *partial, QuadJob &job)
{
    const int n_k = (int)p->k.size();
    const int n_chunks = (p->n_tot + l.chunk - 1) / l.chunk;
    job.tab = tab;
    job.pos = prec == SC_FP64 ? (fact ? p->posf64.p : p->pos64.p) : (fact ? p->posf.p : p->pos32.p);
    job.factored = fact ? 1 : 0;
    job.tied = fact && p->allow_tie && (prec == SC_FP64 ? p->tie64_ok : p->tie_ok) ? 1 : 0;
    job.beta = job.tied ? (prec == SC_FP64 ? p->betaf64.p : p->betaf.p) : nullptr;
    job.tabp = job.tied && prec != SC_FP64 ? p->tabp.p : nullptr;
    // |delta| = ||R| - |r_s|| <= |r'|, so the split phase k delta stays below k_max |r'|_max; the
    // hardware sin / cos take up to 256 turns directly (kept below 250 for the FP32 rounding of k delta;
    // the tied charge adds the phase of s, at most half a turn)
    {
        const double kmax = *std::max_element(p->k.begin(), p->k.end());
        const double tmax = p->obs_r2max >= 0.0 ? kmax / (2.0 * M_PI) * std::sqrt(p->obs_r2max) : 1e300;
        job.raw_phase = prec == SC_FP32_SPLIT && tmax < 250.0 ? 1 : 0;
    }
    // delta = (|r'|^2 - 2 r_s.r') / (|R| + |r_s|) by its series in x = delta_1 / (2|r_s|), where
    // |x| <= |r'| / (2|r_s|) <= 2e-4 keeps the truncation (5 x^3, relative) far below FP32 rounding
    // (1 / (2|r_s|) rides in the factored node records, or in hinv32); per job, like the phase path
    job.hinv = prec == SC_FP64 ? p->hinv64.p : p->hinv32.p;
    job.series_delta = (prec == SC_FP32_SPLIT || prec == SC_FP64) && p->rs_min > 0.0 && p->obs_r2max >= 0.0 &&
                               std::sqrt(p->obs_r2max) <= 4e-4 * p->rs_min
                           ? 1
                           : 0;
    job.obs = prec == SC_FP64 ? p->obs64.p : p->obs32.p;
    job.k = p->d_k.as<double>();
    job.partial = partial;
    job.n_tot = p->n_tot;
    job.n_obs_pad = p->n_obs_pad;
    job.n_k = n_k;
    job.chunk = l.chunk;
    job.n_chunks = n_chunks;
    job.obs_blocks = p->n_obs_pad / (64 * l.obs_per_lane);
    job.tile0 = 0;
    job.tile_offset = 0;
    job.n_tiles = (int64_t)job.obs_blocks * n_chunks * ((n_k + l.freq_per_lane - 1) / l.freq_per_lane);
}

// Bytes of the split-K partials of an evaluation of p with launch l.
static size_t partial_bytes(const sc_prob *p, sc_precision prec, const sc_launch &l)
{
    const size_t n_chunks = ((size_t)p->n_tot + l.chunk - 1) / l.chunk;
    return real_size(prec) * 12 * n_chunks * p->k.size() * (size_t)p->n_obs_pad;
}

// Make sure the tables of precision `prec` exist; size the partial and result buffers.
sc_status sc::prepare(sc_prob *p, sc_precision prec, const sc_launch &l, QuadJob &job)
{
    const void *tab = nullptr;
    bool fact = false;
    SC_TRY(select_tables(p, prec, true, &tab, &fact));
    const size_t rs = real_size(prec);
    const int n_k = (int)p->k.size();
    SC_TRY(p->partial.reserve(partial_bytes(p, prec, l), p->alloc_stream));
    SC_TRY(p->resE.reserve(rs * 6 * (size_t)n_k * p->n_obs, p->alloc_stream));
    SC_TRY(p->resB.reserve(rs * 6 * (size_t)n_k * p->n_obs, p->alloc_stream));
    fill_job(p, prec, l, tab, fact, p->partial.p, job);
    return SC_OK;
}

size_t sc::footprint_bytes(int n_r, int n_phi, int n_k, int n_obs, int n_t, sc_precision prec, int chunk)
{
    const size_t n_tot = (size_t)(n_r + 1) * n_phi;
    const size_t pad = round_up((size_t)n_obs, OBS_PAD);
    const size_t rs = real_size(prec);
    const size_t n_chunks = (n_tot + chunk - 1) / chunk;
    size_t b = 0;
    b += sizeof(double) * (2 * (size_t)n_r + 1 + 2 * (size_t)n_phi + 3 * (size_t)n_phi);   // 1-D rule, rim tangents
    b += n_tot * (sizeof(double) * (4 + 3 + 1 + 1) + sizeof(float) * 5);                    // node records
    b += sizeof(double) * n_k;
    b += sizeof(double) * (size_t)n_k * (1 + (size_t)power_partial_count(1));                // incident power
    // FP64 tables (kept for SC_FP64; for the FP32 forms they exist only while the FP32 tables are cast)
    b += (size_t)n_k * n_tot * sizeof(double) * 8;
    if (prec != SC_FP64) b += (size_t)n_k * n_tot * sizeof(float) * 8;                      // FP32 tables
    if (prec == SC_FP32_SPLIT)                                                               // factored tables
        b += (size_t)n_k * n_tot * sizeof(float) * 6 + n_tot * sizeof(float) * 9;
    if (prec == SC_FP64) b += (size_t)n_k * n_tot * sizeof(double) * 4 + n_tot * sizeof(double) * 9;
    b += pad * (sizeof(double) + sizeof(float)) * 4;                                        // observation records
    b += sizeof(double) * (2 * (size_t)n_k + 3 * (size_t)n_obs);                             // upload staging
    b += rs * 12 * (size_t)n_k * n_obs;                                                      // results E, B
    b += rs * 12 * n_chunks * (size_t)n_k * pad;                                             // split-K partials
    if (n_t > 0) b += sizeof(double) * ((size_t)n_t + 2 * (size_t)n_t * n_k) + rs * 12 * (size_t)n_t * n_obs;
    return b;
}

// Workgroups of a persistent quadrature launch: the resident limit (or the launch's blocks per CU)
// on every CU, but no more than the tiles need (one wave per tile).
static int quad_grid(const sc_ctx *c, sc_precision prec, const sc_launch &l, int64_t n_tiles)
{
    int bpc = l.blocks_per_cu;
    const int occ = quad_max_blocks_per_cu(mode_of(prec), l.obs_per_lane, l.freq_per_lane, l.waves_per_block);
    if (bpc <= 0 || bpc > occ) bpc = occ;
    int64_t grid = (int64_t)bpc * c->n_cu;
    const int64_t blocks_needed = (n_tiles + l.waves_per_block - 1) / l.waves_per_block;
    if (grid > blocks_needed) grid = blocks_needed;
    return (int)std::max<int64_t>(grid, 1);
}

// Upload jobs and run one persistent quadrature launch over all their tiles.
sc_status sc::run_quad(sc_ctx *c, std::vector<QuadJob> &jobs, sc_precision prec, const sc_launch &l,
                          sc_prob *timed)
{
    hipStream_t st = c->stream;
    int64_t n_tiles = 0;
    for (auto &j : jobs) {
        j.tile0 = n_tiles;
        n_tiles += j.n_tiles;
    }
    if (n_tiles >= (1LL << 31) - (1LL << 24)) return fail(SC_E_UNSUPPORTED, "evaluate: too many tiles (%lld)",
                                                           (long long)n_tiles);
    SC_TRY(c->jobs.reserve(sizeof(QuadJob) * jobs.size()));
    // the previous upload from host_jobs must have completed before it is overwritten
    HIP_TRY(hipEventSynchronize(c->upload_done));
    c->host_jobs = jobs;
    HIP_TRY(hipMemcpyAsync(c->jobs.p, c->host_jobs.data(), sizeof(QuadJob) * jobs.size(), hipMemcpyHostToDevice,
                           st));
    HIP_TRY(hipEventRecord(c->upload_done, st));
    HIP_TRY(launch_fill_u32(st, c->counter.as<unsigned int>(), 0u, QUAD_SEGMENTS));
    const int grid = quad_grid(c, prec, l, n_tiles);
    if (timed) ev_record(timed, EV_Q0);
    HIP_TRY(launch_quad(st, mode_of(prec), l.obs_per_lane, l.freq_per_lane, l.waves_per_block, grid,
                        c->jobs.as<QuadJob>(), (int)jobs.size(), n_tiles, c->counter.as<unsigned int>()));
    if (timed) ev_record(timed, EV_Q1);
    return SC_OK;
}

static sc_status copy_out(sc_prob *p, void *E, void *B, int on_device, size_t bytes)
{
    hipStream_t st = p->ctx->stream;
    const hipMemcpyKind kind = on_device ? hipMemcpyDeviceToDevice : hipMemcpyDeviceToHost;
    if (E) HIP_TRY(hipMemcpyAsync(E, p->resE.p, bytes, kind, st));
    if (B) HIP_TRY(hipMemcpyAsync(B, p->resB.p, bytes, kind, st));
    if (!on_device && (E || B)) HIP_TRY(hipStreamSynchronize(st));
    return SC_OK;
}

extern "C" sc_status sc_evaluate(sc_prob *p, sc_precision prec, void *E, void *B, int on_device)
{
    if (!p) return fail(SC_E_INVAL, "sc_evaluate: prob is NULL");
    DeviceGuard g(p->ctx->device);
    SC_TRY(settle_factoring(p));
    const sc_launch l = resolve_launch(p, prec);
    SC_TRY(check_launch(l));
    QuadJob job{};
    SC_TRY(prepare(p, prec, l, job));
    std::vector<QuadJob> jobs{job};
    p->res_prec = -1;
    SC_TRY(run_quad(p->ctx, jobs, prec, l, p));
    HIP_TRY(launch_reduce(p->ctx->stream, mode_of(prec), p->partial.p, job.n_chunks, job.n_k, p->n_obs,
                          p->n_obs_pad, p->d_k.as<double>(), job.tied, p->resE.p, p->resB.p));
    ev_record(p, EV_R1);
    p->ev_quad = p->ctx->profiling;
    p->res_prec = (int)prec;
    p->last_evals = (int64_t)p->n_obs * job.n_k * p->n_surf;
    p->last_tiles = job.n_tiles;
    p->last_chunk = l.chunk;
    return copy_out(p, E, B, on_device, real_size(prec) * 6 * (size_t)job.n_k * p->n_obs);
}

// ------------------------------------------------------- evaluation without allocation
// A statically allocated device array serves sc_evaluate_noalloc as its scratch memory: the work
// counters, the job record and the split-K partials.  The array's name is a host-side stand-in;
// its device address (one copy per GPU) is looked up once per device with hipGetSymbolAddress
// when a context is created there, and only that address is handed to kernels.
static __device__ __align__(256) unsigned char scratch[SC_NOALLOC_SCRATCH_BYTES];

namespace {
constexpr int MAX_DEVICES = 64;
constexpr size_t SCRATCH_COUNTERS = 0;        // QUAD_SEGMENTS work counters
constexpr size_t SCRATCH_JOB = 256;           // one QuadJob
constexpr size_t SCRATCH_PARTIAL = 1024;      // split-K partials from here on
std::mutex scratch_mu;
void *scratch_dev[MAX_DEVICES] = {};
}  // namespace

static_assert(QUAD_SEGMENTS * sizeof(unsigned int) <= SCRATCH_JOB, "work counters overlap the job record");
static_assert(SCRATCH_JOB + sizeof(QuadJob) <= SCRATCH_PARTIAL, "job record overlaps the partials");

// Called with the device current (sc_ctx_create).
static sc_status scratch_init(int device)
{
    if (device < 0 || device >= MAX_DEVICES) return SC_OK;   // sc_evaluate_noalloc reports it
    std::lock_guard<std::mutex> lk(scratch_mu);
    if (scratch_dev[device]) return SC_OK;
    void *ptr = nullptr;
    hipError_t e = hipGetSymbolAddress(&ptr, HIP_SYMBOL(scratch));
    if (e != hipSuccess || !ptr)
        return fail(SC_E_DEVICE, "hipGetSymbolAddress(scratch) failed on device %d: %s", device, hipGetErrorString(e));
    scratch_dev[device] = ptr;
    return SC_OK;
}

extern "C" sc_status sc_evaluate_noalloc(sc_prob *p, sc_precision prec, void *E, void *B)
{
    if (!p || !E || !B) return fail(SC_E_INVAL, "sc_evaluate_noalloc: NULL argument");
    const int dev = p->ctx->device;
    void *base = nullptr;
    {
        std::lock_guard<std::mutex> lk(scratch_mu);
        if (dev >= 0 && dev < MAX_DEVICES) base = scratch_dev[dev];
    }
    if (!base) return fail(SC_E_STATE, "sc_evaluate_noalloc: no scratch memory on device %d", dev);
    DeviceGuard g(dev);
    SC_TRY(settle_factoring(p));   // only a problem of the serving loop can have a test pending
    const sc_launch l = resolve_launch(p, prec);
    SC_TRY(check_launch(l));
    const void *tab = nullptr;
    bool fact = false;
    SC_TRY(select_tables(p, prec, false, &tab, &fact));
    const size_t need = partial_bytes(p, prec, l);
    if (need > SC_NOALLOC_SCRATCH_BYTES - SCRATCH_PARTIAL)
        return fail(SC_E_INVAL,
                    "sc_evaluate_noalloc: the split-K partials need %zu bytes (12 x %d node chunks x %zu frequencies x "
                    "%d padded points), the scratch holds %zu",
                    need, (p->n_tot + l.chunk - 1) / l.chunk, p->k.size(), p->n_obs_pad,
                    (size_t)SC_NOALLOC_SCRATCH_BYTES - SCRATCH_PARTIAL);
    char *b = (char *)base;
    unsigned int *counter = (unsigned int *)(b + SCRATCH_COUNTERS);
    QuadJob *djob = (QuadJob *)(b + SCRATCH_JOB);
    QuadJob job{};
    fill_job(p, prec, l, tab, fact, b + SCRATCH_PARTIAL, job);
    hipStream_t st = p->ctx->stream;
    HIP_TRY(launch_store_job(st, job, djob));
    HIP_TRY(launch_fill_u32(st, counter, 0u, QUAD_SEGMENTS));
    HIP_TRY(launch_quad(st, mode_of(prec), l.obs_per_lane, l.freq_per_lane, l.waves_per_block,
                        quad_grid(p->ctx, prec, l, job.n_tiles), djob, 1, job.n_tiles, counter));
    HIP_TRY(launch_reduce(st, mode_of(prec), b + SCRATCH_PARTIAL, job.n_chunks, job.n_k, p->n_obs, p->n_obs_pad,
                          p->d_k.as<double>(), job.tied, E, B));
    return SC_OK;
}

extern "C" sc_status sc_get_result(const sc_prob *p, void *E, void *B, int on_device)
{
    if (!p) return fail(SC_E_INVAL, "sc_get_result: prob is NULL");
    if (p->res_prec < 0) return fail(SC_E_STATE, "sc_get_result: no result (evaluate first)");
    DeviceGuard g(p->ctx->device);
    return copy_out((sc_prob *)p, E, B, on_device,
                    real_size((sc_precision)p->res_prec) * 6 * p->k.size() * (size_t)p->n_obs);
}

// The kernel shape (and, from the tuner, possibly a chunk) of one batched launch: the context's
// batch launch for the precision if one is set, else the library's shape for the table layout that
// carries most of the batch's evaluations (chunk 0: each problem's own).
static sc_launch batch_launch(const sc_ctx *c, sc_prob *const *probs, int n, sc_precision prec)
{
    auto it = c->batch_tune.find((int)prec);
    if (it != c->batch_tune.end()) return it->second;
    double fact_evals = 0.0, all_evals = 0.0;
    for (int i = 0; i < n; ++i) {
        const double e = (double)probs[i]->n_obs * (double)probs[i]->k.size() * (double)probs[i]->n_tot;
        all_evals += e;
        if (uses_factored(probs[i], prec)) fact_evals += e;
    }
    sc_launch l = default_launch(prec);
    l.freq_per_lane = auto_freq_per_lane(prec, 2.0 * fact_evals > all_evals);
    l.chunk = 0;
    return l;
}

// A batch keeps its split-K partials within max(2 x the bytes of its tables read per (frequency,
// node) at 16 B, 8 GiB): the partials of one problem are 12 reals per (chunk, frequency, point),
// so many problems with many points at a small chunk would hold several times their tables.  If
// the chunks chosen so far exceed that, the problems that fix no chunk of their own take the
// smallest power-of-two chunk from 2048 up (never below their own) that fits; the result of each
// problem is then its result alone at that chunk.  Deterministic in the batch's sizes.
static void batch_fit_partials(sc_prob *const *probs, int n, sc_precision prec, std::vector<sc_launch> &ls)
{
    double table_ref = 0.0;
    for (int i = 0; i < n; ++i) table_ref += 16.0 * (double)probs[i]->k.size() * (double)probs[i]->n_tot;
    const double cap = std::max(2.0 * table_ref * (prec == SC_FP64 ? 2.0 : 1.0), 8.0 * 1073741824.0);
    auto total = [&](int floor_chunk) {
        double b = 0.0;
        for (int i = 0; i < n; ++i) {
            sc_launch l = ls[i];
            if (!(probs[i]->has_launch && probs[i]->launch.chunk)) l.chunk = std::max(l.chunk, floor_chunk);
            b += (double)partial_bytes(probs[i], prec, l);
        }
        return b;
    };
    if (total(0) <= cap) return;
    int floor_chunk = 2048;
    while (floor_chunk < (1 << 20) && total(floor_chunk) > cap) floor_chunk *= 2;
    for (int i = 0; i < n; ++i)
        if (!(probs[i]->has_launch && probs[i]->launch.chunk)) ls[i].chunk = std::max(ls[i].chunk, floor_chunk);
}

extern "C" sc_status sc_set_batch_launch(sc_ctx *c, sc_precision prec, const sc_launch *l)
{
    if (!c) return fail(SC_E_INVAL, "sc_set_batch_launch: ctx is NULL");
    if (prec != SC_FP64 && prec != SC_FP32_SPLIT && prec != SC_FP32)
        return fail(SC_E_INVAL, "sc_set_batch_launch: unknown precision %d", (int)prec);
    if (!l) {
        c->batch_tune.erase((int)prec);
        return SC_OK;
    }
    sc_launch full = *l;
    if (full.chunk == 0) full.chunk = 64;   // 0 = each problem's own chunk: check the rest
    SC_TRY(check_launch(full));
    c->batch_tune[(int)prec] = *l;
    return SC_OK;
}

extern "C" sc_status sc_evaluate_batch(sc_ctx *c, sc_prob *const *probs, int n, sc_precision prec)
{
    if (!c || (!probs && n > 0) || n < 0) return fail(SC_E_INVAL, "sc_evaluate_batch: bad arguments");
    if (n == 0) return SC_OK;
    DeviceGuard g(c->device);
    // one launch needs one obs-per-lane / waves shape: take it from the first problem
    for (int i = 0; i < n; ++i)
        if (!probs[i] || probs[i]->ctx != c) return fail(SC_E_INVAL, "sc_evaluate_batch: problem %d not on ctx", i);
    {   // the same partial buffer must not serve two jobs
        std::vector<const sc_prob *> sorted(probs, probs + n);
        std::sort(sorted.begin(), sorted.end());
        if (std::adjacent_find(sorted.begin(), sorted.end()) != sorted.end())
            return fail(SC_E_INVAL, "sc_evaluate_batch: a problem appears twice");
    }
    for (int i = 0; i < n; ++i) SC_TRY(settle_factoring(probs[i]));
    const sc_launch l0 = batch_launch(c, probs, n, prec);
    {
        sc_launch shape = l0;
        if (shape.chunk == 0) shape.chunk = 64;   // 0 = each problem's own chunk
        SC_TRY(check_launch(shape));
    }
    std::vector<QuadJob> jobs(n);
    std::vector<sc_launch> ls(n);
    for (int i = 0; i < n; ++i) {
        // one kernel shape per launch; the chunk stays per problem (it alone fixes the summation
        // order), unless the context's tuned batch launch sets one for problems that fix none
        ls[i] = resolve_launch(probs[i], prec);
        ls[i].obs_per_lane = l0.obs_per_lane;
        ls[i].freq_per_lane = l0.freq_per_lane;
        if (l0.chunk && !(probs[i]->has_launch && probs[i]->launch.chunk)) ls[i].chunk = l0.chunk;
        SC_TRY(check_launch(ls[i]));
    }
    batch_fit_partials(probs, n, prec, ls);
    for (int i = 0; i < n; ++i) {
        SC_TRY(prepare(probs[i], prec, ls[i], jobs[i]));
        probs[i]->res_prec = -1;
    }
    SC_TRY(run_quad(c, jobs, prec, l0, probs[0]));
    for (int i = 0; i < n; ++i) {
        sc_prob *p = probs[i];
        HIP_TRY(launch_reduce(c->stream, mode_of(prec), p->partial.p, jobs[i].n_chunks, jobs[i].n_k, p->n_obs,
                              p->n_obs_pad, p->d_k.as<double>(), jobs[i].tied, p->resE.p, p->resB.p));
        p->res_prec = (int)prec;
        p->last_evals = (int64_t)p->n_obs * jobs[i].n_k * p->n_surf;
        p->last_tiles = jobs[i].n_tiles;
        p->last_chunk = ls[i].chunk;
    }
    ev_record(probs[0], EV_R1);
    probs[0]->ev_quad = c->profiling;
    return SC_OK;
}

extern "C" sc_status sc_to_time_at(sc_prob *p, double dk, const double *t, int n_t, void *Et, void *Bt, int on_device)
{
    if (!p || !t) return fail(SC_E_INVAL, "sc_to_time_at: NULL argument");
    if (n_t < 1 || n_t > SC_MAX_TIMES) return fail(SC_E_INVAL, "sc_to_time_at: need 1 <= n_t <= %d", SC_MAX_TIMES);
    if (!std::isfinite(dk)) return fail(SC_E_INVAL, "sc_to_time_at: dk must be finite");
    if (p->res_prec < 0) return fail(SC_E_STATE, "sc_to_time_at: no spectral result (evaluate first)");
    DeviceGuard g(p->ctx->device);
    hipStream_t st = p->ctx->stream;
    const int n_k = (int)p->k.size();
    const int f64 = p->res_prec == SC_FP64;
    const size_t rs = f64 ? sizeof(double) : sizeof(float);
    const int64_t n_x = (int64_t)p->n_obs * 3;
    SC_TRY(p->d_t.reserve(sizeof(double) * n_t, p->alloc_stream));
    SC_TRY(p->tw.reserve(sizeof(double) * 2 * (size_t)n_t * n_k, p->alloc_stream));
    SC_TRY(p->timeE.reserve(rs * 2 * (size_t)n_t * n_x, p->alloc_stream));
    SC_TRY(p->timeB.reserve(rs * 2 * (size_t)n_t * n_x, p->alloc_stream));
    HIP_TRY(hipMemcpyAsync(p->d_t.p, t, sizeof(double) * n_t, hipMemcpyHostToDevice, st));
    ev_record(p, EV_T0);
    HIP_TRY(launch_twiddles(st, n_k, p->d_k.as<double>(), n_t, p->d_t.as<double>(), dk, p->tw.as<double>()));
    HIP_TRY(launch_time(st, f64, n_k, n_t, n_x, p->tw.as<double>(), p->resE.p, p->timeE.p));
    HIP_TRY(launch_time(st, f64, n_k, n_t, n_x, p->tw.as<double>(), p->resB.p, p->timeB.p));
    ev_record(p, EV_T1);
    p->ev_time = p->ctx->profiling;
    const size_t bytes = rs * 2 * (size_t)n_t * n_x;
    const hipMemcpyKind kind = on_device ? hipMemcpyDeviceToDevice : hipMemcpyDeviceToHost;
    if (Et) HIP_TRY(hipMemcpyAsync(Et, p->timeE.p, bytes, kind, st));
    if (Bt) HIP_TRY(hipMemcpyAsync(Bt, p->timeB.p, bytes, kind, st));
    // t was copied from pageable host memory; complete before returning
    HIP_TRY(hipStreamSynchronize(st));
    return SC_OK;
}

extern "C" sc_status sc_to_time(sc_prob *p, double t0, double dt, int n_t, void *Et, void *Bt, int on_device)
{
    if (!p) return fail(SC_E_INVAL, "sc_to_time: prob is NULL");
    if (n_t < 1 || n_t > SC_MAX_TIMES) return fail(SC_E_INVAL, "sc_to_time: need 1 <= n_t <= %d", SC_MAX_TIMES);
    if (!std::isfinite(t0) || !std::isfinite(dt)) return fail(SC_E_INVAL, "sc_to_time: t0 and dt must be finite");
    const size_t n_k = p->k.size();
    if (n_k < 2) return fail(SC_E_INVAL, "sc_to_time: needs at least two frequencies (else use sc_to_time_at)");
    // the frequency step of a uniform grid; any other grid needs sc_to_time_at with its own weights
    const double dk = (p->k[n_k - 1] - p->k[0]) / (double)(n_k - 1);
    const double kmax = std::max(std::fabs(p->k[0]), std::fabs(p->k[n_k - 1]));
    for (size_t n = 0; n < n_k; ++n)
        if (std::fabs(p->k[n] - (p->k[0] + (double)n * dk)) > 1e-12 * kmax || !(dk > 0.0))
            return fail(SC_E_INVAL, "sc_to_time: the frequencies are not uniformly spaced (use sc_to_time_at)");
    std::vector<double> t((size_t)n_t);
    for (int m = 0; m < n_t; ++m) t[m] = t0 + (double)m * dt;
    return sc_to_time_at(p, dk, t.data(), n_t, Et, Bt, on_device);
}

// ================================================================ diagnostics

extern "C" sc_status sc_stencil_points(const double *xyz, int n_pts, double h, double *out)
{
    if (!xyz || !out) return fail(SC_E_INVAL, "sc_stencil_points: NULL argument");
    if (n_pts < 1) return fail(SC_E_INVAL, "sc_stencil_points: n_pts must be >= 1");
    if (!(h > 0.0) || !std::isfinite(h)) return fail(SC_E_INVAL, "sc_stencil_points: h must be > 0");
    static const double off[4] = {-2.0, -1.0, 1.0, 2.0};
    for (int i = 0; i < n_pts; ++i) {
        double *o = out + (size_t)i * 13 * 3;
        for (int c = 0; c < 3; ++c) o[c] = xyz[3 * (size_t)i + c];
        for (int a = 0; a < 3; ++a)
            for (int j = 0; j < 4; ++j) {
                double *q = o + 3 * (1 + 4 * a + j);
                for (int c = 0; c < 3; ++c) q[c] = xyz[3 * (size_t)i + c];
                q[a] += off[j] * h;
            }
    }
    return SC_OK;
}

static sc_status check_stencil_result(const sc_prob *p, int n_pts, double h, const char *who)
{
    if (n_pts < 1) return fail(SC_E_INVAL, "%s: n_pts must be >= 1", who);
    if (!(h > 0.0) || !std::isfinite(h)) return fail(SC_E_INVAL, "%s: h must be > 0", who);
    if (p->res_prec < 0) return fail(SC_E_STATE, "%s: no spectral result (evaluate first)", who);
    if ((int64_t)p->n_obs != 13LL * n_pts)
        return fail(SC_E_STATE, "%s: the observation set has %d points, not the 13 x %d of a stencil", who, p->n_obs,
                    n_pts);
    return SC_OK;
}

extern "C" sc_status sc_maxwell_residual_freq(sc_prob *p, int n_pts, double h, double *ef)
{
    if (!p || !ef) return fail(SC_E_INVAL, "sc_maxwell_residual_freq: NULL argument");
    SC_TRY(check_stencil_result(p, n_pts, h, "sc_maxwell_residual_freq"));
    DeviceGuard g(p->ctx->device);
    hipStream_t st = p->ctx->stream;
    const int n_k = (int)p->k.size();
    const size_t cells = (size_t)n_k * n_pts;
    DevBuf work, mx, out;
    SC_TRY(work.reserve(sizeof(double) * diag_slots() * cells, p->alloc_stream));
    SC_TRY(mx.reserve(sizeof(double) * 4 * n_k, p->alloc_stream));
    SC_TRY(out.reserve(sizeof(double) * cells, p->alloc_stream));
    HIP_TRY(launch_maxwell_freq(st, p->res_prec == SC_FP64, n_k, n_pts, h, p->d_k.as<double>(), p->resE.p, p->resB.p,
                                work.as<double>(), mx.as<double>(), out.as<double>()));
    HIP_TRY(hipMemcpyAsync(ef, out.p, sizeof(double) * cells, hipMemcpyDeviceToHost, st));
    HIP_TRY(hipStreamSynchronize(st));   // scratch is freed on return
    return SC_OK;
}

// Time-domain fields of the last result at times t (host, n_t) into E, B ([n_t][n_obs][3], result type).
static sc_status time_fields(sc_prob *p, double dk, const std::vector<double> &t, DevBuf &E, DevBuf &B)
{
    hipStream_t st = p->ctx->stream;
    const int n_k = (int)p->k.size(), n_t = (int)t.size();
    const int f64 = p->res_prec == SC_FP64;
    const size_t rs = f64 ? sizeof(double) : sizeof(float);
    const int64_t n_x = (int64_t)p->n_obs * 3;
    DevBuf dt, tw;
    SC_TRY(dt.reserve(sizeof(double) * n_t, p->alloc_stream));
    SC_TRY(tw.reserve(sizeof(double) * 2 * (size_t)n_t * n_k, p->alloc_stream));
    SC_TRY(E.reserve(rs * 2 * (size_t)n_t * n_x, p->alloc_stream));
    SC_TRY(B.reserve(rs * 2 * (size_t)n_t * n_x, p->alloc_stream));
    HIP_TRY(hipMemcpyAsync(dt.p, t.data(), sizeof(double) * n_t, hipMemcpyHostToDevice, st));
    HIP_TRY(launch_twiddles(st, n_k, p->d_k.as<double>(), n_t, dt.as<double>(), dk, tw.as<double>()));
    HIP_TRY(launch_time(st, f64, n_k, n_t, n_x, tw.as<double>(), p->resE.p, E.p));
    HIP_TRY(launch_time(st, f64, n_k, n_t, n_x, tw.as<double>(), p->resB.p, B.p));
    HIP_TRY(hipStreamSynchronize(st));   // t, dt and tw go out of scope
    return SC_OK;
}

extern "C" sc_status sc_maxwell_residual_time(sc_prob *p, int n_pts, double h, const double *t, int n_t, double dt,
                                              double dk, double *et)
{
    if (!p || !t || !et) return fail(SC_E_INVAL, "sc_maxwell_residual_time: NULL argument");
    SC_TRY(check_stencil_result(p, n_pts, h, "sc_maxwell_residual_time"));
    if (n_t < 1 || 5LL * n_t > SC_MAX_TIMES)
        return fail(SC_E_INVAL, "sc_maxwell_residual_time: need 1 <= n_t <= %d", SC_MAX_TIMES / 5);
    if (!(dt > 0.0) || !std::isfinite(dt) || !std::isfinite(dk))
        return fail(SC_E_INVAL, "sc_maxwell_residual_time: dt must be > 0 and dk finite");
    DeviceGuard g(p->ctx->device);
    hipStream_t st = p->ctx->stream;
    std::vector<double> ts(5 * (size_t)n_t);
    for (int m = 0; m < n_t; ++m)
        for (int j = 0; j < 5; ++j) ts[5 * (size_t)m + j] = t[m] + (double)(j - 2) * dt;
    DevBuf E, B, work, mx, out;
    SC_TRY(time_fields(p, dk, ts, E, B));
    const size_t cells = (size_t)n_t * n_pts;
    SC_TRY(work.reserve(sizeof(double) * diag_slots() * cells, p->alloc_stream));
    SC_TRY(mx.reserve(sizeof(double) * 4 * n_t, p->alloc_stream));
    SC_TRY(out.reserve(sizeof(double) * cells, p->alloc_stream));
    HIP_TRY(launch_maxwell_time(st, p->res_prec == SC_FP64, n_t, n_pts, h, dt, E.p, B.p, work.as<double>(),
                                mx.as<double>(), out.as<double>()));
    HIP_TRY(hipMemcpyAsync(et, out.p, sizeof(double) * cells, hipMemcpyDeviceToHost, st));
    HIP_TRY(hipStreamSynchronize(st));
    return SC_OK;
}

extern "C" sc_status sc_field_energy(sc_prob *p, const double *t, int n_t, double dk, double dV, double *W)
{
    if (!p || !t || !W) return fail(SC_E_INVAL, "sc_field_energy: NULL argument");
    if (n_t < 1 || n_t > SC_MAX_FREQUENCIES)
        return fail(SC_E_INVAL, "sc_field_energy: need 1 <= n_t <= %d", SC_MAX_FREQUENCIES);
    if (!(dV > 0.0) || !std::isfinite(dV) || !std::isfinite(dk))
        return fail(SC_E_INVAL, "sc_field_energy: dV must be > 0 and dk finite");
    if (p->res_prec < 0) return fail(SC_E_STATE, "sc_field_energy: no spectral result (evaluate first)");
    DeviceGuard g(p->ctx->device);
    hipStream_t st = p->ctx->stream;
    DevBuf E, B, part, dW;
    SC_TRY(time_fields(p, dk, std::vector<double>(t, t + n_t), E, B));
    SC_TRY(part.reserve(sizeof(double) * energy_partial_count(n_t), p->alloc_stream));
    SC_TRY(dW.reserve(sizeof(double) * n_t, p->alloc_stream));
    HIP_TRY(launch_energy(st, p->res_prec == SC_FP64, n_t, p->n_obs, E.p, B.p, 0.5 * dV, part.as<double>(),
                          dW.as<double>()));
    HIP_TRY(hipMemcpyAsync(W, dW.p, sizeof(double) * n_t, hipMemcpyDeviceToHost, st));
    HIP_TRY(hipStreamSynchronize(st));
    return SC_OK;
}

extern "C" sc_status sc_get_timing(const sc_prob *p, sc_timing *out)
{
    if (!p || !out) return fail(SC_E_INVAL, "sc_get_timing: NULL argument");
    memset(out, 0, sizeof *out);
    DeviceGuard g(p->ctx->device);
    float ms = 0.f;
    if (p->ev_prep && hipEventElapsedTime(&ms, p->ev[EV_PREP0], p->ev[EV_PREP1]) == hipSuccess) out->prep_ms = ms;
    if (p->ev_quad) {
        if (hipEventElapsedTime(&ms, p->ev[EV_Q0], p->ev[EV_Q1]) == hipSuccess) out->quad_ms = ms;
        if (hipEventElapsedTime(&ms, p->ev[EV_Q1], p->ev[EV_R1]) == hipSuccess) out->reduce_ms = ms;
    }
    if (p->ev_time && hipEventElapsedTime(&ms, p->ev[EV_T0], p->ev[EV_T1]) == hipSuccess) out->time_ms = ms;
    (void)hipGetLastError();
    out->evals = p->last_evals;
    out->tiles = p->last_tiles;
    out->chunk = p->last_chunk;
    return SC_OK;
}

// Every device buffer a problem owns.
static std::vector<DevBuf *> prob_buffers(sc_prob *p)
{
    return {&p->d_r,    &p->d_wr,    &p->d_c,       &p->d_s,     &p->pos64,    &p->pos32,  &p->hinv64,
            &p->hinv32, &p->nrm,     &p->wgt,       &p->tan,     &p->d_k,      &p->tab64,  &p->tab32,
            &p->tab32n, &p->tabf,    &p->posf,      &p->betaf,   &p->tabp,     &p->tabf64, &p->posf64,
            &p->betaf64, &p->fact_flag, &p->d_power, &p->obs64,  &p->obs32,    &p->resE,   &p->resB,
            &p->partial, &p->d_t,    &p->tw,        &p->timeE,   &p->timeB,    &p->d_spec, &p->d_obs_in,
            &p->d_modes};
}

void sc::prob_free_on(sc_prob *p, hipStream_t st)
{
    for (DevBuf *b : prob_buffers(p))
        if (b->p && b->stream) b->stream = st;
}

extern "C" sc_status sc_prob_device_bytes(const sc_prob *p, size_t *bytes)
{
    if (!p || !bytes) return fail(SC_E_INVAL, "sc_prob_device_bytes: NULL argument");
    size_t s = 0;
    for (const DevBuf *b : prob_buffers(const_cast<sc_prob *>(p))) s += b->bytes;
    *bytes = s;
    return SC_OK;
}

// ================================================================== autotuner

// Candidate kernel shapes (points x frequencies per lane) of the tuner.
static const int TUNE_SHAPES[5][2] = {{1, 4}, {1, 2}, {2, 2}, {1, 1}, {2, 1}};

// Device time of the quadrature and its reduction in the last evaluation timed on p (ms).
static double timed_ms(const sc_prob *p)
{
    float ms = 0.f;
    if (hipEventElapsedTime(&ms, p->ev[EV_Q0], p->ev[EV_R1]) != hipSuccess) {
        (void)hipGetLastError();
        return 1e300;
    }
    return ms;
}

// Time `run` (best of two) for each candidate in order until the budget is spent; returns the
// index of the fastest.
template <typename Run>
static sc_status tune_loop(const std::vector<sc_launch> &cands, double budget_ms,
                           std::chrono::steady_clock::time_point t_start, Run run, int *best_i, double *best_ms)
{
    for (size_t i = 0; i < cands.size(); ++i) {
        double tmin = 1e300;
        for (int rep = 0; rep < 2; ++rep) {
            double ms = 0.0;
            SC_TRY(run(cands[i], &ms));
            tmin = std::min(tmin, ms);
        }
        if (tmin < *best_ms) {
            *best_ms = tmin;
            *best_i = (int)i;
        }
        const double spent =
            std::chrono::duration<double, std::milli>(std::chrono::steady_clock::now() - t_start).count();
        if (spent > budget_ms) break;
    }
    return SC_OK;
}

extern "C" sc_status sc_autotune(sc_prob *p, sc_precision prec, double budget_ms, sc_launch *best)
{
    if (!p) return fail(SC_E_INVAL, "sc_autotune: prob is NULL");
    DeviceGuard g(p->ctx->device);
    SC_TRY(settle_factoring(p));
    if (budget_ms <= 0) budget_ms = 20000.0;
    sc_ctx *c = p->ctx;
    const int saved_prof = c->profiling;
    const bool saved_has = p->has_launch;
    const sc_launch saved = p->launch;
    c->profiling = 1;
    auto run = [&](const sc_launch &l, double *ms) -> sc_status {
        p->launch = l;
        p->has_launch = true;
        SC_TRY(sc_evaluate(p, prec, nullptr, nullptr, 1));
        HIP_TRY(hipStreamSynchronize(c->stream));
        *ms = timed_ms(p);
        return SC_OK;
    };
    // stage 1: kernel shape and waves per workgroup at the library's chunk; stage 2: the chunk (it
    // sets the split-K partials' size and the summation order) and workgroups per CU for that shape
    const sc_launch lib = resolve_launch(p, prec);
    std::vector<sc_launch> cands;
    for (auto &sh : TUNE_SHAPES)
        for (int wpb : {4, 2, 1}) {
            sc_launch l = lib;
            l.obs_per_lane = sh[0];
            l.freq_per_lane = sh[1];
            l.waves_per_block = wpb;
            l.blocks_per_cu = 0;
            cands.push_back(l);
        }
    const auto t_start = std::chrono::steady_clock::now();
    double best_ms = 1e300;
    int bi = -1;
    sc_status st = tune_loop(cands, 0.6 * budget_ms, t_start, run, &bi, &best_ms);
    sc_launch best_l = bi >= 0 ? cands[bi] : lib;
    if (st == SC_OK && bi >= 0) {
        std::vector<sc_launch> c2;
        for (int chunk = 512; chunk <= 16384; chunk *= 2) {
            if (chunk > 2 * p->n_tot && chunk != best_l.chunk) continue;
            for (int bpc : {0, 2, 1}) {
                if (chunk == best_l.chunk && bpc == 0) continue;   // timed in stage 1
                sc_launch l = best_l;
                l.chunk = chunk;
                l.blocks_per_cu = bpc;
                c2.push_back(l);
            }
        }
        int bi2 = -1;
        st = tune_loop(c2, budget_ms, t_start, run, &bi2, &best_ms);
        if (bi2 >= 0) best_l = c2[bi2];
    }
    c->profiling = saved_prof;
    p->launch = saved;
    p->has_launch = saved_has;
    if (st != SC_OK) return st;
    c->tune[tune_key(p, prec)] = best_l;
    if (best) *best = best_l;
    return SC_OK;
}

extern "C" sc_status sc_autotune_batch(sc_ctx *c, sc_prob *const *probs, int n, sc_precision prec, double budget_ms,
                                       sc_launch *best)
{
    if (!c || !probs || n < 1) return fail(SC_E_INVAL, "sc_autotune_batch: bad arguments");
    if (prec != SC_FP64 && prec != SC_FP32_SPLIT && prec != SC_FP32)
        return fail(SC_E_INVAL, "sc_autotune_batch: unknown precision %d", (int)prec);
    DeviceGuard g(c->device);
    if (budget_ms <= 0) budget_ms = 20000.0;
    const int saved_prof = c->profiling;
    auto it = c->batch_tune.find((int)prec);
    const bool had = it != c->batch_tune.end();
    const sc_launch saved = had ? it->second : sc_launch{};
    c->profiling = 1;
    auto run = [&](const sc_launch &l, double *ms) -> sc_status {
        c->batch_tune[(int)prec] = l;
        SC_TRY(sc_evaluate_batch(c, probs, n, prec));
        HIP_TRY(hipStreamSynchronize(c->stream));
        *ms = timed_ms(probs[0]);
        return SC_OK;
    };
    c->batch_tune.erase((int)prec);
    const sc_launch lib = batch_launch(c, probs, n, prec);
    std::vector<sc_launch> cands;
    for (auto &sh : TUNE_SHAPES)
        for (int wpb : {4, 2}) {
            sc_launch l = lib;
            l.obs_per_lane = sh[0];
            l.freq_per_lane = sh[1];
            l.waves_per_block = wpb;
            cands.push_back(l);
        }
    const auto t_start = std::chrono::steady_clock::now();
    double best_ms = 1e300;
    int bi = -1;
    sc_status st = tune_loop(cands, 0.6 * budget_ms, t_start, run, &bi, &best_ms);
    sc_launch best_l = bi >= 0 ? cands[bi] : lib;
    if (st == SC_OK && bi >= 0) {
        // one chunk for the whole batch (0: each problem's own), and workgroups per CU
        std::vector<sc_launch> c2;
        for (int chunk : {0, 1024, 2048, 4096, 8192, 16384})
            for (int bpc : {0, 2}) {
                if (chunk == best_l.chunk && bpc == best_l.blocks_per_cu) continue;
                sc_launch l = best_l;
                l.chunk = chunk;
                l.blocks_per_cu = bpc;
                c2.push_back(l);
            }
        int bi2 = -1;
        st = tune_loop(c2, budget_ms, t_start, run, &bi2, &best_ms);
        if (bi2 >= 0) best_l = c2[bi2];
    }
    c->profiling = saved_prof;
    if (st != SC_OK) {
        if (had) c->batch_tune[(int)prec] = saved;
        else c->batch_tune.erase((int)prec);
        return st;
    }
    c->batch_tune[(int)prec] = best_l;
    if (best) *best = best_l;
    return SC_OK;
}

extern "C" sc_status sc_autotune_save(sc_ctx *c, const char *path)
{
    if (!c || !path) return fail(SC_E_INVAL, "sc_autotune_save: NULL argument");
    std::ofstream f(path);
    if (!f) return fail(SC_E_INVAL, "sc_autotune_save: cannot open %s", path);
    f << "# prec factored log2_obs log2_k log2_nodes obs_per_lane waves_per_block chunk blocks_per_cu "
         "freq_per_lane\n";
    for (auto &kv : c->tune)
        f << kv.first.prec << ' ' << kv.first.fact << ' ' << kv.first.b_obs << ' ' << kv.first.b_k << ' '
          << kv.first.b_nodes << ' ' << kv.second.obs_per_lane << ' ' << kv.second.waves_per_block << ' '
          << kv.second.chunk << ' ' << kv.second.blocks_per_cu << ' ' << kv.second.freq_per_lane << '\n';
    return f ? SC_OK : fail(SC_E_INVAL, "sc_autotune_save: write failed");
}

extern "C" sc_status sc_autotune_load(sc_ctx *c, const char *path)
{
    if (!c || !path) return fail(SC_E_INVAL, "sc_autotune_load: NULL argument");
    std::ifstream f(path);
    if (!f) return fail(SC_E_INVAL, "sc_autotune_load: cannot open %s", path);
    std::string line;
    std::map<TuneKey, sc_launch> m;
    while (std::getline(f, line)) {
        if (line.empty() || line[0] == '#') continue;
        std::istringstream is(line);
        TuneKey k{};
        sc_launch l{};
        if (!(is >> k.prec >> k.fact >> k.b_obs >> k.b_k >> k.b_nodes >> l.obs_per_lane >> l.waves_per_block >>
              l.chunk >> l.blocks_per_cu >> l.freq_per_lane))
            return fail(SC_E_INVAL, "sc_autotune_load: malformed line '%s'", line.c_str());
        if (check_launch(l) != SC_OK) return fail(SC_E_INVAL, "sc_autotune_load: invalid launch in '%s'", line.c_str());
        m[k] = l;
    }
    for (auto &kv : m) c->tune[kv.first] = kv.second;
    return SC_OK;
}
