// sc_host.h -- host-side objects shared by the C ABI (sc_api.cpp) and the
// serving loop (sc_serve.cpp): device buffers, contexts, problems.
#pragma once

#include <hip/hip_runtime.h>

#include <atomic>
#include <map>
#include <string>
#include <tuple>
#include <vector>

#include "sc.h"
#include "sc_internal.h"

namespace sc {

// Record a thread-local error message and return `st`.
sc_status fail(sc_status st, const char *fmt, ...) __attribute__((format(printf, 2, 3)));

#define HIP_TRY(expr)                                                                                      \
    do {                                                                                                   \
        hipError_t e_ = (expr);                                                                            \
        if (e_ != hipSuccess)                                                                              \
            return ::sc::fail(SC_E_DEVICE, "%s: %s (%s:%d)", #expr, hipGetErrorString(e_), __FILE__, __LINE__); \
    } while (0)

#define SC_TRY(expr)                \
    do {                            \
        sc_status s_ = (expr);      \
        if (s_ != SC_OK) return s_; \
    } while (0)

// Allocation hook for tests: SC_DEBUG_FAIL_ALLOC=<n> makes the n-th device
// allocation of the process report SC_E_NOMEM.
bool debug_fail_this_alloc();

// A device allocation that frees itself.  With a non-null `stream` it uses the
// stream-ordered allocator (hipMallocAsync / hipFreeAsync on that stream), so
// that freeing never waits for unrelated work on the device.
struct DevBuf {
    void *p = nullptr;
    size_t bytes = 0;
    hipStream_t stream = nullptr;
    DevBuf() = default;
    DevBuf(const DevBuf &) = delete;
    DevBuf &operator=(const DevBuf &) = delete;
    ~DevBuf() { release(); }
    void release()
    {
        if (p) {
            if (stream) (void)hipFreeAsync(p, stream);
            else (void)hipFree(p);
        }
        p = nullptr;
        bytes = 0;
    }
    // capacity >= n bytes (contents are not preserved on growth)
    sc_status reserve(size_t n, hipStream_t st = nullptr)
    {
        if (n <= bytes && p) return SC_OK;
        release();
        if (n == 0) n = 16;
        if (debug_fail_this_alloc()) return fail(SC_E_NOMEM, "injected allocation failure (%zu bytes)", n);
        hipError_t e = st ? hipMallocAsync(&p, n, st) : hipMalloc(&p, n);
        if (e != hipSuccess) {
            p = nullptr;
            (void)hipGetLastError();
            return fail(SC_E_NOMEM, "device allocation of %zu bytes failed: %s", n, hipGetErrorString(e));
        }
        bytes = n;
        stream = st;
        return SC_OK;
    }
    template <typename T>
    T *as() const
    {
        return (T *)p;
    }
};

struct DeviceGuard {
    int prev = -1;
    explicit DeviceGuard(int dev)
    {
        if (hipGetDevice(&prev) != hipSuccess) prev = -1;
        if (prev != dev) (void)hipSetDevice(dev);
    }
    ~DeviceGuard()
    {
        if (prev >= 0) (void)hipSetDevice(prev);
    }
};

// Autotuner cache key: precision, table layout (2 factored current with the tied charge, 1 factored
// current, 0 general tables) and the log2 size buckets of points, frequencies and nodes.
struct TuneKey {
    int prec, fact, b_obs, b_k, b_nodes;
    bool operator<(const TuneKey &o) const
    {
        return std::tie(prec, fact, b_obs, b_k, b_nodes) < std::tie(o.prec, o.fact, o.b_obs, o.b_k, o.b_nodes);
    }
};

enum { EV_PREP0, EV_PREP1, EV_Q0, EV_Q1, EV_R1, EV_T0, EV_T1, EV_N };

}  // namespace sc

struct sc_ctx {
    int device = 0;
    hipStream_t stream = nullptr;
    bool own_stream = false;
    int profiling = 0;
    int n_cu = 256;
    sc::DevBuf counter;   // persistent-launch work counter
    sc::DevBuf jobs;      // QuadJob array for launches
    std::vector<sc::QuadJob> host_jobs;
    hipEvent_t upload_done = nullptr;
    std::map<sc::TuneKey, sc_launch> tune;
    std::map<int, sc_launch> batch_tune;   // batched-launch shape per precision (chunk 0: per problem)
    std::map<int, std::pair<std::vector<double>, std::vector<double>>> gauss;   // Gauss-Legendre rules by order
    std::atomic<int> n_probs{0};   // live problems and servers (a context outlives them)
};

struct sc_prob {
    sc_ctx *ctx = nullptr;
    hipStream_t alloc_stream = nullptr;   // stream-ordered allocations (serving loop)
    // mirror
    bool has_mirror = false;
    double f = 0, a = 0;
    int n_r = 0, n_phi = 0, n_surf = 0, n_rim = 0, n_tot = 0;
    sc::DevBuf d_r, d_wr, d_c, d_s;          // 1-D rule (device copies)
    sc::DevBuf pos64, pos32, nrm, wgt, tan;  // node records
    sc::DevBuf hinv64, hinv32;                 // [n_tot] 1 / (2|r_s|), FP64 and FP32
    // frequencies
    std::vector<double> k;
    sc::DevBuf d_k;
    // tables (tab64 may be released after casting when keep_fp64 is off)
    bool has_tab = false, tab32_ok = false, tab32n_ok = false;
    bool keep_fp64 = true, has_tab64 = false;
    sc::DevBuf tab64, tab32, tab32n;
    // factored tables (current Jt = u s with a real direction u per node), built from tab64: the
    // test runs once per table set (fact_ok: FP32 split tolerance, fact64_ok: FP64 tolerance), the
    // FP32 (tabf, posf, betaf, and tabp: s in polar form) and FP64 (tabf64, posf64, betaf64) tables
    // are built when first needed; tie_ok, tie64_ok: the charge is tied to the current as well
    // (rho_t = -i beta s / k)
    bool allow_fact = true, allow_tie = true, fact_checked = false, fact_ok = false, fact64_ok = false;
    bool tie_ok = false, tie64_ok = false;
    bool fact32_built = false, fact64_built = false;
    sc::DevBuf tabf, posf, betaf, tabp, tabf64, posf64, betaf64, fact_flag;
    // deferred test (set by a caller that must not wait, the serving loop): the flag goes to the
    // pinned word fact_flag_host, fact_ev marks its arrival, and resolve_factoring completes the test
    unsigned int *fact_flag_host = nullptr;
    hipEvent_t fact_ev = nullptr;
    bool fact_pending = false, fact_req32 = false, fact_req64 = false;
    // FP32-only storage with a test pending: the FP64 tables are dropped when the test completes,
    // after a cast to the general FP32 tables only if the current did not factor
    bool cast_pending = false;
    // a stream with nothing else queued (the serving loop's release stream): buffers whose last user
    // is known to have finished are freed there, not behind the work queued on the problem's stream
    hipStream_t free_stream = nullptr;
    // the factored tables built with the test when the incident field is set: FP32 split by
    // default; a caller that knows its one precision (the serving loop) picks that one's
    sc_precision eager_prec = SC_FP32_SPLIT;
    // incident power per frequency through the aperture: [n_k] then the reduction scratch
    bool has_power = false;
    sc::DevBuf d_power;
    // lower bound of |r_s| over the nodes (the paraboloid: f), -1 if unknown
    double rs_min = -1.0;
    // observation points; obs_r2max = max |r'|^2 when they came from host memory, else -1
    int n_obs = 0, n_obs_pad = 0;
    double obs_r2max = -1.0;
    sc::DevBuf obs64, obs32;
    // result of the last evaluate
    int res_prec = -1;
    sc::DevBuf resE, resB;
    sc::DevBuf partial;
    // time transform
    sc::DevBuf d_t, tw, timeE, timeB;
    // host staging of small uploads (rule, spectrum, points), reused across calls so that set-up calls
    // need not wait for their copies; stage_ev marks the last upload from them
    std::vector<double> h_stage_rule, h_stage_spec, h_stage_obs, h_stage_modes;
    sc::DevBuf d_spec, d_obs_in, d_modes;
    hipEvent_t stage_ev = nullptr;
    bool stage_pending = false;
    // an optional pinned host area for the uploads (the serving loop's request block): pageable
    // sources make a copy wait for the earlier work on the stream, pinned ones do not.  Bump
    // allocated, never reused while the problem lives.
    char *stage_ext = nullptr;
    size_t stage_ext_cap = 0, stage_ext_off = 0;
    // launch override
    bool has_launch = false;
    sc_launch launch{};
    // profiling
    hipEvent_t ev[sc::EV_N] = {};
    bool ev_prep = false, ev_quad = false, ev_time = false;
    int64_t last_evals = 0, last_tiles = 0;
    int last_chunk = 0;   // node chunk of the last evaluation
};

namespace sc {

constexpr int OBS_PAD = 128;   // observation padding (64 lanes x up to 2 points per lane)

// Gauss-Legendre nodes (ascending) and weights on [-1, 1], correctly rounded (sc_gauss_host.cpp).
void gauss_legendre_rule(int n, std::vector<double> &x, std::vector<double> &w);

// Launch shape for a problem and precision (override > tuned > default).
sc_launch resolve_launch(const sc_prob *p, sc_precision prec);
sc_status check_launch(const sc_launch &l);
int mode_of(sc_precision prec);
size_t real_size(sc_precision prec);
// Completes a deferred factoring test: with `block`, waits for its flag; without, *ready tells whether
// the flag had arrived (and the test is complete).  A no-op when no test is pending.
sc_status resolve_factoring(sc_prob *p, bool block, bool *ready);
// Have a problem's stream-ordered buffers freed on `st` when it is destroyed (for a caller that
// knows no queued work still uses them, so that the frees need not wait behind that stream's work).
void prob_free_on(sc_prob *p, hipStream_t st);
// Tables of the precision, partial and result buffers; fills `job` (tile0 = 0, offset 0, all tiles).
sc_status prepare(sc_prob *p, sc_precision prec, const sc_launch &l, QuadJob &job);
// Upload `jobs` (tile0 assigned here) and run one persistent quadrature launch on ctx's stream.
sc_status run_quad(sc_ctx *c, std::vector<QuadJob> &jobs, sc_precision prec, const sc_launch &l, sc_prob *timed);
// Device bytes a problem of this shape holds after an evaluate (+ time transform with n_t samples).
size_t footprint_bytes(int n_r, int n_phi, int n_k, int n_obs, int n_t, sc_precision prec, int chunk);

}  // namespace sc
