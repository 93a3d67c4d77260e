// sc_serve.cpp -- continuous-batching serving loop for field solves.
//
// Requests (mirror + beam + spectrum + observation points) arrive from any
// host thread.  A scheduler thread admits them in arrival order while their
// HBM footprint fits the budget and the running count allows; a preparation
// thread builds their mirror / incident tables on a preparation stream
// (tables stay resident for the request's lifetime); the scheduler launches
// the quadrature tiles of ALL running
// requests together: each scheduling quantum is one persistent launch whose
// tile list holds a share of every running request's remaining tiles, sized to
// about `quantum_ms` of work.  A request that arrives while others are on the
// GPU joins the next quantum.  Two quanta are kept in flight so the device
// never idles while the next one is built.  When a request's last tile has
// been scheduled, its split-K reduction (and time transform) and the copy of
// its results to pinned host memory are queued behind that quantum.
//
// Every (chunk, k, observation block) partial of a request is computed by
// exactly one tile with the same kernel and chunking as sc_evaluate uses, so
// a request's result does not depend on what it was batched with.
//
// Nothing slow runs under the server lock or on the scheduling path: result
// buffers in pinned host memory come from a pool (pinning memory costs far
// more than the small requests' compute), the copies to them run on their own
// stream behind the quantum that finished the request, finished problems are
// released by the preparation thread, and waiters copy results out after
// dropping the lock.
#include <algorithm>
#include <chrono>
#include <cmath>
#include <condition_variable>
#include <cstdlib>
#include <cstring>
#include <deque>
#include <map>
#include <mutex>
#include <new>
#include <string>
#include <thread>
#include <vector>

#include <unistd.h>

#include "sc_host.h"

using namespace sc;
using Clock = std::chrono::steady_clock;

namespace {

enum ReqState { R_QUEUED, R_RUNNING, R_FINISHING, R_DONE, R_FAILED, R_CANCELLED };

struct Req {
    uint64_t ticket = 0;
    double f = 0, a = 0, w0 = 0, pol = 0, dk = 0;
    int n_r = 0, n_phi = 0, consistent = 0, n_t = 0, n_obs = 0, beam = 0;
    sc_precision prec = SC_FP32_SPLIT;
    std::vector<double> k, spec, obs, t;
    size_t bytes = 0;        // device bytes charged against the budget
    size_t held_bytes = 0;   // device bytes held once prepared
    size_t host_bytes = 0;   // pinned host bytes of its block (results, flag, upload staging)
    ReqState state = R_QUEUED;
    sc_status status = SC_OK;
    std::string err;
    sc_prob *prob = nullptr;
    QuadJob job{};
    int64_t cursor = 0;
    hipEvent_t ready_ev = nullptr;   // tables built (preparation stream)
    hipEvent_t fin_ev = nullptr;     // last kernel of the request done (compute stream)
    hipEvent_t done_ev = nullptr;    // results in host memory (copy stream)
    void *hE = nullptr, *hB = nullptr, *hEt = nullptr, *hBt = nullptr;   // views into host_block
    void *host_block = nullptr;
    size_t host_block_bytes = 0;
    size_t res_bytes = 0, time_bytes = 0;
    Clock::time_point t_submit, t_admit, t_done;
    int64_t evals = 0;
};

struct Quantum {
    int slot;
    int64_t evals;
    Clock::time_point t_launch;
};

double ms_between(Clock::time_point a, Clock::time_point b)
{
    return std::chrono::duration<double, std::milli>(b - a).count();
}

// Pinned host blocks for results, reused across requests.  Sizes are rounded
// up to powers of two (at least 1 MiB); up to CACHE_BYTES of free blocks are
// kept, larger surpluses are unpinned.
struct PinnedPool {
    static constexpr size_t MIN_BLOCK = size_t(1) << 20;
    static constexpr size_t CACHE_BYTES = size_t(16) << 30;
    std::mutex mu;
    std::multimap<size_t, void *> free_blocks;
    size_t cached = 0;

    static size_t bucket(size_t n)
    {
        size_t b = MIN_BLOCK;
        while (b < n) b <<= 1;
        return b;
    }
    hipError_t get(size_t n, void **p, size_t *got)
    {
        const size_t b = bucket(n);
        {
            std::lock_guard<std::mutex> lk(mu);
            auto it = free_blocks.find(b);
            if (it != free_blocks.end()) {
                *p = it->second;
                *got = b;
                free_blocks.erase(it);
                cached -= b;
                return hipSuccess;
            }
        }
        *got = b;
        return hipHostMalloc(p, b, hipHostMallocDefault);
    }
    void put(void *p, size_t b)
    {
        if (!p) return;
        {
            std::lock_guard<std::mutex> lk(mu);
            if (cached + b <= CACHE_BYTES) {
                free_blocks.emplace(b, p);
                cached += b;
                return;
            }
        }
        (void)hipHostFree(p);
    }
    void clear()
    {
        std::lock_guard<std::mutex> lk(mu);
        for (auto &kv : free_blocks) (void)hipHostFree(kv.second);
        free_blocks.clear();
        cached = 0;
    }
};

}  // namespace

struct sc_server {
    sc_ctx *ctx = nullptr;
    sc_ctx *prep = nullptr;
    size_t budget = 0;
    int max_running = 1;
    double quantum_ms = 20.0;
    std::thread worker;     // scheduler: admission, quanta, completion
    std::thread preparer;   // builds admitted requests' tables off the scheduling path
    std::mutex mu;
    std::condition_variable cv_work, cv_done, cv_prep;
    bool stop = false;
    std::deque<Req *> to_prepare;   // admitted, tables not built yet
    std::vector<sc_prob *> to_release;   // finished problems, released by the preparation thread
    int preparing = 0;
    hipStream_t copy_stream = nullptr;   // device-to-host copies of results
    hipStream_t release_stream = nullptr;   // frees of finished problems (nothing else queued on it)
    hipMemPool_t pool = nullptr;             // the device's default pool, if this server set its threshold
    size_t host_budget = 0, host_in_use = 0; // pinned host bytes of admitted, not yet collected requests
    PinnedPool pinned;
    uint64_t next_ticket = 1;
    std::deque<Req *> queue;
    std::vector<Req *> active;
    std::map<uint64_t, Req *> all;
    sc_server_stats stats{};
    static constexpr int RING = 3;
    DevBuf jobbuf[RING];
    QuadJob *hjobs[RING] = {};
    size_t hjobs_cap[RING] = {};
    hipEvent_t slot_ev[RING] = {};     // end of the quantum launched from this slot (timed)
    hipEvent_t slot_start[RING] = {};  // start of that quantum (timed)
    bool slot_busy[RING] = {};
    std::deque<Quantum> inflight;
    double evals_per_ms = 1.0e8;   // running throughput estimate used to size quanta
    int next_slot = 0;
    std::string worker_error;
};

static void free_req_host(sc_server *s, Req *r)
{
    s->pinned.put(r->host_block, r->host_block_bytes);
    r->host_block = nullptr;
    r->hE = r->hB = r->hEt = r->hBt = nullptr;
    for (hipEvent_t *e : {&r->ready_ev, &r->fin_ev, &r->done_ev})
        if (*e) {
            (void)hipEventDestroy(*e);
            *e = nullptr;
        }
}

static void release_prob(Req *r)
{
    if (r->prob) {
        (void)sc_prob_destroy(r->prob);
        r->prob = nullptr;
    }
}

// Test hook: SC_DEBUG_FAIL_QUANTUM=<n> makes the job-buffer reservation of the
// n-th scheduling quantum of the process report SC_E_NOMEM (before anything of
// that quantum is enqueued), so the failure path can be exercised from the host.
static bool debug_fail_this_quantum()
{
    static std::mutex mu;
    static long count = 0;
    static long fail_at = -2;
    std::lock_guard<std::mutex> lk(mu);
    if (fail_at == -2) {
        const char *e = getenv("SC_DEBUG_FAIL_QUANTUM");
        fail_at = e ? atol(e) : -1;
    }
    ++count;
    return fail_at > 0 && count == fail_at;
}

// One kernel shape per precision, so that requests of a precision share launches: the FP32 forms
// take four frequencies per lane (the built-in beams of the requests factor), FP64 two.
static int server_opl(sc_precision) { return 1; }
static int server_fpb(sc_precision prec) { return prec == SC_FP64 ? 2 : 4; }

// Build the request's device state on the preparation stream, in two steps so that the
// preparation thread never waits for the device: setup_begin enqueues the tables and the factoring
// test, whose flag arrives in the request's pinned block; setup_finish, once it has, sizes the
// partials and results for the table layout the test chose and fills the request's job.
// Layout of a request's pinned block: E, B, then Et, Bt (each 256-byte aligned), the factoring flag
// (256 bytes), and the staging area of the set-up's uploads (rule, frequencies, spectrum, points,
// times), each upload 64-byte aligned.
struct BlockLayout {
    size_t re, te, tb, stage, total;
};
static BlockLayout block_layout(const Req *r)
{
    BlockLayout b;
    b.re = (r->res_bytes + 255) & ~size_t(255);
    b.te = (r->time_bytes + 255) & ~size_t(255);
    b.tb = r->n_t > 0 ? 2 * b.te : 0;
    auto up = [](size_t n) { return (sizeof(double) * n + 63) & ~size_t(63); };
    b.stage = up(2 * (size_t)r->n_r + 1 + 2 * (size_t)r->n_phi) + up(r->k.size()) + up(2 * r->k.size()) +
              up(3 * (size_t)r->n_obs) + up((size_t)r->n_t);
    b.total = 2 * b.re + b.tb + 256 + b.stage;
    return b;
}

static sc_status setup_begin(sc_server *s, Req *r)
{
    SC_TRY(sc_prob_create(s->prep, &r->prob));
    sc_prob *p = r->prob;
    p->alloc_stream = s->prep->stream;
    p->keep_fp64 = r->prec == SC_FP64;   // FP32 requests keep only their FP32 tables
    p->eager_prec = r->prec;             // and the factored tables of their own precision only
    p->free_stream = s->release_stream;
    const int n_k = (int)r->k.size();
    const size_t rs = real_size(r->prec);
    {   // one pinned block (block_layout)
        const BlockLayout bl = block_layout(r);
        HIP_TRY(s->pinned.get(bl.total, &r->host_block, &r->host_block_bytes));
        char *b = (char *)r->host_block;
        r->hE = b;
        r->hB = b + bl.re;
        if (r->n_t > 0) {
            r->hEt = b + 2 * bl.re;
            r->hBt = b + 2 * bl.re + bl.te;
        }
        p->fact_flag_host = (unsigned int *)(b + 2 * bl.re + bl.tb);
        p->stage_ext = b + 2 * bl.re + bl.tb + 256;
        p->stage_ext_cap = bl.stage;
        p->stage_ext_off = 0;
    }
    SC_TRY(sc_set_mirror(p, r->f, r->a, r->n_r, r->n_phi));
    SC_TRY(sc_set_frequencies(p, r->k.data(), n_k));
    SC_TRY(sc_set_incident_beam(p, r->beam, r->w0, r->pol, r->spec.empty() ? nullptr : r->spec.data(),
                                r->consistent));
    SC_TRY(sc_set_observation(p, r->obs.data(), r->n_obs, 0));
    if (r->n_t > 0) {
        SC_TRY(p->d_t.reserve(sizeof(double) * r->n_t, p->alloc_stream));
        SC_TRY(p->tw.reserve(sizeof(double) * 2 * (size_t)r->n_t * n_k, p->alloc_stream));
        SC_TRY(p->timeE.reserve(rs * 6 * (size_t)r->n_t * r->n_obs, p->alloc_stream));
        SC_TRY(p->timeB.reserve(rs * 6 * (size_t)r->n_t * r->n_obs, p->alloc_stream));
        const size_t tbytes = sizeof(double) * r->n_t;
        const void *src = r->t.data();
        if (p->stage_ext_off + tbytes <= p->stage_ext_cap) {   // the times from the pinned area
            std::memcpy(p->stage_ext + p->stage_ext_off, r->t.data(), tbytes);
            src = p->stage_ext + p->stage_ext_off;
            p->stage_ext_off += (tbytes + 63) & ~size_t(63);
        }
        HIP_TRY(hipMemcpyAsync(p->d_t.p, src, tbytes, hipMemcpyHostToDevice, s->prep->stream));
    }
    HIP_TRY(hipEventCreateWithFlags(&r->ready_ev, hipEventDisableTiming));
    HIP_TRY(hipEventCreateWithFlags(&r->fin_ev, hipEventDisableTiming));
    HIP_TRY(hipEventCreateWithFlags(&r->done_ev, hipEventDisableTiming));
    return SC_OK;
}

// *ready = false (and nothing done) while the factoring flag is still on its way.
static sc_status setup_finish(sc_server *s, Req *r, bool *ready)
{
    sc_prob *p = r->prob;
    SC_TRY(resolve_factoring(p, false, ready));
    if (!*ready) return SC_OK;
    sc_launch l = resolve_launch(p, r->prec);
    l.obs_per_lane = server_opl(r->prec);
    l.freq_per_lane = server_fpb(r->prec);
    SC_TRY(prepare(p, r->prec, l, r->job));
    HIP_TRY(hipEventRecord(r->ready_ev, s->prep->stream));
    // what the request holds from now on (the admission charged the set-up's peak: FP64 tables,
    // general FP32 tables and factored ones at once)
    SC_TRY(sc_prob_device_bytes(p, &r->held_bytes));
    // the time samples are copied from r->t, which lives as long as the request
    r->evals = (int64_t)r->n_obs * (int64_t)r->k.size() * p->n_surf;
    return SC_OK;
}

// After the last tile of `r` is queued: reduction, time transform, copies to pinned host memory.
static sc_status finish_request(sc_server *s, Req *r)
{
    hipStream_t st = s->ctx->stream;
    sc_prob *p = r->prob;
    const int n_k = (int)r->k.size();
    HIP_TRY(launch_reduce(st, mode_of(r->prec), p->partial.p, r->job.n_chunks, n_k, r->n_obs, p->n_obs_pad,
                          p->d_k.as<double>(), r->job.tied, p->resE.p, p->resB.p));
    if (r->n_t > 0) {
        const int f64 = r->prec == SC_FP64;
        const int64_t n_x = (int64_t)r->n_obs * 3;
        HIP_TRY(launch_twiddles(st, n_k, p->d_k.as<double>(), r->n_t, p->d_t.as<double>(), r->dk, p->tw.as<double>()));
        HIP_TRY(launch_time(st, f64, n_k, r->n_t, n_x, p->tw.as<double>(), p->resE.p, p->timeE.p));
        HIP_TRY(launch_time(st, f64, n_k, r->n_t, n_x, p->tw.as<double>(), p->resB.p, p->timeB.p));
    }
    // the copies overlap the next quanta: the copy stream waits for this request's last kernel only
    hipStream_t cs = s->copy_stream;
    HIP_TRY(hipEventRecord(r->fin_ev, st));
    HIP_TRY(hipStreamWaitEvent(cs, r->fin_ev, 0));
    HIP_TRY(hipMemcpyAsync(r->hE, p->resE.p, r->res_bytes, hipMemcpyDeviceToHost, cs));
    HIP_TRY(hipMemcpyAsync(r->hB, p->resB.p, r->res_bytes, hipMemcpyDeviceToHost, cs));
    if (r->n_t > 0) {
        HIP_TRY(hipMemcpyAsync(r->hEt, p->timeE.p, r->time_bytes, hipMemcpyDeviceToHost, cs));
        HIP_TRY(hipMemcpyAsync(r->hBt, p->timeB.p, r->time_bytes, hipMemcpyDeviceToHost, cs));
    }
    HIP_TRY(hipEventRecord(r->done_ev, cs));
    return SC_OK;
}

// Launch one scheduling quantum over the running requests of one precision.
// Called with the server lock held.
static sc_status launch_quantum(sc_server *s)
{
    // the oldest running request with tiles left decides the precision of this quantum
    sc_precision prec = SC_FP32_SPLIT;
    bool found = false;
    for (Req *r : s->active)
        if (r->state == R_RUNNING && r->cursor < r->job.n_tiles) {
            prec = r->prec;
            found = true;
            break;
        }
    if (!found) return SC_OK;
    std::vector<Req *> group;
    for (Req *r : s->active)
        if (r->state == R_RUNNING && r->cursor < r->job.n_tiles && r->prec == prec) group.push_back(r);
    const int opl = server_opl(prec);
    const int fpb = server_fpb(prec);
    const double budget_evals = std::max(1.0, s->quantum_ms * s->evals_per_ms);
    const double share = budget_evals / (double)group.size();
    std::vector<QuadJob> jobs;
    std::vector<Req *> finals;
    int64_t total = 0, evals = 0;
    for (Req *r : group) {
        const double per_tile = 64.0 * opl * fpb * std::min<double>(r->job.chunk, r->job.n_tot);
        int64_t n = (int64_t)std::ceil(share / per_tile);
        n = std::max<int64_t>(1, std::min<int64_t>(n, r->job.n_tiles - r->cursor));
        QuadJob j = r->job;
        j.tile0 = total;
        j.tile_offset = r->cursor;
        j.n_tiles = n;
        jobs.push_back(j);
        total += n;
        evals += (int64_t)(n * per_tile);
        r->cursor += n;
        if (r->cursor == r->job.n_tiles) finals.push_back(r);
    }
    // a free ring slot (at most two quanta are in flight, the ring has three)
    int slot = -1;
    for (int i = 0; i < sc_server::RING; ++i) {
        int c = (s->next_slot + i) % sc_server::RING;
        if (!s->slot_busy[c]) {
            slot = c;
            break;
        }
    }
    if (slot < 0) return fail(SC_E_DEVICE, "serving: no free launch slot");
    s->next_slot = (slot + 1) % sc_server::RING;
    hipStream_t st = s->ctx->stream;
    if (s->hjobs_cap[slot] < jobs.size()) {
        if (s->hjobs[slot]) (void)hipHostFree(s->hjobs[slot]);
        s->hjobs[slot] = nullptr;
        s->hjobs_cap[slot] = 0;
        size_t cap = std::max<size_t>(64, jobs.size() * 2);
        HIP_TRY(hipHostMalloc((void **)&s->hjobs[slot], sizeof(QuadJob) * cap, hipHostMallocDefault));
        s->hjobs_cap[slot] = cap;
    }
    if (debug_fail_this_quantum()) return fail(SC_E_NOMEM, "injected job-buffer allocation failure");
    SC_TRY(s->jobbuf[slot].reserve(sizeof(QuadJob) * s->hjobs_cap[slot]));
    memcpy(s->hjobs[slot], jobs.data(), sizeof(QuadJob) * jobs.size());
    for (Req *r : group) HIP_TRY(hipStreamWaitEvent(st, r->ready_ev, 0));
    HIP_TRY(hipMemcpyAsync(s->jobbuf[slot].p, s->hjobs[slot], sizeof(QuadJob) * jobs.size(), hipMemcpyHostToDevice,
                           st));
    HIP_TRY(launch_fill_u32(st, s->ctx->counter.as<unsigned int>(), 0u, QUAD_SEGMENTS));
    HIP_TRY(hipEventRecord(s->slot_start[slot], st));
    const int mode = mode_of(prec);
    const int wpb = 4;
    const int occ = quad_max_blocks_per_cu(mode, opl, fpb, wpb);
    int64_t grid = std::min<int64_t>((int64_t)occ * s->ctx->n_cu, (total + wpb - 1) / wpb);
    grid = std::max<int64_t>(grid, 1);
    HIP_TRY(launch_quad(st, mode, opl, fpb, wpb, (int)grid, s->jobbuf[slot].as<QuadJob>(), (int)jobs.size(),
                        total, s->ctx->counter.as<unsigned int>()));
    HIP_TRY(hipEventRecord(s->slot_ev[slot], st));
    s->slot_busy[slot] = true;
    s->inflight.push_back({slot, evals, Clock::now()});
    s->stats.launches++;
    s->stats.evals_launched += evals;
    for (Req *r : finals) {
        sc_status fs = finish_request(s, r);
        if (fs != SC_OK) return fs;
        r->state = R_FINISHING;
    }
    return SC_OK;
}

static void complete_request(sc_server *s, Req *r, ReqState state, sc_status st, const std::string &err)
{
    r->state = state;
    r->status = st;
    r->err = err;
    r->t_done = Clock::now();
    if (s->stats.running > 0) s->stats.running--;
    if (state == R_DONE) {
        s->stats.completed++;
        s->stats.evals_done += r->evals;
    }
    s->stats.hbm_in_use -= std::min(s->stats.hbm_in_use, r->bytes);
    if (r->prob) {   // its device work is complete; freeing it waits on the preparation stream
        s->to_release.push_back(r->prob);
        r->prob = nullptr;
        s->cv_prep.notify_one();
    }
    s->cv_done.notify_all();
}

// Preparation thread: starts admitted requests' set-up on the preparation stream (up to
// MAX_STARTED at a time) and completes each once its factoring flag has arrived, then hands it to
// the scheduler; finished problems are released here too.
static void prep_main(sc_server *s)
{
    constexpr int MAX_STARTED = 8;
    (void)hipSetDevice(s->ctx->device);
    std::deque<std::pair<Req *, Clock::time_point>> started;   // set-up begun, flag not in yet
    std::unique_lock<std::mutex> lk(s->mu);
    for (;;) {
        auto work = [s, &started] {
            return (s->stop && started.empty()) || !s->to_release.empty() ||
                   (!s->to_prepare.empty() && (int)started.size() < MAX_STARTED);
        };
        if (started.empty()) s->cv_prep.wait(lk, work);
        else s->cv_prep.wait_for(lk, std::chrono::microseconds(500), work);   // poll the flags
        if (!s->to_release.empty()) {   // frees first, so the next request's allocations can reuse them
            std::vector<sc_prob *> rel;
            rel.swap(s->to_release);
            lk.unlock();
            for (sc_prob *p : rel) {
                // no queued work uses a finished request's buffers: free them on a stream of their own,
                // not behind the next requests' set-up on the preparation stream
                prob_free_on(p, s->release_stream);
                (void)sc_prob_destroy(p);
            }
            // the frees run at once on that stream; synchronising it lets the pool return what it holds
            // beyond its release threshold
            (void)hipStreamSynchronize(s->release_stream);
            lk.lock();
            continue;
        }
        // at shutdown the admitted requests still run (the scheduler waits for them), so the started
        // ones are completed first
        if (s->stop && s->to_prepare.empty() && started.empty()) break;
        // complete, in order, the started requests whose flag has arrived
        while (!started.empty()) {
            Req *r = started.front().first;
            lk.unlock();
            bool ready = false;
            const Clock::time_point h0 = Clock::now();
            const sc_status st = setup_finish(s, r, &ready);
            const double host_ms = ms_between(h0, Clock::now());
            const std::string err = st == SC_OK ? std::string() : std::string(sc_last_error());
            if (st != SC_OK) (void)hipStreamSynchronize(s->prep->stream);
            lk.lock();
            s->stats.prep_host_ms += host_ms;
            if (st == SC_OK && !ready) break;
            s->stats.prep_ms += ms_between(started.front().second, Clock::now());
            started.pop_front();
            s->preparing--;
            if (st == SC_OK) {
                if (r->held_bytes < r->bytes) {   // give back what the set-up no longer holds
                    s->stats.hbm_in_use -= std::min(s->stats.hbm_in_use, r->bytes - r->held_bytes);
                    r->bytes = r->held_bytes;
                }
                s->active.push_back(r);
            } else {
                complete_request(s, r, R_FAILED, st, err);
            }
            s->cv_work.notify_one();
        }
        if (s->to_prepare.empty() || (int)started.size() >= MAX_STARTED) continue;
        Req *r = s->to_prepare.front();
        s->to_prepare.pop_front();
        s->preparing++;
        lk.unlock();
        const Clock::time_point t0 = Clock::now();
        const sc_status st = setup_begin(s, r);
        const double host_ms = ms_between(t0, Clock::now());
        const std::string err = st == SC_OK ? std::string() : std::string(sc_last_error());
        // a failed request may still have copies from its host arrays in flight
        if (st != SC_OK) (void)hipStreamSynchronize(s->prep->stream);
        lk.lock();
        s->stats.prep_host_ms += host_ms;
        if (st == SC_OK) {
            started.emplace_back(r, t0);
        } else {
            s->stats.prep_ms += ms_between(t0, Clock::now());
            s->preparing--;
            complete_request(s, r, R_FAILED, st, err);
            s->cv_work.notify_one();
        }
    }
}

static void worker_main(sc_server *s)
{
    (void)hipSetDevice(s->ctx->device);
    std::unique_lock<std::mutex> lk(s->mu);
    for (;;) {
        // 1. admission, in arrival order, while memory and running slots allow
        bool admitted = false;
        while (!s->queue.empty() &&
               (int)(s->active.size() + s->to_prepare.size()) + s->preparing < s->max_running) {
            Req *r = s->queue.front();
            if (s->stats.hbm_in_use + r->bytes > s->budget) break;
            // results wait in pinned host memory until collected: admit only while they fit
            if (s->host_in_use > 0 && s->host_in_use + r->host_bytes > s->host_budget) break;
            s->queue.pop_front();
            s->host_in_use += r->host_bytes;
            s->stats.host_in_use = s->host_in_use;
            r->state = R_RUNNING;
            r->t_admit = Clock::now();
            s->stats.hbm_in_use += r->bytes;
            s->stats.admitted++;
            s->stats.queued--;
            s->stats.running++;
            s->to_prepare.push_back(r);
            admitted = true;
        }
        if (admitted) s->cv_prep.notify_one();
        // 2. requests whose results reached the host
        for (size_t i = 0; i < s->active.size();) {
            Req *r = s->active[i];
            if (r->state == R_FINISHING && hipEventQuery(r->done_ev) == hipSuccess) {
                complete_request(s, r, R_DONE, SC_OK, "");
                s->active.erase(s->active.begin() + i);
            } else {
                ++i;
            }
        }
        // 3. finished quanta: their measured device time sizes the next ones
        while (!s->inflight.empty() && hipEventQuery(s->slot_ev[s->inflight.front().slot]) == hipSuccess) {
            const Quantum &q = s->inflight.front();
            float ms = 0.f;
            if (hipEventElapsedTime(&ms, s->slot_start[q.slot], s->slot_ev[q.slot]) == hipSuccess) {
                s->stats.quad_ms += ms;
                if (ms > 0.05f) s->evals_per_ms = 0.7 * s->evals_per_ms + 0.3 * (q.evals / (double)ms);
            }
            s->slot_busy[q.slot] = false;
            s->inflight.pop_front();
        }
        // 4. keep two quanta in flight
        bool more = false;
        for (Req *r : s->active)
            if (r->state == R_RUNNING && r->cursor < r->job.n_tiles) more = true;
        if (more && s->inflight.size() < 2) {
            sc_status st = launch_quantum(s);
            if (st != SC_OK) {
                // The quanta already queued still read and write the running requests' buffers, and
                // finished requests may still be copying to their pinned blocks: completing a request
                // releases both, so wait for the compute and copy streams first.
                std::string err = sc_last_error();
                (void)hipStreamSynchronize(s->ctx->stream);
                (void)hipStreamSynchronize(s->copy_stream);
                while (!s->inflight.empty()) {
                    s->slot_busy[s->inflight.front().slot] = false;
                    s->inflight.pop_front();
                }
                // Requests whose results reached the host complete normally; the others have lost
                // tiles (or share a failing device) and fail with the quantum's status.
                for (Req *r : s->active) {
                    if (r->state == R_FINISHING && hipEventQuery(r->done_ev) == hipSuccess)
                        complete_request(s, r, R_DONE, SC_OK, "");
                    else
                        complete_request(s, r, R_FAILED, st, err);
                }
                (void)hipGetLastError();
                s->active.clear();
                s->worker_error = err;
            }
            continue;
        }
        if (s->stop && s->queue.empty() && s->active.empty() && s->inflight.empty() && s->to_prepare.empty() &&
            s->preparing == 0)
            break;
        // 5. wait for a submission or a prepared request, or poll the device
        if (s->active.empty() && s->inflight.empty())
            s->cv_work.wait_for(lk, std::chrono::milliseconds(s->queue.empty() ? 50 : 1));
        else
            s->cv_work.wait_for(lk, std::chrono::microseconds(200));
    }
}

// ======================================================================= ABI

// While servers run on a device, its default memory pool keeps some freed memory for reuse (a fresh
// mapping of a request's buffers costs host time on every set-up): up to half of what the budget
// leaves of the device, at most 32 GiB, so that the runtime keeps room of its own.  The first server
// on a device sets the threshold and the last one restores it and trims the pool.
static std::mutex pool_mu;
static std::map<int, std::pair<int, uint64_t>> pool_users;   // device -> (servers, saved threshold)

static void pool_cache_acquire(sc_server *s, size_t budget)
{
    std::lock_guard<std::mutex> lk(pool_mu);
    hipMemPool_t pool = nullptr;
    if (hipDeviceGetDefaultMemPool(&pool, s->ctx->device) != hipSuccess) {
        (void)hipGetLastError();
        return;
    }
    auto &u = pool_users[s->ctx->device];
    if (u.first == 0) {
        size_t free_b = 0, total_b = 0;
        (void)hipMemGetInfo(&free_b, &total_b);
        uint64_t keep = total_b > budget ? std::min<uint64_t>(uint64_t(32) << 30, (total_b - budget) / 2) : 0;
        if (hipMemPoolGetAttribute(pool, hipMemPoolAttrReleaseThreshold, &u.second) != hipSuccess ||
            hipMemPoolSetAttribute(pool, hipMemPoolAttrReleaseThreshold, &keep) != hipSuccess) {
            (void)hipGetLastError();
            return;
        }
    }
    u.first++;
    s->pool = pool;
}

static void pool_cache_release(sc_server *s)
{
    if (!s->pool) return;
    std::lock_guard<std::mutex> lk(pool_mu);
    auto &u = pool_users[s->ctx->device];
    if (--u.first == 0) {   // the pool as it was, and what the servers left in it returned
        (void)hipMemPoolSetAttribute(s->pool, hipMemPoolAttrReleaseThreshold, &u.second);
        (void)hipMemPoolTrimTo(s->pool, 0);
    }
    s->pool = nullptr;
}

extern "C" sc_status sc_server_create(sc_ctx *ctx, size_t hbm_budget, int max_running, double quantum_ms,
                                      sc_server **out)
{
    if (!ctx || !out) return fail(SC_E_INVAL, "sc_server_create: NULL argument");
    if (hbm_budget == 0 || max_running < 1 || !(quantum_ms > 0.0))
        return fail(SC_E_INVAL, "sc_server_create: need hbm_budget > 0, max_running >= 1, quantum_ms > 0");
    *out = nullptr;
    DeviceGuard g(ctx->device);
    sc_server *s = new (std::nothrow) sc_server();
    if (!s) return fail(SC_E_NOMEM, "sc_server_create: out of host memory");
    s->ctx = ctx;
    s->budget = hbm_budget;
    s->max_running = max_running;
    s->quantum_ms = quantum_ms;
    s->stats.hbm_budget = hbm_budget;
    {   // pinned host memory for results not yet collected: a quarter of the host memory, at most 64 GiB
        const long pages = sysconf(_SC_PHYS_PAGES), page = sysconf(_SC_PAGE_SIZE);
        const uint64_t phys = pages > 0 && page > 0 ? (uint64_t)pages * (uint64_t)page : (uint64_t(16) << 30);
        s->host_budget = (size_t)std::min<uint64_t>(uint64_t(64) << 30, phys / 4);
        s->stats.host_budget = s->host_budget;
    }
    sc_status st = sc_ctx_create(ctx->device, nullptr, &s->prep);
    if (st != SC_OK) {
        delete s;
        return st;
    }
    s->prep->tune = ctx->tune;
    if (hipStreamCreateWithFlags(&s->copy_stream, hipStreamNonBlocking) != hipSuccess) {
        (void)sc_ctx_destroy(s->prep);
        delete s;
        return fail(SC_E_DEVICE, "sc_server_create: hipStreamCreateWithFlags failed");
    }
    if (hipStreamCreateWithFlags(&s->release_stream, hipStreamNonBlocking) != hipSuccess) {
        (void)hipStreamDestroy(s->copy_stream);
        (void)sc_ctx_destroy(s->prep);
        delete s;
        return fail(SC_E_DEVICE, "sc_server_create: hipStreamCreateWithFlags failed");
    }
    for (int i = 0; i < sc_server::RING; ++i)
        if (hipEventCreate(&s->slot_ev[i]) != hipSuccess || hipEventCreate(&s->slot_start[i]) != hipSuccess) {
            for (int j = 0; j <= i; ++j) {
                if (s->slot_ev[j]) (void)hipEventDestroy(s->slot_ev[j]);
                if (s->slot_start[j]) (void)hipEventDestroy(s->slot_start[j]);
            }
            (void)hipStreamDestroy(s->copy_stream);
            (void)hipStreamDestroy(s->release_stream);
            (void)sc_ctx_destroy(s->prep);
            delete s;
            return fail(SC_E_DEVICE, "sc_server_create: hipEventCreate failed");
        }
    pool_cache_acquire(s, hbm_budget);
    ctx->n_probs++;   // the context must outlive the server
    s->worker = std::thread(worker_main, s);
    s->preparer = std::thread(prep_main, s);
    *out = s;
    return SC_OK;
}

static sc_status validate_request(const sc_request *q)
{
    if (!q) return fail(SC_E_INVAL, "sc_server_submit: request is NULL");
    if (!(q->f > 0.0) || !(q->r_max > 0.0)) return fail(SC_E_INVAL, "request: f and r_max must be > 0");
    if (q->n_r < 1 || q->n_phi < 1 || (int64_t)(q->n_r + 1) * q->n_phi >= (1LL << 31))
        return fail(SC_E_INVAL, "request: bad quadrature size");
    if (q->n_k < 1 || !q->k) return fail(SC_E_INVAL, "request: need n_k >= 1 wavenumbers");
    if (q->n_k > SC_MAX_FREQUENCIES) return fail(SC_E_INVAL, "request: at most %d wavenumbers", SC_MAX_FREQUENCIES);
    if (q->n_t < 0 || q->n_t > SC_MAX_TIMES) return fail(SC_E_INVAL, "request: at most %d time samples", SC_MAX_TIMES);
    for (int i = 0; i < q->n_k; ++i)
        if (!(q->k[i] > 0.0) || !std::isfinite(q->k[i])) return fail(SC_E_INVAL, "request: k[%d] invalid", i);
    if (!(q->w0 > 0.0)) return fail(SC_E_INVAL, "request: w0 must be > 0");
    if (q->beam != SC_BEAM_LINEAR && q->beam != SC_BEAM_RADIAL && q->beam != SC_BEAM_AZIMUTHAL)
        return fail(SC_E_INVAL, "request: unknown beam %d", q->beam);
    if (q->beam != SC_BEAM_LINEAR && !std::isfinite(q->w0))
        return fail(SC_E_INVAL, "request: a cylindrical beam needs a finite w0");
    if (q->n_obs < 1 || !q->obs) return fail(SC_E_INVAL, "request: need n_obs >= 1 points");
    if (q->prec != SC_FP64 && q->prec != SC_FP32_SPLIT && q->prec != SC_FP32)
        return fail(SC_E_INVAL, "request: unknown precision");
    if (q->n_t < 0 || (q->n_t > 0 && !q->t)) return fail(SC_E_INVAL, "request: bad time samples");
    return SC_OK;
}

extern "C" sc_status sc_server_submit(sc_server *s, const sc_request *q, uint64_t *ticket)
{
    if (!s || !ticket) return fail(SC_E_INVAL, "sc_server_submit: NULL argument");
    SC_TRY(validate_request(q));
    Req *r = new (std::nothrow) Req();
    if (!r) return fail(SC_E_NOMEM, "sc_server_submit: out of host memory");
    r->f = q->f;
    r->a = q->r_max;
    r->n_r = q->n_r;
    r->n_phi = q->n_phi;
    r->k.assign(q->k, q->k + q->n_k);
    if (q->spectrum) r->spec.assign(q->spectrum, q->spectrum + 2 * q->n_k);
    r->w0 = q->w0;
    r->pol = q->pol_angle;
    r->consistent = q->consistent;
    r->beam = q->beam;
    r->n_obs = q->n_obs;
    r->obs.assign(q->obs, q->obs + 3 * (size_t)q->n_obs);
    r->prec = q->prec;
    r->n_t = q->n_t;
    if (q->n_t > 0) r->t.assign(q->t, q->t + q->n_t);
    r->dk = q->dk;
    {
        // the chunk the request will be evaluated with (same rule as sc_evaluate)
        sc_prob probe;
        probe.ctx = s->ctx;
        probe.n_obs = q->n_obs;
        probe.k = r->k;
        probe.n_tot = (q->n_r + 1) * q->n_phi;
        const sc_launch l = resolve_launch(&probe, q->prec);
        r->bytes = footprint_bytes(q->n_r, q->n_phi, q->n_k, q->n_obs, q->n_t, q->prec, l.chunk);
    }
    r->res_bytes = real_size(q->prec) * 6 * (size_t)q->n_k * q->n_obs;
    r->time_bytes = real_size(q->prec) * 6 * (size_t)q->n_t * q->n_obs;
    r->host_bytes = PinnedPool::bucket(block_layout(r).total);
    r->t_submit = Clock::now();
    std::lock_guard<std::mutex> lk(s->mu);
    if (s->stop) {
        delete r;
        return fail(SC_E_STATE, "sc_server_submit: server is shutting down");
    }
    if (r->bytes > s->budget) {
        s->stats.rejected++;
        size_t b = r->bytes;
        delete r;
        return fail(SC_E_REJECTED, "request needs %zu device bytes, budget is %zu", b, s->budget);
    }
    r->ticket = s->next_ticket++;
    s->all[r->ticket] = r;
    s->queue.push_back(r);
    s->stats.submitted++;
    s->stats.queued++;
    *ticket = r->ticket;
    s->cv_work.notify_one();
    return SC_OK;
}

extern "C" sc_status sc_server_wait(sc_server *s, uint64_t ticket, double timeout_ms, void *E, void *B, void *Et,
                                    void *Bt, sc_request_stats *stats)
{
    if (!s) return fail(SC_E_INVAL, "sc_server_wait: server is NULL");
    std::unique_lock<std::mutex> lk(s->mu);
    auto it = s->all.find(ticket);
    if (it == s->all.end()) return fail(SC_E_INVAL, "sc_server_wait: unknown ticket %llu", (unsigned long long)ticket);
    Req *r = it->second;
    auto ready = [r] { return r->state == R_DONE || r->state == R_FAILED || r->state == R_CANCELLED; };
    if (timeout_ms < 0) s->cv_done.wait(lk, ready);
    else if (!s->cv_done.wait_for(lk, std::chrono::duration<double, std::milli>(timeout_ms), ready))
        return fail(SC_E_TIMEOUT, "sc_server_wait: ticket %llu not ready", (unsigned long long)ticket);
    // the request leaves the server's books here; its results are copied out without the lock
    s->all.erase(it);
    lk.unlock();
    sc_status st = SC_OK;
    if (r->state == R_DONE) {
        if (E) memcpy(E, r->hE, r->res_bytes);
        if (B) memcpy(B, r->hB, r->res_bytes);
        if (Et && r->hEt) memcpy(Et, r->hEt, r->time_bytes);
        if (Bt && r->hBt) memcpy(Bt, r->hBt, r->time_bytes);
        if (stats) {
            stats->queue_ms = ms_between(r->t_submit, r->t_admit);
            stats->run_ms = ms_between(r->t_admit, r->t_done);
            stats->total_ms = ms_between(r->t_submit, r->t_done);
            stats->evals = r->evals;
            stats->device_bytes = r->bytes;
        }
    } else if (r->state == R_CANCELLED) {
        st = fail(SC_E_CANCELLED, "ticket %llu was cancelled", (unsigned long long)ticket);
    } else {
        st = fail(r->status, "request failed: %s", r->err.c_str());
    }
    free_req_host(s, r);
    if (r->state != R_CANCELLED && r->host_bytes) {   // admitted: its host bytes go back to the budget
        std::lock_guard<std::mutex> lk2(s->mu);
        s->host_in_use -= std::min(s->host_in_use, r->host_bytes);
        s->stats.host_in_use = s->host_in_use;
        s->cv_work.notify_one();
    }
    delete r;
    return st;
}

extern "C" sc_status sc_server_cancel(sc_server *s, uint64_t ticket)
{
    if (!s) return fail(SC_E_INVAL, "sc_server_cancel: server is NULL");
    std::lock_guard<std::mutex> lk(s->mu);
    auto it = s->all.find(ticket);
    if (it == s->all.end()) return fail(SC_E_INVAL, "sc_server_cancel: unknown ticket");
    Req *r = it->second;
    if (r->state != R_QUEUED) return fail(SC_E_STATE, "sc_server_cancel: request already admitted");
    s->queue.erase(std::remove(s->queue.begin(), s->queue.end(), r), s->queue.end());
    r->state = R_CANCELLED;
    s->stats.queued--;
    s->stats.cancelled++;
    s->cv_done.notify_all();
    return SC_OK;
}

extern "C" sc_status sc_server_get_stats(sc_server *s, sc_server_stats *out)
{
    if (!s || !out) return fail(SC_E_INVAL, "sc_server_get_stats: NULL argument");
    std::lock_guard<std::mutex> lk(s->mu);
    *out = s->stats;
    return SC_OK;
}

extern "C" sc_status sc_server_destroy(sc_server *s)
{
    if (!s) return SC_OK;
    {
        std::lock_guard<std::mutex> lk(s->mu);
        s->stop = true;
        for (Req *r : s->queue) {
            r->state = R_CANCELLED;
            s->stats.cancelled++;
        }
        s->queue.clear();
        s->stats.queued = 0;
        s->cv_done.notify_all();
    }
    s->cv_work.notify_all();
    s->cv_prep.notify_all();
    if (s->worker.joinable()) s->worker.join();
    {
        std::lock_guard<std::mutex> lk(s->mu);
        s->cv_prep.notify_all();
    }
    if (s->preparer.joinable()) s->preparer.join();
    DeviceGuard g(s->ctx->device);
    (void)hipStreamSynchronize(s->ctx->stream);
    (void)hipStreamSynchronize(s->copy_stream);
    for (sc_prob *p : s->to_release) (void)sc_prob_destroy(p);
    s->to_release.clear();
    for (auto &kv : s->all) {
        release_prob(kv.second);
        free_req_host(s, kv.second);
        delete kv.second;
    }
    s->all.clear();
    s->pinned.clear();
    (void)hipStreamSynchronize(s->release_stream);
    (void)hipStreamDestroy(s->release_stream);
    pool_cache_release(s);
    (void)hipStreamDestroy(s->copy_stream);
    for (int i = 0; i < sc_server::RING; ++i) {
        if (s->slot_ev[i]) (void)hipEventDestroy(s->slot_ev[i]);
        if (s->slot_start[i]) (void)hipEventDestroy(s->slot_start[i]);
        if (s->hjobs[i]) (void)hipHostFree(s->hjobs[i]);
        s->jobbuf[i].release();
    }
    (void)sc_ctx_destroy(s->prep);
    s->ctx->n_probs--;
    delete s;
    return SC_OK;
}
