// abi_sanitized.cpp -- drives the library's C ABI through its main paths with the
// host code built under a sanitizer (AddressSanitizer, on the host side only; the
// gfx950 kernels are the library's own): set-up of every
// incident-field kind, the three precisions and table layouts, results in host
// memory, the time transform, a batch, evaluation without allocation, the
// launch tuner on a small problem, error returns, and a serving loop fed from
// two client threads with cancellations and a shutdown while requests are
// still queued.  Exits 0 and prints one line when every call returned as
// expected; a sanitizer report ends the process with an error first.
#include <hip/hip_runtime_api.h>
#include <sc.h>

#include <atomic>
#include <cmath>
#include <complex>
#include <cstdio>
#include <cstdlib>
#include <thread>
#include <vector>

static int failures = 0;

#define EXPECT(call, want)                                                                           \
    do {                                                                                             \
        const sc_status st_ = (call);                                                                \
        if (st_ != (want)) {                                                                         \
            std::fprintf(stderr, "%s:%d: %s returned %d (%s), expected %d\n", __FILE__, __LINE__, #call, \
                         (int)st_, sc_last_error(), (int)(want));                                   \
            ++failures;                                                                              \
        }                                                                                            \
    } while (0)

static std::vector<double> ks(int n)
{
    std::vector<double> k(n);
    for (int i = 0; i < n; ++i) k[i] = 2.0 * M_PI * (0.9 + 0.1 * i);
    return k;
}

static std::vector<double> points(int n)
{
    std::vector<double> o(3 * n);
    for (int i = 0; i < n; ++i) {
        o[3 * i] = 0.05 * std::cos(0.7 * i);
        o[3 * i + 1] = 0.05 * std::sin(1.3 * i);
        o[3 * i + 2] = 0.02 * (i % 5) - 0.04;
    }
    return o;
}

static sc_prob *problem(sc_ctx *ctx, int n_k, int n_obs, int kind)
{
    sc_prob *p = nullptr;
    EXPECT(sc_prob_create(ctx, &p), SC_OK);
    EXPECT(sc_set_mirror(p, 20.0, 25.0, 24 + 4 * kind, 16), SC_OK);
    const std::vector<double> k = ks(n_k);
    EXPECT(sc_set_frequencies(p, k.data(), n_k), SC_OK);
    std::vector<double> spec(2 * n_k);
    for (int i = 0; i < n_k; ++i) {
        spec[2 * i] = 1.0 / (1 + i);
        spec[2 * i + 1] = 0.1 * i;
    }
    if (kind == 0) {
        EXPECT(sc_set_incident_gaussian(p, 12.0, 0.3, spec.data(), 0), SC_OK);
    } else if (kind == 1) {
        EXPECT(sc_set_incident_beam(p, SC_BEAM_RADIAL, 12.0, 0.0, spec.data(), 1), SC_OK);
    } else if (kind == 2) {
        sc_lg_mode m[2] = {{0, 1, {1.0, 0.0}, {0.0, 0.0}}, {1, -1, {0.2, 0.1}, {0.0, 0.3}}};
        EXPECT(sc_set_incident_lg(p, m, 2, 12.0, spec.data()), SC_OK);
    } else {
        int ns = 0, nr = 0;
        EXPECT(sc_get_num_nodes(p, &ns, &nr), SC_OK);
        const size_t n = (size_t)n_k * (ns + nr) * 3;
        std::vector<std::complex<double>> E(n), B(n);
        for (size_t i = 0; i < n; ++i) {
            E[i] = {std::sin(0.1 * i), std::cos(0.3 * i)};
            B[i] = {std::cos(0.2 * i), -std::sin(0.5 * i)};
        }
        EXPECT(sc_set_incident(p, (const double *)E.data(), (const double *)B.data(), 0), SC_OK);
    }
    const std::vector<double> o = points(n_obs);
    EXPECT(sc_set_observation(p, o.data(), n_obs, 0), SC_OK);
    return p;
}

static void single_problems(sc_ctx *ctx)
{
    const int n_k = 3, n_obs = 70, n_t = 5;
    for (int kind = 0; kind < 4; ++kind) {
        sc_prob *p = problem(ctx, n_k, n_obs, kind);
        for (int layout = 0; layout <= 2; ++layout) {
            EXPECT(sc_set_factoring(p, layout), SC_OK);
            for (sc_precision prec : {SC_FP64, SC_FP32_SPLIT, SC_FP32}) {
                const size_t rs = prec == SC_FP64 ? sizeof(double) : sizeof(float);
                std::vector<char> E(rs * 6 * n_k * n_obs), B(E.size());
                EXPECT(sc_evaluate(p, prec, E.data(), B.data(), 0), SC_OK);
                std::vector<char> Et(rs * 6 * n_t * n_obs), Bt(Et.size());
                EXPECT(sc_to_time(p, -1.0, 0.5, n_t, Et.data(), Bt.data(), 0), SC_OK);
                int active = -1;
                EXPECT(sc_get_factoring_for(p, prec, &active), SC_OK);
            }
        }
        sc_timing tm{};
        EXPECT(sc_get_timing(p, &tm), SC_OK);
        size_t bytes = 0;
        EXPECT(sc_prob_device_bytes(p, &bytes), SC_OK);
        EXPECT(sc_prob_destroy(p), SC_OK);
    }
}

static void batch_noalloc_tune(sc_ctx *ctx)
{
    std::vector<sc_prob *> probs;
    for (int i = 0; i < 4; ++i) probs.push_back(problem(ctx, 2 + i, 40 + 30 * i, i % 3));
    EXPECT(sc_evaluate_batch(ctx, probs.data(), (int)probs.size(), SC_FP32_SPLIT), SC_OK);
    std::vector<float> E(6 * 5 * 130), B(E.size());
    EXPECT(sc_get_result(probs[3], E.data(), B.data(), 0), SC_OK);
    // evaluation without allocation, into device buffers of the result's size (2 frequencies x 40 points)
    EXPECT(sc_evaluate(probs[0], SC_FP32_SPLIT, nullptr, nullptr, 0), SC_OK);
    EXPECT(sc_evaluate_noalloc(probs[0], SC_FP32_SPLIT, nullptr, nullptr), SC_E_INVAL);
    void *dE = nullptr, *dB = nullptr;
    const size_t bytes = sizeof(float) * 6 * 2 * 40;
    if (hipMalloc(&dE, bytes) != hipSuccess || hipMalloc(&dB, bytes) != hipSuccess) {
        std::fprintf(stderr, "hipMalloc failed\n");
        ++failures;
    } else {
        EXPECT(sc_evaluate_noalloc(probs[0], SC_FP32_SPLIT, dE, dB), SC_OK);
        EXPECT(sc_ctx_synchronize(ctx), SC_OK);
        std::vector<float> Eh(6 * 2 * 40), Ea(Eh.size()), Ba(Eh.size());
        EXPECT(sc_get_result(probs[0], Ea.data(), Ba.data(), 0), SC_OK);
        if (hipMemcpy(Eh.data(), dE, bytes, hipMemcpyDeviceToHost) != hipSuccess || Eh != Ea) {
            std::fprintf(stderr, "evaluation without allocation differs from the stored result\n");
            ++failures;
        }
        (void)hipFree(dE);
        (void)hipFree(dB);
    }
    sc_launch best{};
    EXPECT(sc_autotune(probs[1], SC_FP32_SPLIT, 50.0, &best), SC_OK);
    for (sc_prob *p : probs) EXPECT(sc_prob_destroy(p), SC_OK);
}

static void error_returns(sc_ctx *ctx)
{
    sc_prob *p = nullptr;
    EXPECT(sc_prob_create(ctx, &p), SC_OK);
    EXPECT(sc_evaluate(p, SC_FP32_SPLIT, nullptr, nullptr, 0), SC_E_STATE);
    EXPECT(sc_set_mirror(p, -1.0, 25.0, 10, 8), SC_E_INVAL);
    EXPECT(sc_set_mirror(p, 20.0, 25.0, 10, 8), SC_OK);
    EXPECT(sc_set_frequencies(p, nullptr, 3), SC_E_INVAL);
    EXPECT(sc_set_factoring(p, 3), SC_E_INVAL);
    EXPECT(sc_evaluate(p, (sc_precision)7, nullptr, nullptr, 0), SC_E_INVAL);
    EXPECT(sc_prob_destroy(p), SC_OK);
    EXPECT(sc_prob_create(nullptr, &p), SC_E_INVAL);
}

static void serving(sc_ctx *ctx)
{
    sc_server *s = nullptr;
    EXPECT(sc_server_create(ctx, (size_t)8 << 30, 16, 5.0, &s), SC_OK);
    const int n_clients = 2, per_client = 24;
    std::atomic<int> done{0};
    auto client = [&](int c) {
        for (int i = 0; i < per_client; ++i) {
            const int n_k = 1 + (i % 4), n_obs = 16 + 8 * (i % 5), n_t = (i % 3) ? 4 : 0;
            const std::vector<double> k = ks(n_k), o = points(n_obs);
            std::vector<double> t(n_t ? n_t : 1);
            for (int j = 0; j < n_t; ++j) t[j] = -1.0 + 0.5 * j;
            sc_request r{};
            r.f = 20.0;
            r.r_max = 25.0;
            r.n_r = 20 + 2 * (i % 3);
            r.n_phi = 12;
            r.n_k = n_k;
            r.k = k.data();
            r.w0 = 12.0;
            r.pol_angle = 0.2 * c;
            r.consistent = i % 2;
            r.n_obs = n_obs;
            r.obs = o.data();
            r.prec = (i % 3 == 0) ? SC_FP64 : SC_FP32_SPLIT;
            r.n_t = n_t;
            r.t = n_t ? t.data() : nullptr;
            r.dk = 0.25;
            r.beam = i % 3;
            uint64_t ticket = 0;
            EXPECT(sc_server_submit(s, &r, &ticket), SC_OK);
            const size_t rs = r.prec == SC_FP64 ? sizeof(double) : sizeof(float);
            std::vector<char> E(rs * 6 * n_k * n_obs), B(E.size()), Et(rs * 6 * (n_t ? n_t : 1) * n_obs),
                Bt(Et.size());
            if (i % 7 == 3) {   // cancel: either it is cancelled or it had started and completes
                (void)sc_server_cancel(s, ticket);
                const sc_status st = sc_server_wait(s, ticket, -1.0, E.data(), B.data(), n_t ? Et.data() : nullptr,
                                                    n_t ? Bt.data() : nullptr, nullptr);
                if (st != SC_OK && st != SC_E_CANCELLED) {
                    std::fprintf(stderr, "cancelled wait returned %d\n", (int)st);
                    ++failures;
                }
            } else {
                sc_request_stats rst{};
                EXPECT(sc_server_wait(s, ticket, -1.0, E.data(), B.data(), n_t ? Et.data() : nullptr,
                                      n_t ? Bt.data() : nullptr, &rst),
                       SC_OK);
            }
        }
        done++;
    };
    std::vector<std::thread> th;
    for (int c = 0; c < n_clients; ++c) th.emplace_back(client, c);
    for (auto &t : th) t.join();
    sc_server_stats st{};
    EXPECT(sc_server_get_stats(s, &st), SC_OK);
    // requests still queued when the server stops: submitted, never waited for
    for (int i = 0; i < 6; ++i) {
        const std::vector<double> k = ks(2), o = points(24);
        sc_request r{};
        r.f = 20.0;
        r.r_max = 25.0;
        r.n_r = 20;
        r.n_phi = 12;
        r.n_k = 2;
        r.k = k.data();
        r.w0 = 12.0;
        r.n_obs = 24;
        r.obs = o.data();
        r.prec = SC_FP32_SPLIT;
        uint64_t ticket = 0;
        EXPECT(sc_server_submit(s, &r, &ticket), SC_OK);
    }
    EXPECT(sc_server_destroy(s), SC_OK);
}

int main()
{
    sc_ctx *ctx = nullptr;
    EXPECT(sc_ctx_create(0, nullptr, &ctx), SC_OK);
    if (!ctx) return 2;
    EXPECT(sc_ctx_set_profiling(ctx, 1), SC_OK);
    single_problems(ctx);
    batch_noalloc_tune(ctx);
    error_returns(ctx);
    EXPECT(sc_ctx_synchronize(ctx), SC_OK);
    serving(ctx);
    EXPECT(sc_ctx_destroy(ctx), SC_OK);
    if (failures) {
        std::fprintf(stderr, "%d unexpected returns\n", failures);
        return 1;
    }
    std::printf("C ABI paths clean under the sanitizer\n");
    return 0;
}
