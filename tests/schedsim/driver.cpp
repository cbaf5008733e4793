// Drives the serving scheduler of the library's host runtime, built for the
// CPU against the HIP stand-in (tests/schedsim), through the scenarios the
// GPU tests use, randomised streams and streams of both arithmetic paths,
// and checks that every request completes, within a time limit, with the
// value of its lone evaluation.
// Exit status 0 when all scenarios pass; 1 on a wrong value or status; 3 when
// a scenario does not finish in time (the scheduler hung).
#include <atomic>
#include <chrono>
#include <cmath>
#include <cstdio>
#include <cstdlib>
#include <random>
#include <thread>
#include <vector>

#include "../../include/tor.h"

namespace {
int g_fail = 0;
std::atomic<int> g_phase{0};
std::atomic<bool> g_done{false};

void check(bool ok, const char *what, int i = -1)
{
    if (!ok) {
        std::fprintf(stderr, "check failed: %s (%d)\n", what, i);
        g_fail = 1;
    }
}

// a 2n x 2n complex matrix whose first entry is c, with imaginary part 1 for
// general Hermitian input (the stand-in reads only that entry)
std::vector<double> matrix(int n, double c, bool general = false)
{
    std::vector<double> m(8 * (size_t)n * n, 0.0);
    m[0] = c;
    m[1] = general ? 1.0 : 0.0;
    return m;
}

struct Req {
    int n;
    std::vector<double> O;
    unsigned long long ticket = 0;
    tor_result lone{}, served{};
};

void serve_and_check(tor_ctx *ctx, std::vector<Req> &rs, std::mt19937_64 *rng, int max_gap_us, const char *name)
{
    for (auto &r : rs)
        check(tor_eval(ctx, r.n, r.O.data(), 2L * r.n, &r.lone) == TOR_OK, "lone eval");
    std::uniform_int_distribution<int> gap(0, std::max(max_gap_us, 0));
    for (size_t i = 0; i < rs.size(); i++) {
        int rc;
        while ((rc = tor_submit(ctx, rs[i].n, rs[i].O.data(), 2L * rs[i].n, &rs[i].ticket)) == TOR_E_BUSY)
            std::this_thread::sleep_for(std::chrono::microseconds(50));
        check(rc == TOR_OK, "submit", (int)i);
        if (rng && max_gap_us > 0)
            std::this_thread::sleep_for(std::chrono::microseconds(gap(*rng)));
    }
    check(tor_drain(ctx, 60000) == TOR_OK, "drain");
    for (size_t i = 0; i < rs.size(); i++) {
        check(tor_poll(ctx, rs[i].ticket, &rs[i].served) == TOR_OK, "poll", (int)i);
        check(rs[i].served.status == TOR_OK, "served status", (int)i);
        check(rs[i].served.tor == rs[i].lone.tor && rs[i].served.tor_lo == rs[i].lone.tor_lo &&
                  rs[i].served.sum_abs == rs[i].lone.sum_abs,
              "served value equals the lone one", (int)i);
        check(rs[i].served.tor != 0.0, "nonzero value", (int)i);
    }
    std::printf("%s: %zu requests done\n", name, rs.size());
    std::fflush(stdout);
}
}  // namespace

int main(int argc, char **argv)
{
    const double limit_s = argc > 1 ? std::atof(argv[1]) : 120.0;
    std::thread watchdog([limit_s] {
        const auto t0 = std::chrono::steady_clock::now();
        while (!g_done.load()) {
            std::this_thread::sleep_for(std::chrono::milliseconds(50));
            if (std::chrono::duration<double>(std::chrono::steady_clock::now() - t0).count() > limit_s) {
                std::fprintf(stderr, "timeout in scenario %d\n", g_phase.load());
                std::fflush(stderr);
                std::_Exit(3);
            }
        }
    });
    tor_options opt;
    tor_default_options(&opt);
    opt.max_n = 34;
    tor_ctx *ctx = nullptr;
    if (tor_create(&ctx, &opt) != TOR_OK) {
        std::fprintf(stderr, "tor_create failed\n");
        return 4;
    }
    std::mt19937_64 rng(12345);

    // 1: the sizes and policy of the sanitized GPU driver
    g_phase = 1;
    {
        check(tor_serve_config(ctx, 1 << 20, 1 << 12, 0.5, 64) == TOR_OK, "config");
        std::vector<Req> rs;
        int i = 0;
        for (int n : {5, 8, 10, 12, 14, 16, 20})
            rs.push_back(Req{n, matrix(n, 1.0 + 0.125 * i++)});
        serve_and_check(ctx, rs, nullptr, 0, "sanitized-driver sizes");
    }
    // 2: express and chunked requests mixed, arriving over time
    g_phase = 2;
    {
        check(tor_serve_config(ctx, 1 << 22, 1 << 16, 0.5, 1 << 16) == TOR_OK, "config");
        std::vector<Req> rs;
        std::uniform_int_distribution<int> nd(8, 26);
        for (int i = 0; i < 300; i++) {
            const int n = nd(rng);
            rs.push_back(Req{n, matrix(n, 1.0 + i / 1024.0)});
        }
        serve_and_check(ctx, rs, &rng, 200, "mixed stream");
    }
    // 3: all at once, default policy
    g_phase = 3;
    {
        check(tor_serve_config(ctx, 1ll << 30, 1ll << 24, 0.5, 1 << 16) == TOR_OK, "config");
        std::vector<Req> rs;
        std::uniform_int_distribution<int> nd(8, 30);
        for (int i = 0; i < 200; i++) {
            const int n = nd(rng);
            rs.push_back(Req{n, matrix(n, 2.0 + i / 1024.0)});
        }
        serve_and_check(ctx, rs, nullptr, 0, "saturated default policy");
    }
    // 4: small chunks, no express launches, a second wave while the first runs
    g_phase = 4;
    {
        check(tor_serve_config(ctx, 1 << 18, 0, 0.5, 1 << 16) == TOR_OK, "config");
        std::vector<Req> rs;
        for (int i = 0; i < 40; i++) {
            const int n = 14 + (i % 11);
            rs.push_back(Req{n, matrix(n, 3.0 + i / 64.0)});
        }
        serve_and_check(ctx, rs, &rng, 500, "chunks only");
    }
    // 5: both arithmetic paths in one stream (the lanes take the paths in turn)
    g_phase = 5;
    {
        check(tor_serve_config(ctx, 1 << 21, 1 << 14, 0.5, 1 << 16) == TOR_OK, "config");
        std::vector<Req> rs;
        std::uniform_int_distribution<int> nd(8, 24);
        for (int i = 0; i < 200; i++) {
            const int n = nd(rng);
            rs.push_back(Req{n, matrix(n, 5.0 + i / 1024.0, i % 3 == 1)});
        }
        serve_and_check(ctx, rs, &rng, 100, "both paths");
        int cplx = 0;
        for (auto &r : rs)
            cplx += r.served.path == 2;
        check(cplx > 0 && cplx < (int)rs.size(), "both paths served");
    }
    // 6: destroy with requests in flight
    g_phase = 6;
    {
        check(tor_serve_config(ctx, 1 << 20, 1 << 12, 0.5, 1 << 16) == TOR_OK, "config");
        std::vector<Req> rs;
        for (int i = 0; i < 30; i++) {
            const int n = 10 + (i % 17);
            rs.push_back(Req{n, matrix(n, 4.0 + i / 64.0)});
        }
        for (auto &r : rs)
            check(tor_submit(ctx, r.n, r.O.data(), 2L * r.n, &r.ticket) == TOR_OK, "submit");
        std::this_thread::sleep_for(std::chrono::milliseconds(2));
    }
    tor_destroy(ctx);
    g_done = true;
    watchdog.join();
    std::printf("done %d\n", g_fail);
    return g_fail;
}
