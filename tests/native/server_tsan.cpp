// server_tsan.cpp -- concurrency check of the serving loop on the CPU.
//
// server.cpp runs on the data-free stub executor (server_stub.cpp), built
// with ThreadSanitizer: several client threads submit pack and unpack
// requests of mixed sizes against a small admission budget (so requests
// queue, batch and wait for memory), test or wait for them, read their
// results and release them, while the progress thread runs, another thread
// drives progress rounds of its own and one reads the statistics.  Then the
// same without a progress thread, with injected arena failures, and a free
// that drains queued requests.  Every request must complete exactly once with
// the right byte count and the counters must balance; a data race makes
// ThreadSanitizer fail the run.  Prints "server tsan ok".
#include <atomic>
#include <chrono>
#include <cstdlib>
#include <functional>
#include <cstdio>
#include <random>
#include <thread>
#include <vector>

#include "mdt.h"

mdt_type stub_type(int64_t size, int64_t extent);
int64_t stub_launches();

#define CHECK(cond)                                                                  \
    do {                                                                             \
        if (!(cond)) {                                                               \
            std::fprintf(stderr, "%s:%d: check failed: %s\n", __FILE__, __LINE__, #cond); \
            std::exit(1);                                                            \
        }                                                                            \
    } while (0)

namespace {

struct Pending {
    mdt_request r;
    int64_t bytes;
};

std::atomic<int64_t> g_done{0}, g_failed{0}, g_bytes{0};

void client(mdt_server srv, const std::vector<mdt_type> &types, int id, int nreq, bool use_wait)
{
    std::mt19937_64 g(1234 + (uint64_t)id);
    static uint8_t dummy[64];
    std::vector<Pending> pend;
    auto finish = [&](Pending &p) {
        int st = -1;
        void *pk = nullptr;
        mdt_count nb = -1;
        double lat = -1;
        CHECK(mdt_server_request_result(srv, p.r, &st, &pk, &nb, &lat) == MDT_SUCCESS);
        if (st == MDT_SUCCESS) {
            CHECK(nb == p.bytes && lat >= 0);
            g_done++;
            g_bytes += nb;
        } else {
            CHECK(st == MDT_ERR_NO_MEM);
            g_failed++;
        }
        CHECK(mdt_server_request_release(srv, &p.r) == MDT_SUCCESS && p.r == nullptr);
    };
    for (int i = 0; i < nreq; i++) {
        mdt_type t = types[g() % types.size()];
        // sizes from 64 B to 4 MiB, most of them small
        const int64_t want = (int64_t)64 << (g() % 17);
        mdt_request r = nullptr;
        int64_t bytes;
        if (g() & 1) {
            const int64_t count = 1 + want / 64;
            CHECK(mdt_server_submit_pack(srv, dummy, count, t, 0, want, &r) == MDT_SUCCESS);
            bytes = want;
        } else {
            CHECK(mdt_server_submit_unpack(srv, dummy, want, dummy, 1 + want / 64, t, 0, &r) == MDT_SUCCESS);
            bytes = want;
        }
        pend.push_back({r, bytes});
        // test the oldest few now and then; wait when many are pending
        if (pend.size() > 24 || (i % 7) == 0) {
            for (size_t k = 0; k < pend.size();) {
                int flag = 0;
                if (use_wait && pend.size() > 24 && k == 0) {
                    CHECK(mdt_server_request_wait(srv, pend[k].r) == MDT_SUCCESS);
                    flag = 1;
                } else {
                    CHECK(mdt_server_request_test(srv, pend[k].r, &flag) == MDT_SUCCESS);
                }
                if (flag) {
                    finish(pend[k]);
                    pend.erase(pend.begin() + (long)k);
                } else {
                    k++;
                }
            }
        }
    }
    for (auto &p : pend) {
        CHECK(mdt_server_request_wait(srv, p.r) == MDT_SUCCESS);
        finish(p);
    }
}

void run(bool thread, int inject)
{
    std::vector<mdt_type> types;
    for (int k = 0; k < 6; k++) types.push_back(stub_type(64, 64 + 16 * k));  // 64 packed bytes per element
    mdt_server_config cfg{8, (mdt_count)24 << 20, 16, 2, (mdt_count)24 << 20};
    mdt_server srv = nullptr;
    CHECK(mdt_server_create(&cfg, &srv) == MDT_SUCCESS);
    if (thread) CHECK(mdt_server_start_progress_thread(srv) == MDT_SUCCESS);
    if (inject) CHECK(mdt_server_inject_alloc_failures(srv, inject) == MDT_SUCCESS);
    g_done = g_failed = g_bytes = 0;
    const int nclients = 4, nreq = 1500;
    std::atomic<bool> stop{false};
    std::thread stats([&] {
        while (!stop.load()) {
            mdt_server_stats s{};
            CHECK(mdt_server_stats_get(srv, &s) == MDT_SUCCESS);
            CHECK(s.completed + s.failed <= s.submitted);
            std::this_thread::sleep_for(std::chrono::microseconds(200));
        }
    });
    std::thread driver([&] {  // progress rounds from a caller beside the progress thread
        while (!stop.load()) {
            CHECK(mdt_server_progress(srv) == MDT_SUCCESS);
            std::this_thread::sleep_for(std::chrono::microseconds(50));
        }
    });
    std::vector<std::thread> cl;
    for (int c = 0; c < nclients; c++) cl.emplace_back(client, srv, std::cref(types), c, nreq, c % 2 == 0);
    for (auto &t : cl) t.join();
    stop = true;
    stats.join();
    driver.join();
    mdt_server_stats s{};
    CHECK(mdt_server_stats_get(srv, &s) == MDT_SUCCESS);
    CHECK(s.submitted == (mdt_count)nclients * nreq);
    CHECK(g_done + g_failed == s.submitted && s.completed == g_done && s.failed == g_failed);
    CHECK(g_failed == inject && s.bytes == g_bytes);
    CHECK(s.inflight_bytes == 0 && s.peak_inflight_bytes <= cfg.budget_bytes + ((mdt_count)4 << 20) * 2);
    CHECK(s.launches > 0 && s.p99_us >= s.p50_us);
    if (thread) CHECK(mdt_server_stop_progress_thread(srv) == MDT_SUCCESS);
    // queued requests are drained by free
    static uint8_t dummy[64];
    std::vector<mdt_request> more(40);
    for (auto &r : more) CHECK(mdt_server_submit_pack(srv, dummy, 1 << 12, types[0], 0, -1, &r) == MDT_SUCCESS);
    CHECK(mdt_server_free(&srv) == MDT_SUCCESS && srv == nullptr);
    std::printf("  thread=%d inject=%d: %lld done, %lld failed, %lld launches so far, deferred %lld\n", (int)thread,
                inject, (long long)g_done.load(), (long long)g_failed.load(), (long long)stub_launches(),
                (long long)s.deferred);
}

}  // namespace

int main()
{
    run(true, 0);
    run(false, 0);
    run(true, 5);
    std::printf("server tsan ok\n");
    return 0;
}
