// loadgen.cpp -- open-loop load generator for the serving workload, written
// against the public C ABI only (include/mdt.h).  Built as its own shared
// library (libmdt_loadgen.so); bench.py drives it.
//
// A trace is a list of requests (arrival time, pack or unpack, type, count,
// byte range [0, target)), generated on the Python side from seeded inputs.
// Two runs replay the same trace open loop (requests are issued at their
// scheduled time, latency = completion seen by the host - scheduled arrival,
// so a slow issuer cannot hide queueing):
//   served:      every request goes to an mdt_server (continuous batching on
//                its own streams, admission by memory);
//   per-request: every request is one plain stream-ordered launch on stream
//                (id mod nstreams), completion polled through its event.
#include <hip/hip_runtime_api.h>

#include <algorithm>
#include <atomic>
#include <chrono>
#include <cstdint>
#include <cstring>
#include <deque>
#include <thread>
#include <vector>

#include "../../include/mdt.h"

extern "C" {

struct mdt_lg_req {
    double t_arrive_us;   // scheduled arrival, from the start of the run
    int32_t unpack;       // 0 pack, 1 unpack
    int32_t type_index;
    int64_t count;
    int64_t target;       // bytes [0, target) of the stream
    const void *typed;    // pack source / unpack destination origin
    const void *packed;   // unpack input
    void *out;            // pack output (per-request mode)
};

struct mdt_lg_result {
    int64_t completed, failed;
    int64_t bytes;
    double elapsed_s;     // first arrival to last completion
    double p50_us, p99_us, max_us, mean_us;
    int64_t launches;
    int64_t late_issues;  // requests issued more than 50 us after their scheduled time
    double p50_queue_us, p99_queue_us, p50_run_us, p99_run_us;  // served: server-side split
    double p50_issue_us, p99_issue_us;  // duration of the submit / enqueue call
};

}  // extern "C"

namespace {

double now_us()
{
    using namespace std::chrono;
    return (double)duration_cast<nanoseconds>(steady_clock::now().time_since_epoch()).count() * 1e-3;
}

// Between arrivals the issuing thread polls: a timed sleep on Linux lasts
// tens of microseconds longer than asked (timer slack), which would show up
// as latency of whatever completes meanwhile.  It sleeps only when the next
// arrival is more than a millisecond away, and wakes well before it.
void wait_for_next(double t_next)
{
    const double gap = t_next - now_us();
    if (gap > 1000.0) std::this_thread::sleep_for(std::chrono::microseconds((int64_t)(gap - 500.0)));
}

double pctl(std::vector<double> v, double f)
{
    if (v.empty()) return 0.0;
    std::sort(v.begin(), v.end());
    return v[std::min(v.size() - 1, (size_t)(f * (double)(v.size() - 1) + 0.5))];
}

void summarize(std::vector<double> &lat, mdt_lg_result *r)
{
    if (lat.empty()) return;
    std::sort(lat.begin(), lat.end());
    auto q = [&](double f) { return lat[std::min(lat.size() - 1, (size_t)(f * (double)(lat.size() - 1) + 0.5))]; };
    r->p50_us = q(0.50);
    r->p99_us = q(0.99);
    r->max_us = lat.back();
    double s = 0;
    for (double x : lat) s += x;
    r->mean_us = s / (double)lat.size();
}

}  // namespace

extern "C" {

// Serve the trace through an mdt_server (progress thread on).  Pack outputs
// live in the server's arena and are released as soon as they complete.
// lat_out (optional, n entries): each request's latency in us, -1 if it failed.
__attribute__((visibility("default"))) int mdt_lg_run_served(const mdt_lg_req *reqs, int64_t n, const mdt_type *types,
                                                             const mdt_server_config *cfg, mdt_lg_result *res,
                                                             double *lat_out)
{
    std::memset(res, 0, sizeof *res);
    if (lat_out)
        for (int64_t k = 0; k < n; k++) lat_out[k] = -1.0;
    mdt_server srv = nullptr;
    int rc = mdt_server_create(cfg, &srv);
    if (rc) return rc;
    rc = mdt_server_start_progress_thread(srv);
    if (rc) {
        mdt_server_free(&srv);
        return rc;
    }
    struct Pending {
        mdt_request r;
        double t_arrive;
        int64_t idx;
    };
    std::deque<Pending> pend;
    std::vector<double> lat, issue;
    lat.reserve((size_t)n);
    issue.reserve((size_t)n);
    const double t0 = now_us() + 1000.0;
    double last_done = t0;
    int64_t i = 0;
    auto reap = [&](bool all) {
        while (!pend.empty()) {
            // complete in any order: scan a window of the oldest requests
            bool progressed = false;
            size_t lim = std::min<size_t>(pend.size(), 4096);
            for (size_t k = 0; k < lim; k++) {
                if (!pend[k].r) continue;
                int flag = 0;
                mdt_server_request_test(srv, pend[k].r, &flag);
                if (!flag) continue;
                int st = 0;
                double l = 0;
                int64_t nb = 0;
                mdt_server_request_result(srv, pend[k].r, &st, nullptr, &nb, &l);
                double t = now_us();
                if (st == MDT_SUCCESS) {
                    res->completed++;
                    res->bytes += nb;
                    lat.push_back(t - pend[k].t_arrive);
                    if (lat_out) lat_out[pend[k].idx] = t - pend[k].t_arrive;
                } else {
                    res->failed++;
                }
                last_done = std::max(last_done, t);
                mdt_server_request_release(srv, &pend[k].r);
                pend[k].r = nullptr;
                progressed = true;
            }
            while (!pend.empty() && pend.front().r == nullptr) pend.pop_front();
            if (!all || !progressed) break;
        }
    };
    while (i < n || !pend.empty()) {
        double t = now_us();
        while (i < n && t0 + reqs[i].t_arrive_us <= t) {
            const mdt_lg_req &q = reqs[i];
            mdt_request r = nullptr;
            int e;
            const double ti = now_us();
            if (q.unpack)
                e = mdt_server_submit_unpack(srv, q.packed, q.target, const_cast<void *>(q.typed), q.count,
                                             types[q.type_index], 0, &r);
            else
                e = mdt_server_submit_pack(srv, q.typed, q.count, types[q.type_index], 0, q.target, &r);
            issue.push_back(now_us() - ti);
            if (t - (t0 + q.t_arrive_us) > 50.0) res->late_issues++;
            if (e) res->failed++;
            else pend.push_back({r, t0 + q.t_arrive_us, i});
            i++;
        }
        reap(false);
        wait_for_next(i < n ? t0 + reqs[i].t_arrive_us : 0.0);
    }
    mdt_server_stats st{};
    mdt_server_stats_get(srv, &st);
    res->launches = st.launches;
    res->p50_queue_us = st.p50_queue_us;
    res->p99_queue_us = st.p99_queue_us;
    res->p50_run_us = st.p50_run_us;
    res->p99_run_us = st.p99_run_us;
    mdt_server_free(&srv);
    res->elapsed_s = (last_done - t0) * 1e-6;
    summarize(lat, res);
    res->p50_issue_us = pctl(issue, 0.50);
    res->p99_issue_us = pctl(issue, 0.99);
    return MDT_SUCCESS;
}

// One plain launch per request on stream (index mod nstreams).
__attribute__((visibility("default"))) int mdt_lg_run_plain(const mdt_lg_req *reqs, int64_t n, const mdt_type *types,
                                                            int nstreams, mdt_lg_result *res, double *lat_out)
{
    std::memset(res, 0, sizeof *res);
    if (lat_out)
        for (int64_t k = 0; k < n; k++) lat_out[k] = -1.0;
    std::vector<hipStream_t> hs((size_t)nstreams);
    std::vector<mdt_stream> ms((size_t)nstreams);
    for (int s = 0; s < nstreams; s++) {
        if (hipStreamCreateWithFlags(&hs[s], hipStreamNonBlocking) != hipSuccess) return MDT_ERR_HIP;
        mdt_stream_create(reinterpret_cast<mdt_hip_stream>(hs[s]), &ms[s]);
    }
    struct Pending {
        mdt_request r;
        double t_arrive;
        int64_t bytes;
        int64_t idx;
    };
    // requests on one stream complete in order: poll only each stream's oldest
    std::vector<std::deque<Pending>> pend((size_t)nstreams);
    int64_t npend = 0;
    std::vector<double> lat, issue;
    lat.reserve((size_t)n);
    issue.reserve((size_t)n);
    const double t0 = now_us() + 1000.0;
    double last_done = t0;
    int64_t i = 0;
    while (i < n || npend > 0) {
        double t = now_us();
        while (i < n && t0 + reqs[i].t_arrive_us <= t) {
            const mdt_lg_req &q = reqs[i];
            mdt_request r = nullptr;
            int64_t got = 0;
            mdt_stream s = ms[(size_t)(i % nstreams)];
            int e;
            const double ti = now_us();
            if (q.unpack)
                e = mdt_unpack_enqueue(q.packed, q.target, const_cast<void *>(q.typed), q.count, types[q.type_index], 0,
                                       &got, s, &r);
            else
                e = mdt_pack_enqueue(q.typed, q.count, types[q.type_index], 0, q.out, q.target, &got, s, &r);
            issue.push_back(now_us() - ti);
            if (t - (t0 + q.t_arrive_us) > 50.0) res->late_issues++;
            if (e) res->failed++;
            else {
                pend[(size_t)(i % nstreams)].push_back({r, t0 + q.t_arrive_us, got, i});
                npend++;
                res->launches++;
            }
            i++;
        }
        for (auto &dq : pend) {
            while (!dq.empty()) {
                int flag = 0;
                mdt_test(&dq.front().r, &flag);
                if (!flag) break;
                double tc = now_us();
                res->completed++;
                res->bytes += dq.front().bytes;
                lat.push_back(tc - dq.front().t_arrive);
                if (lat_out) lat_out[dq.front().idx] = tc - dq.front().t_arrive;
                last_done = std::max(last_done, tc);
                dq.pop_front();
                npend--;
            }
        }
        wait_for_next(i < n ? t0 + reqs[i].t_arrive_us : 0.0);
    }
    for (int s = 0; s < nstreams; s++) {
        (void)hipStreamSynchronize(hs[s]);
        mdt_stream_free(&ms[s]);
        (void)hipStreamDestroy(hs[s]);
    }
    res->elapsed_s = (last_done - t0) * 1e-6;
    summarize(lat, res);
    res->p50_issue_us = pctl(issue, 0.50);
    res->p99_issue_us = pctl(issue, 0.99);
    return MDT_SUCCESS;
}

}  // extern "C"
