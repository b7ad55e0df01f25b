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
//
// Destinations never overlap while requests are in flight (the library's
// contract): every request that writes caller memory -- an unpack's typed
// span, a per-request pack's output -- takes its own range of a device ring,
// handed out in issue order and returned when the request completes.  When
// the ring is full the issuer reaps until the oldest range is free (counted
// as ring waits; the wait is part of the waiting requests' latency, since
// latency runs from the scheduled arrival).  Sampled requests write to fixed
// caller buffers instead, so their bytes can be compared after the run
// (served pack results are copied out of the server's arena before release).
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
    const void *typed;    // pack source origin
    const void *packed;   // unpack input
    void *fixed;          // sampled request: its own destination (pack output, or the unpack
                          // span's first byte); NULL: a range of the ring
    int64_t span;         // bytes the request writes: pack output (target), or the unpack's typed span
    int64_t origin_off;   // unpack: the origin is the span's first byte + origin_off (= -true_lb)
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
    int64_t ring_waits;   // issues that waited for a ring range to come free
    double ring_wait_us;  // total time spent waiting for the ring
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


// Destination ring: ranges handed out in issue order over [0, cap), freed
// in any order; the live ranges always form one circular run from the
// oldest (tail) to head.
struct Ring {
    uint8_t *base = nullptr;
    int64_t cap = 0, head = 0;
    struct Range {
        int64_t off, len;
        bool done;
    };
    std::deque<Range> live;
    uint64_t first_id = 0;  // id of live.front()
    static int64_t round(int64_t n) { return std::max<int64_t>(256, (n + 255) / 256 * 256); }
    // returns the range id, or -1 when it does not fit now
    int64_t alloc(int64_t n, int64_t *off)
    {
        n = round(n);
        if (n > cap) return -2;  // never fits
        int64_t at;
        if (live.empty()) {
            at = 0;
        } else {
            const int64_t tail = live.front().off;
            if (head > tail) {  // occupied [tail, head)
                if (head + n <= cap) at = head;
                else if (n <= tail) at = 0;
                else return -1;
            } else {            // wrapped: occupied [tail, cap) and [0, head)
                if (head + n <= tail) at = head;
                else return -1;
            }
        }
        head = at + n;
        live.push_back({at, n, false});
        *off = at;
        return (int64_t)(first_id + live.size() - 1);
    }
    void free(int64_t id)
    {
        if (id < 0) return;
        live[(size_t)((uint64_t)id - first_id)].done = true;
        while (!live.empty() && live.front().done) {
            live.pop_front();
            first_id++;
        }
        if (live.empty()) head = 0;
    }
};

}  // namespace

extern "C" {

// Serve the trace through an mdt_server (progress thread on).  Pack outputs
// live in the server's arena and are released as soon as they complete
// (sampled ones are first copied to their fixed buffer); unpack spans come
// from the ring [ring, ring + ring_bytes).
// lat_out (optional, n entries): each request's latency in us, -1 if it failed.
__attribute__((visibility("default"))) int mdt_lg_run_served(const mdt_lg_req *reqs, int64_t n, const mdt_type *types,
                                                             const mdt_server_config *cfg, void *ring_base,
                                                             int64_t ring_bytes, mdt_lg_result *res, double *lat_out)
{
    std::memset(res, 0, sizeof *res);
    if (lat_out)
        for (int64_t k = 0; k < n; k++) lat_out[k] = -1.0;
    Ring ring;
    ring.base = static_cast<uint8_t *>(ring_base);
    ring.cap = ring_bytes;
    hipStream_t cs = nullptr;  // copies of sampled pack results
    if (hipStreamCreateWithFlags(&cs, hipStreamNonBlocking) != hipSuccess) return MDT_ERR_HIP;
    mdt_server srv = nullptr;
    int rc = mdt_server_create(cfg, &srv);
    if (rc == MDT_SUCCESS) {
        rc = mdt_server_start_progress_thread(srv);
        if (rc) mdt_server_free(&srv);
    }
    if (rc) {
        (void)hipStreamDestroy(cs);
        return rc;
    }
    struct Pending {
        mdt_request r;
        double t_arrive;
        int64_t idx;
        int64_t range;  // ring range id, or -1
    };
    std::deque<Pending> pend;
    std::vector<double> lat, issue;
    lat.reserve((size_t)n);
    issue.reserve((size_t)n);
    const double t0 = now_us() + 1000.0;
    double last_done = t0;
    int64_t i = 0;
    int err = MDT_SUCCESS;
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
                void *pk = nullptr;
                mdt_server_request_result(srv, pend[k].r, &st, &pk, &nb, &l);
                double t = now_us();
                const mdt_lg_req &q = reqs[pend[k].idx];
                if (st == MDT_SUCCESS) {
                    res->completed++;
                    res->bytes += nb;
                    lat.push_back(t - pend[k].t_arrive);
                    if (lat_out) lat_out[pend[k].idx] = t - pend[k].t_arrive;
                    if (!q.unpack && q.fixed && nb > 0) {
                        // a sampled result leaves the arena before it is released
                        hipError_t e = hipMemcpyAsync(q.fixed, pk, (size_t)nb, hipMemcpyDeviceToDevice, cs);
                        if (e == hipSuccess) e = hipStreamSynchronize(cs);
                        if (e != hipSuccess) err = MDT_ERR_HIP;
                    }
                } else {
                    res->failed++;
                }
                last_done = std::max(last_done, t);
                mdt_server_request_release(srv, &pend[k].r);
                pend[k].r = nullptr;
                ring.free(pend[k].range);
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
            void *dst = q.fixed;
            int64_t range = -1;
            if (q.unpack && !dst && q.span > 0) {
                int64_t off = 0;
                range = ring.alloc(q.span, &off);
                if (range == -2) {
                    err = MDT_ERR_NO_MEM;
                    i = n;
                    break;
                }
                if (range < 0) {
                    const double tw = now_us();
                    res->ring_waits++;
                    while ((range = ring.alloc(q.span, &off)) == -1) reap(false);
                    res->ring_wait_us += now_us() - tw;
                }
                dst = ring.base + off;
            }
            mdt_request r = nullptr;
            int e;
            const double ti = now_us();
            if (q.unpack)
                e = mdt_server_submit_unpack(srv, q.packed, q.target, static_cast<uint8_t *>(dst) + q.origin_off,
                                             q.count, types[q.type_index], 0, &r);
            else
                e = mdt_server_submit_pack(srv, q.typed, q.count, types[q.type_index], 0, q.target, &r);
            issue.push_back(now_us() - ti);
            if (t - (t0 + q.t_arrive_us) > 50.0) res->late_issues++;
            if (e) {
                res->failed++;
                ring.free(range);
            } else {
                pend.push_back({r, t0 + q.t_arrive_us, i, range});
            }
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
    (void)hipStreamDestroy(cs);
    res->elapsed_s = (last_done - t0) * 1e-6;
    summarize(lat, res);
    res->p50_issue_us = pctl(issue, 0.50);
    res->p99_issue_us = pctl(issue, 0.99);
    return err;
}

// One plain launch per request on stream (index mod nstreams); pack outputs
// and unpack spans come from the ring.
__attribute__((visibility("default"))) int mdt_lg_run_plain(const mdt_lg_req *reqs, int64_t n, const mdt_type *types,
                                                            int nstreams, void *ring_base, int64_t ring_bytes,
                                                            mdt_lg_result *res, double *lat_out)
{
    std::memset(res, 0, sizeof *res);
    if (lat_out)
        for (int64_t k = 0; k < n; k++) lat_out[k] = -1.0;
    if (nstreams <= 0 || nstreams > 64) return MDT_ERR_ARG;
    Ring ring;
    ring.base = static_cast<uint8_t *>(ring_base);
    ring.cap = ring_bytes;
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
        int64_t range;
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
    int err = MDT_SUCCESS;
    auto reap = [&] {
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
                ring.free(dq.front().range);
                dq.pop_front();
                npend--;
            }
        }
    };
    while (i < n || npend > 0) {
        double t = now_us();
        while (i < n && t0 + reqs[i].t_arrive_us <= t) {
            const mdt_lg_req &q = reqs[i];
            void *dst = q.fixed;
            int64_t range = -1;
            if (!dst && q.span > 0) {
                int64_t off = 0;
                range = ring.alloc(q.span, &off);
                if (range == -2) {
                    err = MDT_ERR_NO_MEM;
                    i = n;
                    break;
                }
                if (range < 0) {
                    const double tw = now_us();
                    res->ring_waits++;
                    while ((range = ring.alloc(q.span, &off)) == -1) reap();
                    res->ring_wait_us += now_us() - tw;
                }
                dst = ring.base + off;
            }
            mdt_request r = nullptr;
            int64_t got = 0;
            mdt_stream s = ms[(size_t)(i % nstreams)];
            int e;
            const double ti = now_us();
            if (q.unpack)
                e = mdt_unpack_enqueue(q.packed, q.target, static_cast<uint8_t *>(dst) + q.origin_off, q.count,
                                       types[q.type_index], 0, &got, s, &r);
            else
                e = mdt_pack_enqueue(q.typed, q.count, types[q.type_index], 0, dst, q.target, &got, s, &r);
            issue.push_back(now_us() - ti);
            if (t - (t0 + q.t_arrive_us) > 50.0) res->late_issues++;
            if (e) {
                res->failed++;
                ring.free(range);
            } else {
                pend[(size_t)(i % nstreams)].push_back({r, t0 + q.t_arrive_us, got, i, range});
                npend++;
                res->launches++;
            }
            i++;
        }
        reap();
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
    return err;
}

}  // extern "C"
