// requests.cpp -- completing requests: those of enqueued GPU work (a HIP
// event recorded after it) and generalized requests, whose task the caller
// runs and reports (Generalized Requests section).  The section's extension
// gives such a request a poll callback, so the task completes inside the
// library's own test and wait calls with no progress thread of the caller's,
// and a wait callback that blocks on many of the caller's tasks at once
// instead of polling each one.
//
// General progress (General Progress section: a progress call not tied to a
// request, per stream, and a progress thread the caller starts and stops):
// mdt_stream_progress(s) looks at the requests of work enqueued on stream s
// and records those whose work has finished; with no stream it also polls
// every generalized request (its poll_fn), so tasks complete in the
// background.  mdt_start_progress_thread(s) runs such passes on a thread of
// the library until mdt_stop_progress_thread(s): busy while requests are
// incomplete, sleeping in short naps while there are none.
#include <hip/hip_runtime_api.h>

#include <algorithm>
#include <atomic>
#include <chrono>
#include <mutex>
#include <new>
#include <thread>
#include <vector>

#include "requests.h"

namespace mdt {

struct GRequest {
    mdt_grequest_query_fn query_fn;
    mdt_grequest_free_fn free_fn;
    mdt_grequest_cancel_fn cancel_fn;
    mdt_grequest_poll_fn poll_fn;
    mdt_grequest_wait_fn wait_fn;
    void *state;
    std::atomic<int> done{0};
    std::atomic<int> polling{0};  // a thread is inside poll_fn (polls never run concurrently)
};

// ---- progress lists ------------------------------------------------------

void list_add(ReqList *l, mdt_request r)
{
    std::lock_guard<std::mutex> g(l->mu);
    r->list = l;
    r->prev = nullptr;
    r->next = l->head;
    if (l->head) l->head->prev = r;
    l->head = r;
    l->count.fetch_add(1, std::memory_order_relaxed);
}

void list_remove(mdt_request r)
{
    ReqList *l = r->list;
    if (!l) return;
    {
        std::lock_guard<std::mutex> g(l->mu);
        if (r->prev) r->prev->next = r->next;
        else l->head = r->next;
        if (r->next) r->next->prev = r->prev;
        r->prev = r->next = nullptr;
        r->list = nullptr;
        l->count.fetch_sub(1, std::memory_order_relaxed);
    }
    // a progress pass that pinned r before it left the list still uses it
    while (r->pins.load(std::memory_order_acquire) != 0) std::this_thread::yield();
}

namespace {

ReqList g_general;  // generalized requests (reached by general progress)

struct StreamRegistry {
    std::mutex mu;
    std::vector<mdt_stream> all;
} g_streams;

struct GeneralThread {
    std::mutex mu;  // start / stop
    std::atomic<bool> run{false};
    std::thread th;
} g_thread;

// Pin the members of a list (under its lock) so they can be used after it
// is released; unpin when done.
void snapshot(ReqList *l, std::vector<mdt_request> *out)
{
    std::lock_guard<std::mutex> g(l->mu);
    for (mdt_request r = l->head; r; r = r->next) {
        r->pins.fetch_add(1, std::memory_order_acq_rel);
        out->push_back(r);
    }
}

void unpin(const std::vector<mdt_request> &v)
{
    for (mdt_request r : v) r->pins.fetch_sub(1, std::memory_order_acq_rel);
}

}  // namespace

void streams_register(mdt_stream s)
{
    std::lock_guard<std::mutex> g(g_streams.mu);
    g_streams.all.push_back(s);
}

void streams_unregister(mdt_stream s)
{
    std::lock_guard<std::mutex> g(g_streams.mu);
    auto it = std::find(g_streams.all.begin(), g_streams.all.end(), s);
    if (it != g_streams.all.end()) g_streams.all.erase(it);
}

static bool valid_req(mdt_request r) { return r && r->magic == REQUEST_MAGIC; }

static GRequest *general_of(mdt_request r)
{
    return valid_req(r) && r->kind == REQ_GENERAL ? static_cast<GRequest *>(r->general) : nullptr;
}

static bool general_done(const GRequest *g) { return g->done.load(std::memory_order_acquire) != 0; }

// The request has completed: run its query and free callbacks (once), then
// free the handle.  Returns the first nonzero callback value.
static int finish(mdt_request *req)
{
    mdt_request r = *req;
    int rc = MDT_SUCCESS;
    list_remove(r);  // first: a progress pass may still hold it
    if (r->kind == REQ_GENERAL) {
        GRequest *g = static_cast<GRequest *>(r->general);
        int q = g->query_fn ? g->query_fn(g->state) : 0;
        int f = g->free_fn ? g->free_fn(g->state) : 0;
        rc = q ? q : f;
        delete g;
        r->general = nullptr;
    }
    free_request(r);
    *req = MDT_REQUEST_NULL;
    return rc;
}

// Block until an event request's work has finished.
static int sync_event(mdt_request r)
{
    hipError_t e = hipEventSynchronize(r->ev);
    if (e != hipSuccess) {
        set_hip_error((int)e);
        return MDT_ERR_HIP;
    }
    return MDT_SUCCESS;
}

// Call a generalized request's poll_fn unless it is done, has none, or
// another thread is polling it right now.
static int poll_once(GRequest *g)
{
    if (general_done(g) || !g->poll_fn) return MDT_SUCCESS;
    if (g->polling.exchange(1, std::memory_order_acq_rel)) return MDT_SUCCESS;
    int rc = general_done(g) ? MDT_SUCCESS : g->poll_fn(g->state);
    g->polling.store(0, std::memory_order_release);
    return rc;
}

// One progress pass over stream s (NULL: every stream, then the generalized
// requests).  *open counts the requests it found incomplete.
static int progress_pass(mdt_stream s, int64_t *open)
{
    std::vector<mdt_stream> streams;
    if (s) {
        streams.push_back(s);
    } else {
        std::lock_guard<std::mutex> g(g_streams.mu);
        streams = g_streams.all;
    }
    int first = MDT_SUCCESS;
    std::vector<mdt_request> v;
    for (mdt_stream st : streams) {
        if (!s) {
            // a stream freed meanwhile has left the registry before its
            // requests leave its list
            std::lock_guard<std::mutex> g(g_streams.mu);
            if (std::find(g_streams.all.begin(), g_streams.all.end(), st) == g_streams.all.end()) continue;
            if (st->live.count.load(std::memory_order_relaxed) == 0) continue;
            snapshot(&st->live, &v);
        } else {
            snapshot(&st->live, &v);
        }
        for (mdt_request r : v) {
            if (r->done.load(std::memory_order_acquire)) continue;
            hipError_t e = hipEventQuery(r->ev);
            if (e == hipSuccess) {
                r->done.store(1, std::memory_order_release);
            } else {
                ++*open;
                if (e != hipErrorNotReady && !first) {
                    set_hip_error((int)e);
                    first = MDT_ERR_HIP;
                }
            }
        }
        unpin(v);
        v.clear();
    }
    if (!s && g_general.count.load(std::memory_order_relaxed) > 0) {
        snapshot(&g_general, &v);
        for (mdt_request r : v) {
            GRequest *g = static_cast<GRequest *>(r->general);
            int rc = poll_once(g);
            if (rc && !first) first = rc;
            if (!general_done(g)) ++*open;
        }
        unpin(v);
    }
    return first;
}

// The progress thread: passes back to back while requests are incomplete,
// 50 us naps while there are none.
static void progress_loop(std::atomic<bool> *run, mdt_stream s, int device)
{
    if (device >= 0) (void)hipSetDevice(device);
    while (run->load(std::memory_order_acquire)) {
        int64_t open = 0;
        (void)progress_pass(s, &open);
        if (open == 0) std::this_thread::sleep_for(std::chrono::microseconds(50));
        else std::this_thread::yield();
    }
}

// Drive the incomplete generalized requests among reqs[0..n) until all are
// done: one wait_fn call per group that shares a wait_fn, poll_fn for the
// others, and a yield when a round made no progress.  Returns the first
// nonzero callback value (the requests then stay incomplete and valid).
static int drive_general(int n, const mdt_request *reqs)
{
    std::vector<void *> states;
    std::vector<GRequest *> open;
    std::vector<mdt_grequest_wait_fn> seen;
    for (;;) {
        open.clear();
        bool others = false;  // incomplete requests without a wait_fn
        for (int i = 0; i < n; i++) {
            GRequest *g = general_of(reqs[i]);
            if (g && !general_done(g)) {
                open.push_back(g);
                others = others || !g->wait_fn;
            }
        }
        if (open.empty()) return MDT_SUCCESS;
        bool progress = false;
        // wait_fn groups, in order of first appearance; with requests that
        // need polling alongside, each group waits a bounded time
        seen.clear();
        for (GRequest *g : open) {
            if (!g->wait_fn) continue;
            bool dup = false;
            for (auto f : seen) dup = dup || f == g->wait_fn;
            if (dup) continue;
            seen.push_back(g->wait_fn);
            states.clear();
            for (GRequest *h : open)
                if (h->wait_fn == g->wait_fn && !general_done(h)) states.push_back(h->state);
            if (states.empty()) continue;
            int rc = g->wait_fn((int)states.size(), states.data(), others ? 1e-3 : -1.0);
            if (rc) return rc;
            progress = true;
        }
        for (GRequest *g : open) {
            if (g->wait_fn || !g->poll_fn || general_done(g)) continue;
            int rc = poll_once(g);
            if (rc) return rc;
            progress = progress || general_done(g);
        }
        if (!progress) std::this_thread::yield();
    }
}

}  // namespace mdt

using namespace mdt;

extern "C" {

MDT_API int mdt_grequest_start(mdt_grequest_query_fn query_fn, mdt_grequest_free_fn free_fn,
                               mdt_grequest_cancel_fn cancel_fn, mdt_grequest_poll_fn poll_fn,
                               mdt_grequest_wait_fn wait_fn, void *extra_state, mdt_request *req)
{
    if (!req) return MDT_ERR_ARG;
    auto *g = new (std::nothrow) GRequest();
    auto *r = new (std::nothrow) mdt_request_s();
    if (!g || !r) {
        delete g;
        delete r;
        return MDT_ERR_NO_MEM;
    }
    g->query_fn = query_fn;
    g->free_fn = free_fn;
    g->cancel_fn = cancel_fn;
    g->poll_fn = poll_fn;
    g->wait_fn = wait_fn;
    g->state = extra_state;
    r->kind = REQ_GENERAL;
    r->general = g;
    list_add(&g_general, r);  // reachable by general progress
    *req = r;
    return MDT_SUCCESS;
}

MDT_API int mdt_grequest_complete(mdt_request req)
{
    GRequest *g = general_of(req);
    if (!g) return MDT_ERR_ARG;
    // the store is this call's last access: a waiter may free the request
    // as soon as it sees it
    return g->done.exchange(1, std::memory_order_acq_rel) ? MDT_ERR_STATE : MDT_SUCCESS;
}

MDT_API int mdt_cancel(mdt_request req)
{
    GRequest *g = general_of(req);
    if (!g) return MDT_ERR_ARG;
    return g->cancel_fn ? g->cancel_fn(g->state, general_done(g) ? 1 : 0) : MDT_SUCCESS;
}

MDT_API int mdt_wait(mdt_request *req)
{
    if (!req) return MDT_ERR_ARG;
    if (*req == MDT_REQUEST_NULL) return MDT_SUCCESS;
    mdt_request r = *req;
    if (!valid_req(r) || r->kind == REQ_SERVER) return MDT_ERR_ARG;
    int rc = r->kind == REQ_EVENT ? sync_event(r) : drive_general(1, &r);
    if (rc) return rc;
    return finish(req);
}

MDT_API int mdt_test(mdt_request *req, int *flag)
{
    if (!req || !flag) return MDT_ERR_ARG;
    if (*req == MDT_REQUEST_NULL) {
        *flag = 1;
        return MDT_SUCCESS;
    }
    mdt_request r = *req;
    if (!valid_req(r) || r->kind == REQ_SERVER) return MDT_ERR_ARG;
    bool done;
    if (r->kind == REQ_EVENT) {
        done = r->done.load(std::memory_order_acquire) != 0;  // seen by a progress pass
        if (!done) {
            hipError_t e = hipEventQuery(r->ev);
            if (e != hipSuccess && e != hipErrorNotReady) {
                set_hip_error((int)e);
                return MDT_ERR_HIP;
            }
            done = e == hipSuccess;
        }
    } else {
        GRequest *g = static_cast<GRequest *>(r->general);
        int rc = poll_once(g);
        if (rc) return rc;
        done = general_done(g);
    }
    if (!done) {
        *flag = 0;
        return MDT_SUCCESS;
    }
    *flag = 1;
    return finish(req);
}

MDT_API int mdt_waitall(int n, mdt_request reqs[])
{
    if (n < 0 || (n > 0 && !reqs)) return MDT_ERR_ARG;
    for (int i = 0; i < n; i++)
        if (reqs[i] != MDT_REQUEST_NULL && (!valid_req(reqs[i]) || reqs[i]->kind == REQ_SERVER)) return MDT_ERR_ARG;
    // the caller's tasks first (GPU work completes on its own meanwhile),
    // then the GPU requests, then every request is freed in order
    int rc = drive_general(n, reqs);
    if (rc) return rc;
    for (int i = 0; i < n; i++) {
        if (reqs[i] == MDT_REQUEST_NULL || reqs[i]->kind != REQ_EVENT) continue;
        rc = sync_event(reqs[i]);
        if (rc) return rc;
    }
    int first = MDT_SUCCESS;
    for (int i = 0; i < n; i++) {
        if (reqs[i] == MDT_REQUEST_NULL) continue;
        int f = finish(&reqs[i]);
        if (f && !first) first = f;
    }
    return first;
}

MDT_API int mdt_stream_progress(mdt_stream s)
{
    if (s && s->magic != STREAM_MAGIC) return MDT_ERR_ARG;
    int64_t open = 0;
    return progress_pass(s, &open);
}

MDT_API int mdt_start_progress_thread(mdt_stream s)
{
    if (s && s->magic != STREAM_MAGIC) return MDT_ERR_ARG;
    int dev = -1;
    (void)hipGetDevice(&dev);
    std::lock_guard<std::mutex> g(g_thread.mu);
    std::atomic<bool> *run = s ? &s->run : &g_thread.run;
    std::thread *th = s ? &s->th : &g_thread.th;
    if (run->exchange(true)) return MDT_SUCCESS;  // already running
    try {
        *th = std::thread(progress_loop, run, s, dev);
    } catch (...) {
        run->store(false);
        return MDT_ERR_NO_MEM;
    }
    return MDT_SUCCESS;
}

MDT_API int mdt_stop_progress_thread(mdt_stream s)
{
    if (s && s->magic != STREAM_MAGIC) return MDT_ERR_ARG;
    std::lock_guard<std::mutex> g(g_thread.mu);
    std::atomic<bool> *run = s ? &s->run : &g_thread.run;
    std::thread *th = s ? &s->th : &g_thread.th;
    if (!run->exchange(false)) return MDT_SUCCESS;
    if (th->joinable()) th->join();
    return MDT_SUCCESS;
}

MDT_API int mdt_request_get_status(mdt_request req, int *flag)
{
    if (!flag) return MDT_ERR_ARG;
    if (req == MDT_REQUEST_NULL) {
        *flag = 1;
        return MDT_SUCCESS;
    }
    if (!valid_req(req) || req->kind == REQ_SERVER) return MDT_ERR_ARG;
    *flag = req->kind == REQ_EVENT ? req->done.load(std::memory_order_acquire) != 0
                                   : general_done(static_cast<GRequest *>(req->general));
    return MDT_SUCCESS;
}

}  // extern "C"
