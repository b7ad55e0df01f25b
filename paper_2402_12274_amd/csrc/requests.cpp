// requests.cpp -- completing requests: those of enqueued GPU work (a HIP
// event recorded after it) and generalized requests, whose task the caller
// runs and reports (Generalized Requests section).  The section's extension
// gives such a request a poll callback, so the task completes inside the
// library's own test and wait calls with no progress thread of the caller's,
// and a wait callback that blocks on many of the caller's tasks at once
// instead of polling each one.
#include <hip/hip_runtime_api.h>

#include <atomic>
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
};

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
            int rc = g->poll_fn(g->state);
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
        hipError_t e = hipEventQuery(r->ev);
        if (e != hipSuccess && e != hipErrorNotReady) {
            set_hip_error((int)e);
            return MDT_ERR_HIP;
        }
        done = e == hipSuccess;
    } else {
        GRequest *g = static_cast<GRequest *>(r->general);
        if (!general_done(g) && g->poll_fn) {
            int rc = g->poll_fn(g->state);
            if (rc) return rc;
        }
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

}  // extern "C"
