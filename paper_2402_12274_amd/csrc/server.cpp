// server.cpp -- continuous-batching progress engine for pack/unpack requests.
//
// Clients submit requests from any thread (a short locked queue); a progress
// round (MPIX_Stream_progress in the General Progress section; run by the
// caller or by a progress thread, MPIX_Start_progress_thread) does three
// things:
//   1. reap: query the completion event of every launch in flight and
//      complete its requests (the poll-callback pattern of generalized
//      requests: query the event, complete the request), stamping latency;
//   2. admit: move queued requests into the admitted set while the bytes
//      they hold (packed buffer, plus the destination span for unpack) fit
//      in the memory budget -- requests that do not fit wait, they do not
//      fail; pack outputs come from a device arena allocated once, so the
//      loop never calls hipMalloc;
//   3. launch: while some stream has a free launch slot, cut up to max_batch
//      admitted requests into one batched persistent launch on the least
//      loaded stream and record its completion event.
// Requests arriving while others run are admitted as soon as slots and
// memory free up, so their work overlaps on the device.  Each request's bytes
// are those of the same request run alone (the batch runs the single-request
// chunk bodies).
#include <hip/hip_runtime_api.h>

#include <algorithm>
#include <atomic>
#include <cstdlib>
#include <chrono>
#include <condition_variable>
#include <deque>
#include <map>
#include <mutex>
#include <new>
#include <thread>
#include <vector>

#include "core.h"
#include "device.h"
#include "requests.h"

namespace mdt {
int batch_launch_internal(mdt_batch b, hipStream_t s);
int pack_common(const void *inbuf, int64_t incount, mdt_type t, int64_t inoffset, void *outbuf, int64_t max_bytes,
                int64_t *actual, hipStream_t s, mdt_request *req);
int unpack_common(const void *inbuf, int64_t insize, void *outbuf, int64_t outcount, mdt_type t, int64_t outoffset,
                  int64_t *actual, hipStream_t s, mdt_request *req);
}

using namespace mdt;

namespace {

constexpr uint32_t SERVER_MAGIC = 0x6d647356u;
constexpr int64_t ARENA_ALIGN = 256;
// A launch stops taking requests once it holds this many bytes, so small
// requests are not held back by a large one in the same launch (a large
// request still goes alone).
const int64_t BATCH_BYTES = [] {
    const char *e = getenv("MDT_SERVER_BATCH_BYTES");
    long long v = e && *e ? atoll(e) : (8ll << 20);
    return (int64_t)(v > 0 ? v : (8ll << 20));
}();
// The progress thread keeps polling for this long after the last activity
// before it sleeps (a sleeping thread wakes with scheduler latency).
constexpr double SPIN_US = 2000.0;

double now_us()
{
    using namespace std::chrono;
    return (double)duration_cast<nanoseconds>(steady_clock::now().time_since_epoch()).count() * 1e-3;
}

struct Item {
    int unpack = 0;
    TypeNode *type = nullptr;  // retained
    const void *in = nullptr;
    void *out = nullptr;
    int64_t count = 0, off = 0, nbytes = 0;
    int64_t charge = 0;
    int64_t arena_off = -1;
    void *packed = nullptr;
    int status = MDT_SUCCESS;
    double t_submit = 0, t_launch = 0, t_done = 0;
    std::atomic<int> state{0};  // 0 queued, 1 admitted, 2 launched, 3 done
    bool deferred = false;
};

// first-fit allocator over one device allocation
struct Arena {
    uint8_t *base = nullptr;
    int64_t size = 0;
    std::map<int64_t, int64_t> free_;  // offset -> length
    int64_t alloc(int64_t n)
    {
        n = (n + ARENA_ALIGN - 1) / ARENA_ALIGN * ARENA_ALIGN;
        if (n == 0) n = ARENA_ALIGN;
        for (auto it = free_.begin(); it != free_.end(); ++it) {
            if (it->second >= n) {
                int64_t off = it->first, len = it->second;
                free_.erase(it);
                if (len > n) free_[off + n] = len - n;
                return off;
            }
        }
        return -1;
    }
    void release(int64_t off, int64_t n)
    {
        n = (n + ARENA_ALIGN - 1) / ARENA_ALIGN * ARENA_ALIGN;
        if (n == 0) n = ARENA_ALIGN;
        auto it = free_.emplace(off, n).first;
        auto nx = std::next(it);
        if (nx != free_.end() && it->first + it->second == nx->first) {
            it->second += nx->second;
            free_.erase(nx);
        }
        if (it != free_.begin()) {
            auto pv = std::prev(it);
            if (pv->first + pv->second == it->first) {
                pv->second += it->second;
                free_.erase(it);
            }
        }
    }
};

struct Slot {
    mdt_batch batch = nullptr;
    hipEvent_t ev = nullptr;
    std::vector<Item *> items;
    bool busy = false;
    uint64_t seq = 0;  // launch order on its stream
};

struct StreamState {
    hipStream_t s = nullptr;
    std::vector<Slot> slots;
    int busy = 0;
    uint64_t next_seq = 0;
};

}  // namespace

struct mdt_server_s {
    uint32_t magic = SERVER_MAGIC;
    mdt_server_config cfg{};
    int device = -1;
    std::vector<StreamState> streams;
    Arena arena;
    std::mutex qmu;              // submit queue
    std::deque<Item *> queue;
    std::mutex mu;               // everything below; held by a progress round
    std::deque<Item *> admitted;
    int64_t inflight = 0, peak_inflight = 0;
    int inject_fail = 0;
    std::atomic<bool> run_thread{false};
    bool draining = false;       // shutdown: admit regardless of the budget
    std::atomic<bool> light{true};  // few launches in flight: submitters may dispatch
    std::condition_variable wake;  // submit -> idle progress thread
    std::thread th;
    // stats
    int64_t submitted = 0, completed = 0, failed = 0, deferred = 0, bytes = 0, launches = 0;
    double first_submit = -1, last_done = 0;
    std::vector<float> lat_us, queue_us, run_us;
};

namespace {

bool valid_server(mdt_server s) { return s && s->magic == SERVER_MAGIC; }

void complete(mdt_server s, Item *it, int status, double t)
{
    it->status = status;
    it->t_done = t;
    if (status == MDT_SUCCESS) {
        s->completed++;
        s->bytes += it->nbytes;
        s->lat_us.push_back((float)(t - it->t_submit));
        if (it->t_launch > 0) {
            s->queue_us.push_back((float)(it->t_launch - it->t_submit));
            s->run_us.push_back((float)(t - it->t_launch));
        }
    } else {
        s->failed++;
    }
    s->last_done = std::max(s->last_done, t);
    it->state.store(3, std::memory_order_release);
}

// one progress round; caller holds s->mu
int progress_locked(mdt_server s)
{
    int rc = MDT_SUCCESS;
    // 1. reap completed launches; a stream finishes its launches in order, so
    // only its oldest running launch is queried
    for (auto &st : s->streams) {
        for (;;) {
            Slot *old = nullptr;
            for (auto &x : st.slots)
                if (x.busy && (!old || x.seq < old->seq)) old = &x;
            if (!old) break;
            Slot &sl = *old;
            hipError_t e = hipEventQuery(sl.ev);
            if (e == hipErrorNotReady) break;
            double t = now_us();
            int status = e == hipSuccess ? MDT_SUCCESS : MDT_ERR_HIP;
            if (e != hipSuccess) set_hip_error((int)e);
            for (Item *it : sl.items) complete(s, it, status, t);
            sl.items.clear();
            sl.busy = false;
            st.busy--;
        }
    }
    // 2. admit queued requests within the budget
    {
        std::lock_guard<std::mutex> q(s->qmu);
        while (!s->queue.empty()) {
            Item *it = s->queue.front();
            if (!s->draining && s->inflight + it->charge > s->cfg.budget_bytes && s->inflight > 0) {
                if (!it->deferred) {
                    it->deferred = true;
                    s->deferred++;
                }
                break;
            }
            if (!it->unpack) {
                if (s->inject_fail > 0) {
                    s->inject_fail--;
                    s->queue.pop_front();
                    complete(s, it, MDT_ERR_NO_MEM, now_us());
                    continue;
                }
                int64_t off = s->arena.alloc(std::max<int64_t>(it->nbytes, 1));
                if (off < 0) {
                    bool busy = false;
                    for (auto &st : s->streams) busy = busy || st.busy > 0;
                    if (s->inflight == 0 || (s->draining && !busy && s->admitted.empty())) {  // cannot fit
                        s->queue.pop_front();
                        complete(s, it, MDT_ERR_NO_MEM, now_us());
                        continue;
                    }
                    if (!it->deferred) {
                        it->deferred = true;
                        s->deferred++;
                    }
                    break;
                }
                it->arena_off = off;
                it->packed = s->arena.base + off;
                it->out = it->packed;
            }
            s->queue.pop_front();
            s->inflight += it->charge;
            s->peak_inflight = std::max(s->peak_inflight, s->inflight);
            it->state.store(1, std::memory_order_release);
            s->admitted.push_back(it);
        }
    }
    // 3. launch batches on free slots, least-loaded stream first
    while (!s->admitted.empty()) {
        StreamState *best = nullptr;
        for (auto &st : s->streams)
            if (st.busy < (int)st.slots.size() && (!best || st.busy < best->busy)) best = &st;
        if (!best) break;
        Slot *sl = nullptr;
        for (auto &x : best->slots)
            if (!x.busy) {
                sl = &x;
                break;
            }
        // a lone request is launched with the single-request kernels (no
        // descriptor upload); several go through one batched launch
        size_t take_n = 0;
        {
            int64_t b = 0;
            for (Item *it : s->admitted) {
                if (take_n >= (size_t)s->cfg.max_batch || (take_n > 0 && b + it->nbytes > BATCH_BYTES)) break;
                b += it->nbytes;
                take_n++;
            }
        }
        if (take_n == 1) {
            Item *it = s->admitted.front();
            s->admitted.pop_front();
            int64_t got = 0;
            mdt_type th = reinterpret_cast<mdt_type>(it->type);
            int r = it->unpack ? unpack_common(it->in, it->nbytes, it->out, it->count, th, it->off, &got, best->s, nullptr)
                               : pack_common(it->in, it->count, th, it->off, it->out, it->nbytes, &got, best->s, nullptr);
            hipError_t e = r == MDT_SUCCESS ? hipEventRecord(sl->ev, best->s) : hipErrorUnknown;
            if (r != MDT_SUCCESS || e != hipSuccess) {
                complete(s, it, r ? r : MDT_ERR_HIP, now_us());
                rc = r ? r : MDT_ERR_HIP;
                continue;
            }
            it->state.store(2, std::memory_order_release);
            it->t_launch = now_us();
            sl->items.push_back(it);
            sl->busy = true;
            sl->seq = best->next_seq++;
            best->busy++;
            s->launches++;
            continue;
        }
        mdt_batch_clear(sl->batch);
        int n = 0;
        int64_t bytes = 0;
        while (!s->admitted.empty() && n < s->cfg.max_batch) {
            Item *it = s->admitted.front();
            if (n > 0 && bytes + it->nbytes > BATCH_BYTES) break;
            bytes += it->nbytes;
            s->admitted.pop_front();
            int64_t got = 0;
            int r;
            mdt_type th = reinterpret_cast<mdt_type>(it->type);
            if (it->unpack)
                r = mdt_batch_add_unpack(sl->batch, it->in, it->nbytes, it->out, it->count, th, it->off, &got);
            else
                r = mdt_batch_add_pack(sl->batch, it->in, it->count, th, it->off, it->out, it->nbytes, &got);
            if (r != MDT_SUCCESS) {
                complete(s, it, r, now_us());
                continue;
            }
            it->state.store(2, std::memory_order_release);
            sl->items.push_back(it);
            n++;
        }
        if (sl->items.empty()) continue;
        int r = batch_launch_internal(sl->batch, best->s);
        {
            double tl = now_us();
            for (Item *it : sl->items) it->t_launch = tl;
        }
        hipError_t e = r == MDT_SUCCESS ? hipEventRecord(sl->ev, best->s) : hipErrorUnknown;
        if (r != MDT_SUCCESS || e != hipSuccess) {
            for (Item *it : sl->items) complete(s, it, r ? r : MDT_ERR_HIP, now_us());
            sl->items.clear();
            rc = r ? r : MDT_ERR_HIP;
            continue;
        }
        sl->busy = true;
        sl->seq = best->next_seq++;
        best->busy++;
        s->launches++;
    }
    int inflight = 0;
    for (auto &st : s->streams) inflight += st.busy;
    s->light.store(inflight < (int)s->streams.size() && s->admitted.empty(), std::memory_order_relaxed);
    return rc;
}

int progress(mdt_server s)
{
    std::lock_guard<std::mutex> g(s->mu);
    return progress_locked(s);
}

// The progress thread polls continuously while anything is queued,
// admitted or in flight, and sleeps on a condition variable (woken by
// submit) when the server is idle.
void thread_main(mdt_server s)
{
    (void)hipSetDevice(s->device);
    double last_active = now_us();
    while (s->run_thread.load(std::memory_order_acquire)) {
        bool idle;
        {
            std::lock_guard<std::mutex> g(s->mu);
            progress_locked(s);
            bool busy = !s->admitted.empty();
            for (auto &st : s->streams) busy = busy || st.busy > 0;
            std::lock_guard<std::mutex> q(s->qmu);
            idle = !busy && s->queue.empty();
        }
        double t = now_us();
        if (!idle) last_active = t;
        if (!idle || t - last_active < SPIN_US) {
            std::this_thread::yield();
            continue;
        }
        {
            std::unique_lock<std::mutex> q(s->qmu);
            s->wake.wait_for(q, std::chrono::milliseconds(1),
                             [s] { return !s->queue.empty() || !s->run_thread.load(std::memory_order_acquire); });
        }
    }
}

bool idle_all(mdt_server s)
{
    std::lock_guard<std::mutex> g(s->mu);
    std::lock_guard<std::mutex> q(s->qmu);
    if (!s->queue.empty() || !s->admitted.empty()) return false;
    for (auto &st : s->streams)
        if (st.busy) return false;
    return true;
}

int submit(mdt_server s, Item *it, mdt_request *req)
{
    auto *r = new (std::nothrow) mdt_request_s();
    if (!r) {
        release(it->type);
        delete it;
        return MDT_ERR_NO_MEM;
    }
    r->kind = REQ_SERVER;
    r->server_item = it;
    it->t_submit = now_us();
    {
        std::lock_guard<std::mutex> g(s->mu);
        s->submitted++;
        if (s->first_submit < 0) s->first_submit = it->t_submit;
    }
    {
        std::lock_guard<std::mutex> q(s->qmu);
        s->queue.push_back(it);
    }
    s->wake.notify_one();
    // light load: dispatch right away when no progress round is running and
    // nothing else waits; under load the progress thread batches instead
    if (s->light.load(std::memory_order_relaxed) && s->mu.try_lock()) {
        progress_locked(s);
        s->mu.unlock();
    }
    *req = r;
    return MDT_SUCCESS;
}

Item *item_of(mdt_request r)
{
    if (!r || r->magic != REQUEST_MAGIC || r->kind != REQ_SERVER) return nullptr;
    return static_cast<Item *>(r->server_item);
}

}  // namespace

extern "C" {

MDT_API int mdt_server_create(const mdt_server_config *cfg, mdt_server *out)
{
    if (!out) return MDT_ERR_ARG;
    mdt_server_config c{8, (int64_t)32 << 30, 256, 2, 0};
    if (cfg) {
        c = *cfg;
        if (c.nstreams <= 0) c.nstreams = 8;
        if (c.budget_bytes <= 0) c.budget_bytes = (int64_t)32 << 30;
        if (c.max_batch <= 0) c.max_batch = 256;
        if (c.max_inflight <= 0) c.max_inflight = 2;
    }
    if (c.arena_bytes <= 0) c.arena_bytes = c.budget_bytes;
    if (c.nstreams > 64 || c.max_inflight > 16) return MDT_ERR_ARG;
    auto *s = new (std::nothrow) mdt_server_s();
    if (!s) return MDT_ERR_NO_MEM;
    s->cfg = c;
    if (hipGetDevice(&s->device) != hipSuccess) {
        delete s;
        return MDT_ERR_HIP;
    }
    hipError_t e = hipMalloc((void **)&s->arena.base, (size_t)c.arena_bytes);
    if (e != hipSuccess) {
        set_hip_error((int)e);
        delete s;
        return MDT_ERR_NO_MEM;
    }
    s->arena.size = c.arena_bytes;
    s->arena.free_[0] = c.arena_bytes;
    s->streams.resize(c.nstreams);
    int rc = MDT_SUCCESS;
    for (auto &st : s->streams) {
        if (hipStreamCreateWithFlags(&st.s, hipStreamNonBlocking) != hipSuccess) rc = MDT_ERR_HIP;
        st.slots.resize(c.max_inflight);
        for (auto &sl : st.slots) {
            if (mdt_batch_create(&sl.batch) != MDT_SUCCESS) rc = MDT_ERR_NO_MEM;
            mdt_batch_config bc{1024, 4, 0, 0};
            if (sl.batch) mdt_batch_set_config(sl.batch, &bc);
            if (hipEventCreateWithFlags(&sl.ev, hipEventDisableTiming) != hipSuccess) rc = MDT_ERR_HIP;
        }
    }
    *out = s;
    if (rc) {
        mdt_server_free(out);
        return rc;
    }
    return MDT_SUCCESS;
}

MDT_API int mdt_server_free(mdt_server *ps)
{
    if (!ps || !valid_server(*ps)) return MDT_ERR_ARG;
    mdt_server s = *ps;
    // drain: everything admitted or queued completes before the server goes
    mdt_server_stop_progress_thread(s);
    {
        std::lock_guard<std::mutex> g(s->mu);
        s->draining = true;
    }
    while (!idle_all(s)) {
        progress(s);
        std::this_thread::sleep_for(std::chrono::microseconds(20));
    }
    (void)hipDeviceSynchronize();
    for (auto &st : s->streams) {
        for (auto &sl : st.slots) {
            if (sl.batch) mdt_batch_free(&sl.batch);
            if (sl.ev) (void)hipEventDestroy(sl.ev);
        }
        if (st.s) (void)hipStreamDestroy(st.s);
    }
    if (s->arena.base) (void)hipFree(s->arena.base);
    s->magic = 0;
    delete s;
    *ps = nullptr;
    return MDT_SUCCESS;
}

MDT_API int mdt_server_submit_pack(mdt_server srv, const void *inbuf, mdt_count incount, mdt_type t,
                                   mdt_count inoffset, mdt_count max_pack_bytes, mdt_request *req)
{
    if (!valid_server(srv) || !req || inoffset < 0 || max_pack_bytes < -1) return MDT_ERR_ARG;
    Compiled *C;
    int64_t total;
    int rc = prepare(t, incount, &C, nullptr, &total);
    if (rc) return rc;
    int64_t n = std::max<int64_t>(0, total - inoffset);
    if (max_pack_bytes >= 0) n = std::min<int64_t>(n, max_pack_bytes);
    if (n > 0 && !inbuf) return MDT_ERR_ARG;
    if (n > srv->arena.size) return MDT_ERR_NO_MEM;
    auto *it = new (std::nothrow) Item();
    if (!it) return MDT_ERR_NO_MEM;
    it->unpack = 0;
    it->type = reinterpret_cast<TypeNode *>(t);
    retain(it->type);
    it->in = inbuf;
    it->count = incount;
    it->off = inoffset;
    it->nbytes = n;
    it->charge = n;
    return submit(srv, it, req);
}

MDT_API int mdt_server_submit_unpack(mdt_server srv, const void *inbuf, mdt_count insize, void *outbuf,
                                     mdt_count outcount, mdt_type t, mdt_count outoffset, mdt_request *req)
{
    if (!valid_server(srv) || !req || insize < 0 || outoffset < 0) return MDT_ERR_ARG;
    Compiled *C;
    int64_t total;
    int rc = prepare(t, outcount, &C, nullptr, &total);
    if (rc) return rc;
    if (insize > std::max<int64_t>(0, total - outoffset)) return MDT_ERR_TRUNCATE;
    rc = check_unpack_overlap(C, outcount);
    if (rc) return rc;
    if (insize > 0 && (!inbuf || !outbuf)) return MDT_ERR_ARG;
    TypeNode *tn = reinterpret_cast<TypeNode *>(t);
    auto *it = new (std::nothrow) Item();
    if (!it) return MDT_ERR_NO_MEM;
    it->unpack = 1;
    it->type = tn;
    retain(tn);
    it->in = inbuf;
    it->out = outbuf;
    it->count = outcount;
    it->off = outoffset;
    it->nbytes = insize;
    // held bytes: the packed input plus the destination span it writes into
    int64_t span = outcount > 0 ? (outcount - 1) * std::llabs(tn->extent()) + (tn->tub - tn->tlb) : 0;
    it->charge = insize + span;
    return submit(srv, it, req);
}

MDT_API int mdt_server_request_test(mdt_server srv, mdt_request req, int *flag)
{
    Item *it = item_of(req);
    if (!valid_server(srv) || !it || !flag) return MDT_ERR_ARG;
    if (it->state.load(std::memory_order_acquire) != 3 && !srv->run_thread.load()) progress(srv);
    *flag = it->state.load(std::memory_order_acquire) == 3;
    return MDT_SUCCESS;
}

MDT_API int mdt_server_request_wait(mdt_server srv, mdt_request req)
{
    Item *it = item_of(req);
    if (!valid_server(srv) || !it) return MDT_ERR_ARG;
    while (it->state.load(std::memory_order_acquire) != 3) {
        if (!srv->run_thread.load()) progress(srv);
        else std::this_thread::sleep_for(std::chrono::microseconds(10));
    }
    return MDT_SUCCESS;
}

MDT_API int mdt_server_request_result(mdt_server srv, mdt_request req, int *status, void **packed,
                                      mdt_count *nbytes, double *latency_us)
{
    Item *it = item_of(req);
    if (!valid_server(srv) || !it) return MDT_ERR_ARG;
    if (it->state.load(std::memory_order_acquire) != 3) return MDT_ERR_STATE;
    if (status) *status = it->status;
    if (packed) *packed = it->unpack ? nullptr : it->packed;
    if (nbytes) *nbytes = it->nbytes;
    if (latency_us) *latency_us = it->t_done - it->t_submit;
    return MDT_SUCCESS;
}

MDT_API int mdt_server_request_release(mdt_server srv, mdt_request *preq)
{
    if (!preq) return MDT_ERR_ARG;
    Item *it = item_of(*preq);
    if (!valid_server(srv) || !it) return MDT_ERR_ARG;
    if (it->state.load(std::memory_order_acquire) != 3) return MDT_ERR_STATE;
    {
        std::lock_guard<std::mutex> g(srv->mu);
        if (it->arena_off >= 0) srv->arena.release(it->arena_off, std::max<int64_t>(it->nbytes, 1));
        // admitted requests hold their charge until released
        if (it->arena_off >= 0 || it->unpack) srv->inflight -= it->charge;
    }
    release(it->type);
    delete it;
    (*preq)->magic = 0;
    delete *preq;
    *preq = nullptr;
    return MDT_SUCCESS;
}

MDT_API int mdt_server_progress(mdt_server srv)
{
    if (!valid_server(srv)) return MDT_ERR_ARG;
    return progress(srv);
}

MDT_API int mdt_server_start_progress_thread(mdt_server srv)
{
    if (!valid_server(srv)) return MDT_ERR_ARG;
    if (srv->run_thread.exchange(true)) return MDT_SUCCESS;
    try {
        srv->th = std::thread(thread_main, srv);
    } catch (...) {
        srv->run_thread.store(false);
        return MDT_ERR_NO_MEM;
    }
    return MDT_SUCCESS;
}

MDT_API int mdt_server_stop_progress_thread(mdt_server srv)
{
    if (!valid_server(srv)) return MDT_ERR_ARG;
    if (!srv->run_thread.exchange(false)) return MDT_SUCCESS;
    srv->wake.notify_all();
    if (srv->th.joinable()) srv->th.join();
    return MDT_SUCCESS;
}

MDT_API int mdt_server_stats_get(mdt_server srv, mdt_server_stats *out)
{
    if (!valid_server(srv) || !out) return MDT_ERR_ARG;
    std::lock_guard<std::mutex> g(srv->mu);
    out->submitted = srv->submitted;
    out->completed = srv->completed;
    out->failed = srv->failed;
    out->deferred = srv->deferred;
    out->bytes = srv->bytes;
    out->launches = srv->launches;
    out->inflight_bytes = srv->inflight;
    out->peak_inflight_bytes = srv->peak_inflight;
    out->elapsed_s = srv->first_submit >= 0 ? (srv->last_done - srv->first_submit) * 1e-6 : 0.0;
    out->p50_us = out->p99_us = out->max_us = 0;
    auto pct = [](std::vector<float> v, double f) {
        if (v.empty()) return 0.0;
        size_t n = v.size();
        size_t k = std::min(n - 1, (size_t)(f * (double)(n - 1) + 0.5));
        std::nth_element(v.begin(), v.begin() + k, v.end());
        return (double)v[k];
    };
    if (!srv->lat_us.empty()) {
        out->p50_us = pct(srv->lat_us, 0.50);
        out->p99_us = pct(srv->lat_us, 0.99);
        out->max_us = *std::max_element(srv->lat_us.begin(), srv->lat_us.end());
    }
    out->p50_queue_us = pct(srv->queue_us, 0.50);
    out->p99_queue_us = pct(srv->queue_us, 0.99);
    out->p50_run_us = pct(srv->run_us, 0.50);
    out->p99_run_us = pct(srv->run_us, 0.99);
    return MDT_SUCCESS;
}

MDT_API int mdt_server_inject_alloc_failures(mdt_server srv, int n)
{
    if (!valid_server(srv) || n < 0) return MDT_ERR_ARG;
    std::lock_guard<std::mutex> g(srv->mu);
    srv->inject_fail = n;
    return MDT_SUCCESS;
}

}  // extern "C"
