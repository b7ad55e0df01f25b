// server.cpp -- continuous-batching progress engine for pack/unpack requests.
//
// Clients submit requests from any thread; every submit, and a progress
// thread while work is outstanding (MPIX_Stream_progress and
// MPIX_Start_progress_thread in the General Progress section), run progress
// rounds.  A round does three things:
//   0. take back what released requests held (arena range, budget charge);
//   1. reap: query the completion event of the oldest launch of each stream
//      (a stream finishes in order) and complete its requests (the
//      poll-callback pattern of generalized requests), stamping latency;
//   2. admit: move queued requests into the admitted set while the bytes
//      they hold (packed buffer, plus the destination span for unpack) fit
//      in the memory budget -- requests that do not fit wait, they do not
//      fail; pack outputs come from a device arena allocated once, so the
//      loop never calls hipMalloc;
//   3. launch: while some stream has a free launch slot, cut admitted
//      requests (up to max_batch, and up to a byte cap so small requests are
//      not held behind a large one) into one launch on the stream with the
//      least work in flight: a lone request with the single-request kernels,
//      several as one batched launch; record its completion event.
// A submit that finds nothing waiting and a launch slot free admits and
// launches its own request directly (one lock, the single-request kernels,
// as a plain enqueue); otherwise it queues, and the progress thread cuts
// whatever has queued into batched launches.  Requests that arrive while
// others run are admitted as soon as slots and memory free up, and their
// work overlaps on the device.  Clients testing their requests query their
// own launch's event; the progress thread then stays out of the HIP runtime
// except to launch queued work.  Each request's bytes are those of the same
// request run alone (the batch runs the single-request tile bodies).
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
#include "trace.h"

namespace mdt {
int batch_launch_internal(mdt_batch b, hipStream_t s);
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
// Requests at least this large (packed bytes) are launched on their own
// hardware queue, in order (MDT_SERVER_LARGE_BYTES).
const int64_t LARGE_BYTES = [] {
    const char *e = getenv("MDT_SERVER_LARGE_BYTES");
    long long v = e && *e ? atoll(e) : (4ll << 20);
    return (int64_t)(v > 0 ? v : (4ll << 20));
}();
// Hardware queues a process's streams are spread over (the runtime's
// GPU_MAX_HW_QUEUES, 4 unless set).
const int HW_QUEUES = [] {
    const char *e = getenv("GPU_MAX_HW_QUEUES");
    int v = e && *e ? atoi(e) : 4;
    return v >= 1 && v <= 64 ? v : 4;
}();
// The progress thread keeps polling for this long after the last activity
// before it sleeps (a sleeping thread wakes with scheduler latency).
constexpr double SPIN_US = 2000.0;
// Completion queries: a client's test reaps at most this often; the
// progress thread, which does not wait on requests itself, reaps launches
// that only need completing at a slower cadence (so it rarely contends with
// clients for the runtime).
constexpr double TEST_REAP_US = 1.0;
const double THREAD_REAP_US = [] {
    const char *e = getenv("MDT_SERVER_THREAD_REAP_US");
    double v = e && *e ? atof(e) : 20.0;
    return v > 0 ? v : 20.0;
}();
// While clients test their own requests (each test queries its launch's
// event, as a plain enqueue's caller would), the progress thread leaves
// completion to them and stays out of the HIP runtime: it reaps only when
// no client has tested for this long.
const double CLIENT_QUIET_US = [] {
    const char *e = getenv("MDT_SERVER_CLIENT_QUIET_US");
    double v = e && *e ? atof(e) : 200.0;
    return v >= 0 ? v : 200.0;
}();
// A submit that finds nothing queued and a launch slot free launches its
// request itself, with no queue round trip (MDT_SERVER_DIRECT=0 turns the
// direct path off: every request then goes through a progress round).
const bool DIRECT = [] {
    const char *e = getenv("MDT_SERVER_DIRECT");
    return !(e && *e == '0');
}();
// While launches are in flight and nothing waits to be launched, the
// progress thread polls its counters at this interval rather than back to
// back: every poll reads cache lines the submitting and testing clients
// write, and a tight loop makes each of their writes a coherence miss.
const double POLL_US = [] {
    const char *e = getenv("MDT_SERVER_POLL_US");
    double v = e && *e ? atof(e) : 2.0;
    return v >= 0 && v <= 1000 ? v : 2.0;
}();
// A client's test records its time (for the progress thread's quiet test)
// only when the recorded time is at least this old, so a client polling its
// requests does not write that line on every poll.
constexpr double CLIENT_MARK_US = 10.0;

double now_us()
{
    using namespace std::chrono;
    return (double)duration_cast<nanoseconds>(steady_clock::now().time_since_epoch()).count() * 1e-3;
}

// one spin-wait hint (the x86 PAUSE instruction)
inline void cpu_relax() { __builtin_ia32_pause(); }

struct Item {
    int unpack = 0;
    TypeNode *type = nullptr;  // retained
    DeviceTables *dt = nullptr;  // the type's resident tables on the server's device
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
    // the launch holding the item (set before state becomes 2): its stream,
    // slot and launch number on that stream
    struct StreamState *st = nullptr;
    struct Slot *slot = nullptr;
    uint64_t seq = 0;
};

// Allocator over one device allocation: free ranges indexed by offset (for
// coalescing) and by length (best fit in O(log n), so a fragmented arena
// does not make every admission scan the free list).
struct Arena {
    uint8_t *base = nullptr;
    int64_t size = 0;
    std::map<int64_t, int64_t> free_;                  // offset -> length
    std::multimap<int64_t, int64_t> by_len;            // length -> offset
    static int64_t round(int64_t n)
    {
        n = (n + ARENA_ALIGN - 1) / ARENA_ALIGN * ARENA_ALIGN;
        return n == 0 ? ARENA_ALIGN : n;
    }
    void add_free(int64_t off, int64_t len)
    {
        free_[off] = len;
        by_len.emplace(len, off);
    }
    void drop_free(int64_t off, int64_t len)
    {
        free_.erase(off);
        auto r = by_len.equal_range(len);
        for (auto it = r.first; it != r.second; ++it)
            if (it->second == off) {
                by_len.erase(it);
                break;
            }
    }
    void init(uint8_t *b, int64_t n)
    {
        base = b;
        size = n;
        free_.clear();
        by_len.clear();
        add_free(0, n);
    }
    int64_t alloc(int64_t n)
    {
        n = round(n);
        auto it = by_len.lower_bound(n);
        if (it == by_len.end()) return -1;
        const int64_t len = it->first, off = it->second;
        drop_free(off, len);
        if (len > n) add_free(off + n, len - n);
        return off;
    }
    void release(int64_t off, int64_t n)
    {
        n = round(n);
        auto nx = free_.lower_bound(off);
        if (nx != free_.end() && off + n == nx->first) {
            const int64_t l = nx->second;
            drop_free(nx->first, l);
            n += l;
        }
        auto pv = free_.lower_bound(off);
        if (pv != free_.begin()) {
            --pv;
            if (pv->first + pv->second == off) {
                const int64_t po = pv->first, pl = pv->second;
                drop_free(po, pl);
                off = po;
                n += pl;
            }
        }
        add_free(off, n);
    }
};

struct Slot {
    mdt_batch batch = nullptr;
    hipEvent_t ev = nullptr;
    std::vector<Item *> items;
    bool busy = false;
    uint64_t seq = 0;    // launch order on its stream
    int64_t bytes = 0;   // packed bytes of the launch
};

struct StreamState {
    hipStream_t s = nullptr;
    std::vector<Slot> slots;
    int busy = 0;
    uint64_t next_seq = 0;
    int64_t bytes = 0;  // packed bytes of the launches in flight
};

}  // namespace

struct mdt_server_s {
    uint32_t magic = SERVER_MAGIC;
    mdt_server_config cfg{};
    int device = -1;
    std::vector<StreamState> streams;
    Arena arena;
    std::mutex qmu;              // submit queue, released items, submit counters
    std::deque<Item *> queue;
    std::vector<Item *> released;  // completed items the client let go of
    std::mutex mu;               // everything below; held by a progress round
    std::deque<Item *> admitted;
    int64_t inflight = 0, peak_inflight = 0;
    int inject_fail = 0;
    bool draining = false;       // shutdown: admit regardless of the budget
    int next_stream = 0;         // where the next stream choice starts looking
    int64_t direct = 0;          // requests launched by their own submit (direct path)
    // What the progress thread polls, on cache lines of their own: the
    // counters every launch and completion update, and the two timestamps
    // (written by reaps and by testing clients) apart from them.
    alignas(64) std::atomic<bool> run_thread{false};
    std::atomic<int64_t> work{0};   // queued + admitted items + launches in flight
    std::atomic<int> launches_inflight{0};
    alignas(64) std::atomic<double> last_reap{0.0};  // time of the last completion query round
    alignas(64) std::atomic<double> last_client_test{0.0};  // time of the last client test of a launched request
    alignas(64) char pad_end_[1] = {};
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

// Return the arena range and budget charge of items the client released;
// caller holds s->mu and s->qmu.
void take_back_released(mdt_server s)
{
    for (Item *it : s->released) {
        if (it->arena_off >= 0) s->arena.release(it->arena_off, std::max<int64_t>(it->nbytes, 1));
        // admitted requests hold their charge until released
        if (it->arena_off >= 0 || it->unpack) s->inflight -= it->charge;
        release(it->type);
        delete it;
    }
    s->released.clear();
}

Slot *oldest_busy(StreamState &st)
{
    Slot *old = nullptr;
    for (auto &x : st.slots)
        if (x.busy && (!old || x.seq < old->seq)) old = &x;
    return old;
}

// complete the requests of a finished launch; caller holds s->mu
void retire(mdt_server s, StreamState &st, Slot &sl, hipError_t e)
{
    double t = now_us();
    int status = e == hipSuccess ? MDT_SUCCESS : MDT_ERR_HIP;
    if (e != hipSuccess) set_hip_error((int)e);
    for (Item *it : sl.items) complete(s, it, status, t);
    sl.items.clear();
    sl.busy = false;
    st.busy--;
    st.bytes -= sl.bytes;
    sl.bytes = 0;
    s->launches_inflight.fetch_sub(1, std::memory_order_relaxed);
}

// Reap under the lock: a stream finishes its launches in order, so only its
// oldest running launch is queried.  Caller holds s->mu.
void reap_locked(mdt_server s)
{
    s->last_reap.store(now_us(), std::memory_order_relaxed);
    for (auto &st : s->streams) {
        for (;;) {
            Slot *old = oldest_busy(st);
            if (!old) break;
            hipError_t e = hipEventQuery(old->ev);
            if (e == hipErrorNotReady) break;
            retire(s, st, *old, e);
        }
    }
}

// Reap from the progress thread: the events are queried with the lock
// released (a submitter is not held up by the queries); only this thread
// retires launches while it runs, so the snapshot stays valid.
bool reap_unlocked(mdt_server s)
{
    struct Cand {
        StreamState *st;
        Slot *sl;
        uint64_t seq;
        hipEvent_t ev;
        hipError_t e;
    };
    Cand c[64];
    int nc = 0;
    {
        std::lock_guard<std::mutex> g(s->mu);
        for (auto &st : s->streams) {
            Slot *old = oldest_busy(st);
            if (old && nc < 64) c[nc++] = {&st, old, old->seq, old->ev, hipSuccess};
        }
    }
    bool any = false;
    for (int k = 0; k < nc; k++) {
        c[k].e = hipEventQuery(c[k].ev);
        any = any || c[k].e != hipErrorNotReady;
    }
    s->last_reap.store(now_us(), std::memory_order_relaxed);
    if (!any) return false;
    std::lock_guard<std::mutex> g(s->mu);
    for (int k = 0; k < nc; k++)
        if (c[k].e != hipErrorNotReady && c[k].sl->busy && c[k].sl->seq == c[k].seq)
            retire(s, *c[k].st, *c[k].sl, c[k].e);
    return true;
}

// The stream a launch goes to: one with a free slot and the fewest bytes in
// flight, ties going round the streams, so that under light load successive
// launches spread over them (the runtime spreads a process's streams over its
// hardware queues, in a pattern of its own choosing: streams that share a
// queue run their work in order).  Large requests take streams 0, Q, 2Q, ...
// (Q = the hardware queue count) in arrival order; the others use the rest.
// Caller holds s->mu.  NULL when no suitable slot is free.
StreamState *pick_stream(mdt_server s, bool large)
{
    const int nst = (int)s->streams.size();
    const int part = std::max(1, std::min(nst, HW_QUEUES));
    StreamState *best = nullptr;
    int64_t best_load = 0;
    for (int k = 0; k < nst; k++) {
        const int i = (s->next_stream + k) % nst;
        StreamState &st = s->streams[(size_t)i];
        if (st.busy >= (int)st.slots.size()) continue;
        if (part > 1 && (i % part == 0) != large) continue;
        if (!best || st.bytes < best_load || (st.bytes == best_load && st.busy < best->busy)) {
            best = &st;
            best_load = st.bytes;
        }
    }
    if (best) s->next_stream = (int)(best - s->streams.data() + 1) % nst;
    return best;
}

Slot *free_slot(StreamState &st)
{
    for (auto &x : st.slots)
        if (!x.busy) return &x;
    return nullptr;
}

// Launch one request with the single-request kernels (no descriptor
// upload) on stream `st`, slot `sl`, and record the slot's event.  Caller
// holds s->mu.  On failure the request is completed with the error.
int launch_single(mdt_server s, Item *it, StreamState *st, Slot *sl)
{
    int r = MDT_SUCCESS;
    if (it->nbytes > 0) {
        XferArgs A = it->unpack ? make_args(it->out, const_cast<void *>(it->in), it->off, it->nbytes)
                                : make_args(it->in, it->out, it->off, it->nbytes);
        r = launch_xfer(it->dt->lay, A, it->unpack != 0, st->s);
    }
    hipError_t e = r == MDT_SUCCESS ? hipEventRecord(sl->ev, st->s) : hipErrorUnknown;
    if (r != MDT_SUCCESS || e != hipSuccess) {
        if (r == MDT_SUCCESS) set_hip_error((int)e);
        complete(s, it, r ? r : MDT_ERR_HIP, now_us());
        return r ? r : MDT_ERR_HIP;
    }
    sl->items.push_back(it);
    sl->busy = true;
    sl->seq = st->next_seq++;
    it->st = st;
    it->slot = sl;
    it->seq = sl->seq;
    it->t_launch = now_us();
    it->state.store(2, std::memory_order_release);
    sl->bytes = it->nbytes;
    st->busy++;
    st->bytes += sl->bytes;
    s->launches++;
    s->launches_inflight.fetch_add(1, std::memory_order_relaxed);
    return MDT_SUCCESS;
}

// Admit and launch; caller holds s->mu.
int progress_locked(mdt_server s)
{
    int rc = MDT_SUCCESS;
    // 2. return what released items held, then admit queued requests within
    // the budget
    {
        std::lock_guard<std::mutex> q(s->qmu);
        take_back_released(s);
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
        const bool large = s->admitted.front()->nbytes >= LARGE_BYTES;
        const int hwq = std::max(1, std::min((int)s->streams.size(), HW_QUEUES));
        StreamState *best = pick_stream(s, large);
        if (!best) {
            // the large queue is full: let a small request behind go first
            auto it = std::find_if(s->admitted.begin(), s->admitted.end(),
                                   [](const Item *x) { return x->nbytes < LARGE_BYTES; });
            if (!large || hwq == 1 || it == s->admitted.end() || it == s->admitted.begin()) break;
            Item *x = *it;
            s->admitted.erase(it);
            s->admitted.push_front(x);
            continue;
        }
        Slot *sl = free_slot(*best);
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
            int r = launch_single(s, it, best, sl);
            if (r) rc = r;
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
        sl->bytes = bytes;
        best->busy++;
        best->bytes += bytes;
        for (Item *it : sl->items) {
            it->st = best;
            it->slot = sl;
            it->seq = sl->seq;
            it->state.store(2, std::memory_order_release);
        }
        s->launches++;
        s->launches_inflight.fetch_add(1, std::memory_order_relaxed);
    }
    int inflight = 0;
    for (auto &st : s->streams) inflight += st.busy;
    {
        // stored under qmu: a later submit or release adds to this value
        std::lock_guard<std::mutex> q(s->qmu);
        s->work.store((int64_t)(s->queue.size() + s->admitted.size()) + inflight, std::memory_order_release);
    }
    return rc;
}

// a progress round from a caller: reaps unless the progress thread does
int progress(mdt_server s)
{
    std::lock_guard<std::mutex> g(s->mu);
    if (!s->run_thread.load(std::memory_order_acquire)) reap_locked(s);
    return progress_locked(s);
}

// The progress thread runs launching rounds while anything is queued or
// admitted (released requests are taken back by whichever round comes
// next); while launches are only in flight it reaps them at a
// slow cadence (clients testing their requests reap too); when idle it spins
// for a while, then sleeps on a condition variable until a submit wakes it.
void thread_main(mdt_server s)
{
    (void)hipSetDevice(s->device);
    double last_active = now_us();
    while (s->run_thread.load(std::memory_order_acquire)) {
        const int64_t w = s->work.load(std::memory_order_acquire);
        const int nl = s->launches_inflight.load(std::memory_order_relaxed);
        if (w > nl) {
            reap_unlocked(s);
            {
                std::lock_guard<std::mutex> g(s->mu);
                progress_locked(s);
            }
            last_active = now_us();
            continue;
        }
        const double t = now_us();
        if (nl > 0) {
            if (t - s->last_reap.load(std::memory_order_relaxed) >= THREAD_REAP_US &&
                t - s->last_client_test.load(std::memory_order_relaxed) >= CLIENT_QUIET_US && reap_unlocked(s)) {
                std::lock_guard<std::mutex> g(s->mu);
                progress_locked(s);
            } else {
                // nothing to launch: wait out the poll interval, ending early
                // when a submit queues work
                while (now_us() - t < POLL_US && s->work.load(std::memory_order_relaxed) <= nl)
                    for (int k = 0; k < 16; k++) cpu_relax();
            }
            last_active = t;
            continue;
        }
        if (t - last_active < SPIN_US) continue;
        std::unique_lock<std::mutex> q(s->qmu);
        // a 1 ms nap against the system clock: its timed wait is
        // pthread_cond_timedwait, which thread checkers follow (the steady
        // clock's is not intercepted by every ThreadSanitizer runtime)
        s->wake.wait_until(q, std::chrono::system_clock::now() + std::chrono::milliseconds(1), [s] {
            return s->work.load(std::memory_order_acquire) > 0 || !s->run_thread.load(std::memory_order_acquire);
        });
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

// Direct path: with nothing queued or admitted ahead of it and a launch
// slot free, the submitter admits and launches its own request under one
// lock (as a plain enqueue launches), without a queue round trip or a full
// progress round.  Returns false when the request has to queue instead
// (requests waiting, no free slot, budget or arena exhausted); nothing has
// changed then.
bool try_direct(mdt_server s, Item *it)
{
    if (s->work.load(std::memory_order_acquire) != (int64_t)s->launches_inflight.load(std::memory_order_relaxed))
        return false;
    std::lock_guard<std::mutex> g(s->mu);
    if (!s->admitted.empty()) return false;
    {
        std::lock_guard<std::mutex> q(s->qmu);
        if (!s->queue.empty()) return false;
        take_back_released(s);
    }
    if (s->inflight + it->charge > s->cfg.budget_bytes && s->inflight > 0) return false;
    if (!it->unpack && s->inject_fail > 0) return false;  // the queued path reports injected failures
    StreamState *st = pick_stream(s, it->nbytes >= LARGE_BYTES);
    if (!st) return false;
    if (!it->unpack) {
        const int64_t off = s->arena.alloc(std::max<int64_t>(it->nbytes, 1));
        if (off < 0) return false;
        it->arena_off = off;
        it->packed = s->arena.base + off;
        it->out = it->packed;
    }
    s->inflight += it->charge;
    s->peak_inflight = std::max(s->peak_inflight, s->inflight);
    it->state.store(1, std::memory_order_release);
    {
        std::lock_guard<std::mutex> q(s->qmu);
        s->submitted++;
        if (s->first_submit < 0) s->first_submit = it->t_submit;
    }
    s->direct++;
    if (launch_single(s, it, st, free_slot(*st)) == MDT_SUCCESS) {
        std::lock_guard<std::mutex> q(s->qmu);
        s->work.fetch_add(1, std::memory_order_release);
    }
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
    // While a launch slot is free and nothing else waits (or without a
    // progress thread) the submitter runs a progress round itself, so its
    // request is admitted and launched now; it takes the progress lock
    // before queuing, so the progress thread does not race it for the same
    // request.  Once the slots are full or requests queue, it only queues:
    // the progress thread cuts whatever has queued into batched launches,
    // which keeps the cost per submit low and the launches few.
    const bool thread = s->run_thread.load(std::memory_order_acquire);
    if (DIRECT && thread && try_direct(s, it)) {
        *req = r;
        return MDT_SUCCESS;
    }
    const int nl = s->launches_inflight.load(std::memory_order_relaxed);
    const bool waiting = s->work.load(std::memory_order_acquire) > (int64_t)nl;
    auto enqueue = [&] {
        std::lock_guard<std::mutex> q(s->qmu);
        s->submitted++;
        if (s->first_submit < 0) s->first_submit = it->t_submit;
        s->queue.push_back(it);
        s->work.fetch_add(1, std::memory_order_release);  // under qmu: a sleeping thread sees it
    };
    if (!thread || (nl < (int)s->streams.size() * s->cfg.max_inflight && !waiting)) {
        std::lock_guard<std::mutex> g(s->mu);
        enqueue();
        if (!thread) reap_locked(s);
        progress_locked(s);
    } else {
        enqueue();
        s->wake.notify_one();
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
    s->arena.init(s->arena.base, c.arena_bytes);
    s->lat_us.reserve(1 << 22);
    s->queue_us.reserve(1 << 22);
    s->run_us.reserve(1 << 22);
    s->streams.resize(c.nstreams);
    int rc = MDT_SUCCESS;
    for (auto &st : s->streams) {
        if (hipStreamCreateWithFlags(&st.s, hipStreamNonBlocking) != hipSuccess) rc = MDT_ERR_HIP;
        st.slots.resize(c.max_inflight);
        for (auto &sl : st.slots) {
            if (mdt_batch_create(&sl.batch) != MDT_SUCCESS) rc = MDT_ERR_NO_MEM;
            mdt_batch_config bc{1024, 4, 0, 0, 0};
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
    {
        std::lock_guard<std::mutex> g(s->mu);
        std::lock_guard<std::mutex> q(s->qmu);
        take_back_released(s);
    }
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
    mdt::TraceRange trace_("mdt_server_submit_pack");
    if (!valid_server(srv) || !req || inoffset < 0 || max_pack_bytes < -1) return MDT_ERR_ARG;
    Compiled *C;
    DeviceTables *D;
    int64_t total;
    int rc = prepare(t, incount, &C, &D, &total);
    if (rc) return rc;
    int64_t n = std::max<int64_t>(0, total - inoffset);
    if (max_pack_bytes >= 0) n = std::min<int64_t>(n, max_pack_bytes);
    if (n > 0 && !inbuf) return MDT_ERR_ARG;
    if (n > srv->arena.size) return MDT_ERR_NO_MEM;
    auto *it = new (std::nothrow) Item();
    if (!it) return MDT_ERR_NO_MEM;
    it->unpack = 0;
    it->type = reinterpret_cast<TypeNode *>(t);
    it->dt = D;
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
    mdt::TraceRange trace_("mdt_server_submit_unpack");
    if (!valid_server(srv) || !req || insize < 0 || outoffset < 0) return MDT_ERR_ARG;
    Compiled *C;
    DeviceTables *D;
    int64_t total;
    int rc = prepare(t, outcount, &C, &D, &total);
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
    it->dt = D;
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
    const int st = it->state.load(std::memory_order_acquire);
    if (st == 2) {
        const double t = now_us();
        if (t - srv->last_client_test.load(std::memory_order_relaxed) >= CLIENT_MARK_US)
            srv->last_client_test.store(t, std::memory_order_relaxed);
    }
    if (st == 2 && srv->run_thread.load()) {
        // the client queries the event of its own launch only (as the caller
        // of a plain enqueue queries its own event); once it has finished,
        // that launch and the earlier ones on its stream (a stream finishes
        // in order) are retired and waiting requests launched
        Slot *sl = it->slot;
        StreamState *ss = it->st;
        const uint64_t seq = it->seq;
        if (hipEventQuery(sl->ev) != hipErrorNotReady) {
            std::lock_guard<std::mutex> g(srv->mu);
            if (sl->busy && sl->seq == seq) {
                for (;;) {
                    Slot *old = oldest_busy(*ss);
                    if (!old || old->seq > seq) break;
                    hipError_t e = hipEventQuery(old->ev);
                    if (e == hipErrorNotReady) break;  // cannot happen on an in-order stream; keep it queued
                    retire(srv, *ss, *old, e);
                }
                progress_locked(srv);
            }
        }
    } else if (st != 3) {
        if (!srv->run_thread.load()) {
            progress(srv);
        } else if (now_us() - srv->last_reap.load(std::memory_order_relaxed) >= TEST_REAP_US && srv->mu.try_lock()) {
            // the caller reaps (as a caller polling its own event would); the
            // progress thread keeps to launching
            reap_locked(srv);
            progress_locked(srv);
            srv->mu.unlock();
        }
    }
    *flag = it->state.load(std::memory_order_acquire) == 3;
    return MDT_SUCCESS;
}

MDT_API int mdt_server_request_wait(mdt_server srv, mdt_request req)
{
    Item *it = item_of(req);
    if (!valid_server(srv) || !it) return MDT_ERR_ARG;
    int flag = 0;
    for (;;) {
        mdt_server_request_test(srv, req, &flag);
        if (flag) break;
        std::this_thread::yield();
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
        // the next progress round returns its arena range and budget charge
        // (the client never waits for a round in progress)
        std::lock_guard<std::mutex> q(srv->qmu);
        srv->released.push_back(it);  // taken back by the next round; no round of its own
    }
    (*preq)->magic = 0;
    delete *preq;
    *preq = nullptr;
    return MDT_SUCCESS;
}

MDT_API int mdt_server_progress(mdt_server srv)
{
    mdt::TraceRange trace_("mdt_server_progress");
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
    std::lock_guard<std::mutex> q(srv->qmu);
    take_back_released(srv);
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
    out->direct = srv->direct;
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
