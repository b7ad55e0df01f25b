// server_stub.cpp -- a data-free executor for host-only builds of the serving
// loop (paper_2402_12274_amd/csrc/server.cpp, compiled unchanged with the
// host compiler): the HIP streams, events and memory calls, the single-request
// launch and the batch calls it uses are replaced by a virtual device on which
// each launch occupies its stream for a time that grows with its bytes.  It
// moves no bytes and reads no data; it exists to run the loop's scheduling and
// host concurrency on the CPU (under ThreadSanitizer in the tests).
#include <hip/hip_runtime_api.h>

#include <algorithm>
#include <atomic>
#include <chrono>
#include <cstdlib>
#include <mutex>
#include <vector>

#include "core.h"
#include "device.h"
#include "requests.h"

namespace {

double now_us()
{
    using namespace std::chrono;
    return (double)duration_cast<nanoseconds>(steady_clock::now().time_since_epoch()).count() * 1e-3;
}

// A virtual stream: work queued on it finishes in order, each launch taking
// 2 us plus 1 us per 16 KiB.
struct StubStream {
    std::mutex mu;
    double busy_until = 0;
};

struct StubEvent {
    std::atomic<double> done_at{-1.0};  // -1: never recorded (complete)
};

StubStream g_null_stream;

StubStream *stream_of(hipStream_t s) { return s ? reinterpret_cast<StubStream *>(s) : &g_null_stream; }

void occupy(hipStream_t s, int64_t bytes)
{
    StubStream *st = stream_of(s);
    std::lock_guard<std::mutex> g(st->mu);
    st->busy_until = std::max(st->busy_until, now_us()) + 2.0 + (double)bytes / 16384.0;
}

std::atomic<int64_t> g_launches{0};

}  // namespace

// ---- HIP runtime calls the serving loop makes ---------------------------

extern "C" {

hipError_t hipGetDevice(int *d)
{
    *d = 0;
    return hipSuccess;
}

hipError_t hipSetDevice(int) { return hipSuccess; }

hipError_t hipDeviceSynchronize(void) { return hipSuccess; }

hipError_t hipMalloc(void **p, size_t n)
{
    // the arena is never touched: reserve address space only
    *p = std::malloc(std::max<size_t>(n, 1));
    return *p ? hipSuccess : hipErrorOutOfMemory;
}

hipError_t hipFree(void *p)
{
    std::free(p);
    return hipSuccess;
}

hipError_t hipStreamCreateWithFlags(hipStream_t *s, unsigned int)
{
    *s = reinterpret_cast<hipStream_t>(new StubStream());
    return hipSuccess;
}

hipError_t hipStreamDestroy(hipStream_t s)
{
    delete reinterpret_cast<StubStream *>(s);
    return hipSuccess;
}

hipError_t hipEventCreateWithFlags(hipEvent_t *e, unsigned)
{
    *e = reinterpret_cast<hipEvent_t>(new StubEvent());
    return hipSuccess;
}

hipError_t hipEventDestroy(hipEvent_t e)
{
    delete reinterpret_cast<StubEvent *>(e);
    return hipSuccess;
}

hipError_t hipEventRecord(hipEvent_t e, hipStream_t s)
{
    StubStream *st = stream_of(s);
    std::lock_guard<std::mutex> g(st->mu);
    reinterpret_cast<StubEvent *>(e)->done_at.store(std::max(st->busy_until, now_us()), std::memory_order_release);
    return hipSuccess;
}

hipError_t hipEventQuery(hipEvent_t e)
{
    const double t = reinterpret_cast<StubEvent *>(e)->done_at.load(std::memory_order_acquire);
    return t <= now_us() ? hipSuccess : hipErrorNotReady;
}

}  // extern "C"

// ---- the library pieces the loop calls ------------------------------------

struct mdt_batch_s {
    std::vector<int64_t> bytes;
};

namespace mdt {

Compiled::~Compiled() = default;

void set_hip_error(int) {}

void retain(TypeNode *t) { t->refs.fetch_add(1, std::memory_order_relaxed); }

void release(TypeNode *t)
{
    if (t->refs.fetch_sub(1, std::memory_order_acq_rel) == 1) delete t;
}

int check_unpack_overlap(Compiled *, int64_t) { return MDT_SUCCESS; }

static DeviceTables g_tables;

int prepare(mdt_type th, int64_t count, Compiled **C, DeviceTables **D, int64_t *total)
{
    TypeNode *t = reinterpret_cast<TypeNode *>(th);
    if (!t || t->magic != 0x6d647421u || !t->committed.load()) return MDT_ERR_TYPE;
    if (count < 0) return MDT_ERR_ARG;
    if (__builtin_mul_overflow(count, t->size, total)) return MDT_ERR_COUNT;
    *C = t->comp.get();
    if (D) *D = &g_tables;
    return MDT_SUCCESS;
}

XferArgs make_args(const void *typed, void *packed, int64_t off, int64_t nbytes)
{
    XferArgs A{};
    A.typed = (const uint8_t *)typed;
    A.packed = (uint8_t *)packed;
    A.off = off;
    A.nbytes = nbytes;
    return A;
}

int launch_xfer(const DevLayout &, const XferArgs &A, bool, hipStream_t s)
{
    g_launches.fetch_add(1, std::memory_order_relaxed);
    occupy(s, A.nbytes);
    return MDT_SUCCESS;
}

int batch_launch_internal(mdt_batch b, hipStream_t s)
{
    int64_t n = 0;
    for (int64_t x : b->bytes) n += x;
    g_launches.fetch_add(1, std::memory_order_relaxed);
    occupy(s, n);
    return MDT_SUCCESS;
}

}  // namespace mdt

// A committed stub type of `size` bytes per element and extent `extent`.
mdt_type stub_type(int64_t size, int64_t extent)
{
    auto *t = new mdt::TypeNode();
    t->size = size;
    t->lb = 0;
    t->ub = extent;
    t->tlb = 0;
    t->tub = extent;
    t->comp = std::make_shared<mdt::Compiled>();
    t->committed.store(true);
    return reinterpret_cast<mdt_type>(t);
}

int64_t stub_launches() { return g_launches.load(); }

extern "C" {

MDT_API int mdt_batch_create(mdt_batch *b)
{
    *b = new mdt_batch_s();
    return MDT_SUCCESS;
}

MDT_API int mdt_batch_free(mdt_batch *b)
{
    delete *b;
    *b = nullptr;
    return MDT_SUCCESS;
}

MDT_API int mdt_batch_clear(mdt_batch b)
{
    b->bytes.clear();
    return MDT_SUCCESS;
}

MDT_API int mdt_batch_set_config(mdt_batch, const mdt_batch_config *) { return MDT_SUCCESS; }

MDT_API int mdt_batch_add_pack(mdt_batch b, const void *, mdt_count incount, mdt_type t, mdt_count inoffset, void *,
                               mdt_count max_pack_bytes, mdt_count *actual)
{
    mdt::TypeNode *n = reinterpret_cast<mdt::TypeNode *>(t);
    int64_t k = std::max<int64_t>(0, incount * n->size - inoffset);
    if (max_pack_bytes >= 0) k = std::min<int64_t>(k, max_pack_bytes);
    b->bytes.push_back(k);
    *actual = k;
    return MDT_SUCCESS;
}

MDT_API int mdt_batch_add_unpack(mdt_batch b, const void *, mdt_count insize, void *, mdt_count, mdt_type, mdt_count,
                                 mdt_count *actual)
{
    b->bytes.push_back(insize);
    *actual = insize;
    return MDT_SUCCESS;
}

}  // extern "C"
