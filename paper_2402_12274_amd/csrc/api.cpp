// api.cpp -- C ABI: pack / unpack (blocking and stream-enqueued), device
// flatten, streams and requests.
//
// Offloading Asynchronous Operations: work enqueued on a GPU stream runs in
// that stream's order; the host side only starts it and later waits for it.
// Accordingly every *_enqueue call validates its arguments, derives the
// number of bytes it will move from sizes alone (so the caller learns it
// immediately), launches on the caller's stream and, if asked, records an
// event into a request.  The blocking calls are enqueue on the null stream
// followed by a wait.
#include <hip/hip_runtime_api.h>

#include <mutex>
#include <vector>

#include "core.h"
#include "device.h"
#include "requests.h"
#include "trace.h"

namespace mdt {

namespace {

struct EventPool {
    std::mutex mu;
    std::vector<hipEvent_t> free;
} g_events;

}  // namespace

int event_get(hipEvent_t *ev)
{
    {
        std::lock_guard<std::mutex> g(g_events.mu);
        if (!g_events.free.empty()) {
            *ev = g_events.free.back();
            g_events.free.pop_back();
            return MDT_SUCCESS;
        }
    }
    hipError_t e = hipEventCreateWithFlags(ev, hipEventDisableTiming);
    if (e != hipSuccess) {
        set_hip_error((int)e);
        return MDT_ERR_HIP;
    }
    return MDT_SUCCESS;
}

void event_put(hipEvent_t ev)
{
    std::lock_guard<std::mutex> g(g_events.mu);
    g_events.free.push_back(ev);
}

int request_from_stream(hipStream_t s, mdt_request *req, mdt_stream owner)
{
    if (!req) return MDT_SUCCESS;
    auto *r = new (std::nothrow) mdt_request_s();
    if (!r) return MDT_ERR_NO_MEM;
    int rc = event_get(&r->ev);
    if (rc) {
        delete r;
        return rc;
    }
    hipError_t e = hipEventRecord(r->ev, s);
    if (e != hipSuccess) {
        event_put(r->ev);
        delete r;
        set_hip_error((int)e);
        return MDT_ERR_HIP;
    }
    r->kind = REQ_EVENT;
    if (owner) list_add(&owner->live, r);  // reachable by the stream's progress
    *req = r;
    return MDT_SUCCESS;
}

// Validate (count x t) and fetch its compiled form and device tables.
int prepare(mdt_type th, int64_t count, Compiled **C, DeviceTables **D, int64_t *total)
{
    TypeNode *t = reinterpret_cast<TypeNode *>(th);
    if (!valid_type(t)) return MDT_ERR_TYPE;
    if (!t->committed.load()) {
        if (!t->predefined) return MDT_ERR_TYPE;
        int rc = commit_type(t);
        if (rc) return rc;
    }
    if (count < 0) return MDT_ERR_ARG;
    int64_t v, w;
    if (__builtin_mul_overflow(count, t->size, total)) return MDT_ERR_COUNT;
    if (count > 0) {
        if (__builtin_mul_overflow(count - 1, t->extent(), &v)) return MDT_ERR_COUNT;
        if (__builtin_add_overflow(v, t->tub, &w) || __builtin_add_overflow(v, t->tlb, &w)) return MDT_ERR_COUNT;
    }
    *C = t->comp.get();
    if (D) return device_tables(*C, D);
    return MDT_SUCCESS;
}

int pack_common(const void *inbuf, int64_t incount, mdt_type t, int64_t inoffset, void *outbuf, int64_t max_bytes,
                int64_t *actual, hipStream_t s, mdt_request *req, mdt_stream owner = nullptr)
{
    if (!actual || inoffset < 0 || max_bytes < -1) return MDT_ERR_ARG;
    Compiled *C;
    DeviceTables *D;
    int64_t total;
    int rc = prepare(t, incount, &C, &D, &total);
    if (rc) return rc;
    int64_t n = total - inoffset;
    if (n < 0) n = 0;
    if (max_bytes >= 0 && n > max_bytes) n = max_bytes;
    if (n > 0 && (!inbuf || !outbuf)) return MDT_ERR_ARG;
    if (n > 0) {
        XferArgs A = make_args(inbuf, outbuf, inoffset, n);
        rc = launch_xfer(D->lay, A, false, s);
        if (rc) return rc;
    }
    rc = request_from_stream(s, req, owner);
    if (rc) return rc;
    *actual = n;
    return MDT_SUCCESS;
}

int unpack_common(const void *inbuf, int64_t insize, void *outbuf, int64_t outcount, mdt_type t, int64_t outoffset,
                  int64_t *actual, hipStream_t s, mdt_request *req, mdt_stream owner = nullptr)
{
    if (!actual || insize < 0 || outoffset < 0) return MDT_ERR_ARG;
    Compiled *C;
    DeviceTables *D;
    int64_t total;
    int rc = prepare(t, outcount, &C, &D, &total);
    if (rc) return rc;
    int64_t remaining = total - outoffset;
    if (remaining < 0) remaining = 0;
    if (insize > remaining) return MDT_ERR_TRUNCATE;
    rc = check_unpack_overlap(C, outcount);
    if (rc) return rc;
    if (insize > 0 && (!inbuf || !outbuf)) return MDT_ERR_ARG;
    if (insize > 0) {
        XferArgs A = make_args(outbuf, const_cast<void *>(inbuf), outoffset, insize);
        rc = launch_xfer(D->lay, A, true, s);
        if (rc) return rc;
    }
    rc = request_from_stream(s, req, owner);
    if (rc) return rc;
    *actual = insize;
    return MDT_SUCCESS;
}

int copy_common(const void *src, int64_t srccount, mdt_type srctype, void *dst, int64_t dstcount, mdt_type dsttype,
                int64_t offset, int64_t max_bytes, int64_t *actual, hipStream_t s, mdt_request *req,
                mdt_stream owner = nullptr)
{
    if (!actual || offset < 0 || max_bytes < -1) return MDT_ERR_ARG;
    Compiled *Cs, *Cd;
    DeviceTables *Ds = nullptr, *Dd = nullptr;
    int64_t total_s, total_d;
    // sizes, truncation and overlap are checked before any device work
    int rc = prepare(srctype, srccount, &Cs, nullptr, &total_s);
    if (rc) return rc;
    rc = prepare(dsttype, dstcount, &Cd, nullptr, &total_d);
    if (rc) return rc;
    int64_t n = total_s - offset;
    if (n < 0) n = 0;
    if (max_bytes >= 0 && n > max_bytes) n = max_bytes;
    int64_t room = total_d - offset;
    if (room < 0) room = 0;
    if (n > room) return MDT_ERR_TRUNCATE;
    rc = check_unpack_overlap(Cd, dstcount);
    if (rc) return rc;
    if (n > 0 && (!src || !dst)) return MDT_ERR_ARG;
    if (n > 0) {
        rc = device_tables(Cs, &Ds);
        if (rc) return rc;
        rc = device_tables(Cd, &Dd);
        if (rc) return rc;
        CopyArgs A{};
        A.src = (const uint8_t *)src;
        A.dst = (uint8_t *)dst;
        A.off = offset;
        A.nbytes = n;
        A.nchunks = (n + 15) / 16;
        A.src_elem1 = offset + n <= Ds->lay.size;
        A.dst_elem1 = offset + n <= Dd->lay.size;
        rc = launch_copy(Ds->lay, Dd->lay, A, s);
        if (rc) return rc;
    }
    rc = request_from_stream(s, req, owner);
    if (rc) return rc;
    *actual = n;
    return MDT_SUCCESS;
}

void free_request(mdt_request r)
{
    if (r->list) list_remove(r);
    if (r->kind == REQ_EVENT) event_put(r->ev);
    r->magic = 0;
    delete r;
}

}  // namespace mdt

using namespace mdt;

static bool valid_stream(mdt_stream s) { return s && s->magic == STREAM_MAGIC; }

extern "C" {

MDT_API int mdt_pack(const void *inbuf, mdt_count incount, mdt_type t, mdt_count inoffset, void *outbuf,
                     mdt_count max_pack_bytes, mdt_count *actual_pack_bytes)
{
    mdt::TraceRange trace_("mdt_pack");
    if (!actual_pack_bytes) return MDT_ERR_ARG;
    int64_t n = 0;
    int rc = pack_common(inbuf, incount, t, inoffset, outbuf, max_pack_bytes, &n, nullptr, nullptr);
    if (rc) return rc;
    hipError_t e = hipStreamSynchronize(nullptr);
    if (e != hipSuccess) {
        set_hip_error((int)e);
        return MDT_ERR_HIP;
    }
    *actual_pack_bytes = n;
    return MDT_SUCCESS;
}

MDT_API int mdt_typed_copy(const void *src, mdt_count srccount, mdt_type srctype, void *dst, mdt_count dstcount,
                           mdt_type dsttype, mdt_count offset, mdt_count max_bytes, mdt_count *actual)
{
    mdt::TraceRange trace_("mdt_typed_copy");
    if (!actual) return MDT_ERR_ARG;
    int64_t n = 0;
    int rc = copy_common(src, srccount, srctype, dst, dstcount, dsttype, offset, max_bytes, &n, nullptr, nullptr);
    if (rc) return rc;
    hipError_t e = hipStreamSynchronize(nullptr);
    if (e != hipSuccess) {
        set_hip_error((int)e);
        return MDT_ERR_HIP;
    }
    *actual = n;
    return MDT_SUCCESS;
}

MDT_API int mdt_unpack(const void *inbuf, mdt_count insize, void *outbuf, mdt_count outcount, mdt_type t,
                       mdt_count outoffset, mdt_count *actual_unpack_bytes)
{
    mdt::TraceRange trace_("mdt_unpack");
    if (!actual_unpack_bytes) return MDT_ERR_ARG;
    int64_t n = 0;
    int rc = unpack_common(inbuf, insize, outbuf, outcount, t, outoffset, &n, nullptr, nullptr);
    if (rc) return rc;
    hipError_t e = hipStreamSynchronize(nullptr);
    if (e != hipSuccess) {
        set_hip_error((int)e);
        return MDT_ERR_HIP;
    }
    *actual_unpack_bytes = n;
    return MDT_SUCCESS;
}

MDT_API int mdt_stream_create(mdt_hip_stream s, mdt_stream *out)
{
    if (!out) return MDT_ERR_ARG;
    auto *st = new (std::nothrow) mdt_stream_s();
    if (!st) return MDT_ERR_NO_MEM;
    st->magic = STREAM_MAGIC;
    st->s = reinterpret_cast<hipStream_t>(s);
    streams_register(st);
    *out = st;
    return MDT_SUCCESS;
}

MDT_API int mdt_stream_free(mdt_stream *s)
{
    if (!s || !valid_stream(*s)) return MDT_ERR_ARG;
    mdt_stream st = *s;
    mdt_stop_progress_thread(st);
    streams_unregister(st);  // no general progress pass reaches it from here on
    // its requests stay valid (completed by test or wait); they leave its list
    for (;;) {
        mdt_request r;
        {
            std::lock_guard<std::mutex> g(st->live.mu);
            r = st->live.head;
        }
        if (!r) break;
        list_remove(r);
    }
    st->magic = 0;
    delete st;
    *s = nullptr;
    return MDT_SUCCESS;
}

MDT_API int mdt_pack_enqueue(const void *inbuf, mdt_count incount, mdt_type t, mdt_count inoffset,
                             void *outbuf, mdt_count max_pack_bytes, mdt_count *actual_pack_bytes,
                             mdt_stream s, mdt_request *req)
{
    mdt::TraceRange trace_("mdt_pack_enqueue");
    if (!valid_stream(s)) return MDT_ERR_ARG;
    return pack_common(inbuf, incount, t, inoffset, outbuf, max_pack_bytes, actual_pack_bytes, s->s, req, s);
}

MDT_API int mdt_unpack_enqueue(const void *inbuf, mdt_count insize, void *outbuf, mdt_count outcount,
                               mdt_type t, mdt_count outoffset, mdt_count *actual_unpack_bytes,
                               mdt_stream s, mdt_request *req)
{
    mdt::TraceRange trace_("mdt_unpack_enqueue");
    if (!valid_stream(s)) return MDT_ERR_ARG;
    return unpack_common(inbuf, insize, outbuf, outcount, t, outoffset, actual_unpack_bytes, s->s, req, s);
}

MDT_API int mdt_typed_copy_enqueue(const void *src, mdt_count srccount, mdt_type srctype, void *dst,
                                   mdt_count dstcount, mdt_type dsttype, mdt_count offset, mdt_count max_bytes,
                                   mdt_count *actual, mdt_stream s, mdt_request *req)
{
    mdt::TraceRange trace_("mdt_typed_copy_enqueue");
    if (!valid_stream(s)) return MDT_ERR_ARG;
    return copy_common(src, srccount, srctype, dst, dstcount, dsttype, offset, max_bytes, actual, s->s, req, s);
}

MDT_API int mdt_type_iov_enqueue(mdt_type t, mdt_count iov_offset, mdt_iov *dev_iov, mdt_count max_iov_len,
                                 const void *base, mdt_count *actual_iov_len, mdt_stream s, mdt_request *req)
{
    mdt::TraceRange trace_("mdt_type_iov_enqueue");
    if (!valid_stream(s) || !actual_iov_len || iov_offset < 0 || max_iov_len < 0) return MDT_ERR_ARG;
    if (max_iov_len > 0 && !dev_iov) return MDT_ERR_ARG;
    Compiled *C;
    DeviceTables *D;
    int64_t total;
    int rc = prepare(t, 1, &C, &D, &total);
    if (rc) return rc;
    int64_t nseg = C->nruns;
    if (!C->merge_free) {
        rc = build_segment_table(C);
        if (rc) return rc;
        nseg = (int64_t)C->seg_addr.size();
    }
    int64_t m = iov_offset >= nseg ? 0 : std::min<int64_t>(max_iov_len, nseg - iov_offset);
    rc = launch_flatten(C, D, iov_offset, m, dev_iov, base, s->s);
    if (rc) return rc;
    rc = request_from_stream(s->s, req, s);
    if (rc) return rc;
    *actual_iov_len = m;
    return MDT_SUCCESS;
}

MDT_API int mdt_type_iov_count_enqueue(mdt_type t, mdt_count count, mdt_count iov_offset, mdt_iov *dev_iov,
                                       mdt_count max_iov_len, const void *base, mdt_count *actual_iov_len,
                                       mdt_stream s, mdt_request *req)
{
    mdt::TraceRange trace_("mdt_type_iov_count_enqueue");
    if (!valid_stream(s) || !actual_iov_len || count < 0 || iov_offset < 0 || max_iov_len < 0) return MDT_ERR_ARG;
    if (max_iov_len > 0 && !dev_iov) return MDT_ERR_ARG;
    Compiled *C;
    DeviceTables *D;
    int64_t total;
    int rc = prepare(t, 1, &C, &D, &total);
    if (rc) return rc;
    SegCount sc{};
    rc = element_segments(reinterpret_cast<TypeNode *>(t), &sc, count);
    if (rc) return rc;
    int64_t m = iov_offset >= sc.total ? 0 : std::min<int64_t>(max_iov_len, sc.total - iov_offset);
    rc = launch_flatten(C, D, iov_offset, m, dev_iov, base, s->s, &sc);
    if (rc) return rc;
    rc = request_from_stream(s->s, req, s);
    if (rc) return rc;
    *actual_iov_len = m;
    return MDT_SUCCESS;
}

}  // extern "C"
