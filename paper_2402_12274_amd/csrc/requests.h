// requests.h -- stream and request objects behind the opaque C handles.
#pragma once

#include <hip/hip_runtime_api.h>

#include <atomic>
#include <mutex>
#include <thread>

#include "core.h"

constexpr uint32_t STREAM_MAGIC = 0x6d647353u;
constexpr uint32_t REQUEST_MAGIC = 0x6d647252u;

enum ReqKind { REQ_EVENT = 0, REQ_SERVER = 1, REQ_GENERAL = 2 };

struct mdt_request_s;

// Requests that a progress call can reach: an intrusive list (O(1) insert
// and removal) under a mutex.  A progress pass pins the requests it looks
// at, so a completion call that frees one waits for the pass to let go.
struct ReqList {
    std::mutex mu;
    mdt_request_s *head = nullptr;
    std::atomic<int64_t> count{0};
};

struct mdt_stream_s {
    uint32_t magic = STREAM_MAGIC;
    hipStream_t s = nullptr;
    ReqList live;                     // event requests of work enqueued on this stream
    std::atomic<bool> run{false};     // its progress thread runs
    std::thread th;
};

struct mdt_request_s {
    uint32_t magic = REQUEST_MAGIC;
    int kind = REQ_EVENT;
    hipEvent_t ev = nullptr;  // REQ_EVENT: completes with the recorded work
    void *server_item = nullptr;  // REQ_SERVER: the server's record of the request
    void *general = nullptr;      // REQ_GENERAL: callbacks and completion flag
    std::atomic<int> done{0};     // REQ_EVENT: completion seen by a test or a progress pass
    // membership of a progress list (event requests of a stream, or the
    // generalized requests)
    ReqList *list = nullptr;
    mdt_request_s *prev = nullptr, *next = nullptr;
    std::atomic<int> pins{0};
};

namespace mdt {
int event_get(hipEvent_t *ev);
void event_put(hipEvent_t ev);
int request_from_stream(hipStream_t s, mdt_request *req, mdt_stream owner = nullptr);
void free_request(mdt_request r);
int prepare(mdt_type t, int64_t count, Compiled **C, DeviceTables **D, int64_t *total);
// progress lists
void list_add(ReqList *l, mdt_request r);
void list_remove(mdt_request r);  // also waits until no progress pass holds r
void streams_register(mdt_stream s);
void streams_unregister(mdt_stream s);
}  // namespace mdt
