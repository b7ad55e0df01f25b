// requests.h -- stream and request objects behind the opaque C handles.
#pragma once

#include <hip/hip_runtime_api.h>

#include "core.h"

constexpr uint32_t STREAM_MAGIC = 0x6d647353u;
constexpr uint32_t REQUEST_MAGIC = 0x6d647252u;

enum ReqKind { REQ_EVENT = 0, REQ_SERVER = 1, REQ_GENERAL = 2 };

struct mdt_stream_s {
    uint32_t magic = STREAM_MAGIC;
    hipStream_t s = nullptr;
};

struct mdt_request_s {
    uint32_t magic = REQUEST_MAGIC;
    int kind = REQ_EVENT;
    hipEvent_t ev = nullptr;  // REQ_EVENT: completes with the recorded work
    void *server_item = nullptr;  // REQ_SERVER: the server's record of the request
    void *general = nullptr;      // REQ_GENERAL: callbacks and completion flag
};

namespace mdt {
int event_get(hipEvent_t *ev);
void event_put(hipEvent_t ev);
int request_from_stream(hipStream_t s, mdt_request *req);
void free_request(mdt_request r);
int prepare(mdt_type t, int64_t count, Compiled **C, DeviceTables **D, int64_t *total);
}  // namespace mdt
