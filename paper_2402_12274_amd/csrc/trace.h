// trace.h -- optional roctx ranges around the library's host-side operations
// (commit, pack/unpack/copy calls and their enqueue forms, device flatten,
// batch launch and tuning, server submits and progress rounds), for a
// profiler's marker trace (rocprofv3 --marker-trace).  Off unless the
// environment sets MDT_ROCTX=1; the roctx library is then loaded at first
// use, and tracing stays off if it is not installed.
#pragma once

namespace mdt {

bool trace_on();
void trace_push(const char *name);
void trace_pop();

// A range for the enclosing scope.
class TraceRange {
public:
    explicit TraceRange(const char *name) : on_(trace_on())
    {
        if (on_) trace_push(name);
    }
    ~TraceRange()
    {
        if (on_) trace_pop();
    }
    TraceRange(const TraceRange &) = delete;
    TraceRange &operator=(const TraceRange &) = delete;

private:
    bool on_;
};

}  // namespace mdt
