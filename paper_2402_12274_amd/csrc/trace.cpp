// trace.cpp -- the roctx calls behind trace.h, resolved at first use.
#include "trace.h"

#include <dlfcn.h>

#include <cstdlib>
#include <cstring>
#include <mutex>

namespace mdt {

namespace {

using push_fn = int (*)(const char *);
using pop_fn = int (*)();

struct Roctx {
    push_fn push = nullptr;
    pop_fn pop = nullptr;
    bool on = false;
};

const Roctx &roctx()
{
    static Roctx r;
    static std::once_flag once;
    std::call_once(once, [] {
        const char *e = std::getenv("MDT_ROCTX");
        if (!e || std::strcmp(e, "1") != 0) return;
        // the profiler SDK's roctx first, then the older library
        for (const char *lib : {"librocprofiler-sdk-roctx.so.1", "librocprofiler-sdk-roctx.so", "libroctx64.so.4",
                                "libroctx64.so"}) {
            void *h = dlopen(lib, RTLD_NOW | RTLD_GLOBAL);
            if (!h) continue;
            r.push = reinterpret_cast<push_fn>(dlsym(h, "roctxRangePushA"));
            r.pop = reinterpret_cast<pop_fn>(dlsym(h, "roctxRangePop"));
            if (r.push && r.pop) {
                r.on = true;
                return;
            }
            r.push = nullptr;
            r.pop = nullptr;
        }
    });
    return r;
}

}  // namespace

bool trace_on() { return roctx().on; }

void trace_push(const char *name)
{
    const Roctx &r = roctx();
    if (r.on) r.push(name);
}

void trace_pop()
{
    const Roctx &r = roctx();
    if (r.on) r.pop();
}

}  // namespace mdt
