// Named ranges for profilers (roctx), off unless the environment variable
// RX_ROCTX is set.  The roctx library is opened at run time, so the library
// has no link dependency on it and costs one branch per range when tracing
// is off.  Under `rocprofv3 --marker-trace` the ranges appear beside the
// kernels they enclose (entry points, server steps).
#include <dlfcn.h>

#include <cstdlib>

#include "rx_internal.h"

namespace rx {

namespace {
struct RoctxFns {
    int (*push)(const char*) = nullptr;
    int (*pop)() = nullptr;
};

RoctxFns load_roctx() {
    RoctxFns f;
    const char* on = std::getenv("RX_ROCTX");
    if (!on || !*on || *on == '0') return f;
    for (const char* name : {"librocprofiler-sdk-roctx.so.1", "/opt/rocm/lib/librocprofiler-sdk-roctx.so.1",
                             "libroctx64.so.4", "/opt/rocm/lib/libroctx64.so.4"}) {
        void* h = dlopen(name, RTLD_NOW | RTLD_LOCAL);
        if (!h) continue;
        f.push = reinterpret_cast<int (*)(const char*)>(dlsym(h, "roctxRangePushA"));
        f.pop = reinterpret_cast<int (*)()>(dlsym(h, "roctxRangePop"));
        if (f.push && f.pop) return f;
        f = RoctxFns();
    }
    return f;
}

const RoctxFns& roctx() {
    static const RoctxFns f = load_roctx();
    return f;
}
}  // namespace

TraceRange::TraceRange(const char* name) : on_(roctx().push != nullptr) {
    if (on_) roctx().push(name);
}

TraceRange::~TraceRange() {
    if (on_) roctx().pop();
}

bool trace_enabled() { return roctx().push != nullptr; }

}  // namespace rx
