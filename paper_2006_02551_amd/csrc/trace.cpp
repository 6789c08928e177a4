// roctx ranges opened at run time (no link-time dependency on the tracer runtime).
#include "trace.hpp"

#include <dlfcn.h>

#include <cstdlib>
#include <mutex>

namespace wdg {
namespace {

using PushFn = int (*)(const char*);
using PopFn = int (*)();

struct Roctx {
    PushFn push = nullptr;
    PopFn pop = nullptr;
};

const Roctx& roctx() {
    static Roctx r;
    static std::once_flag once;
    std::call_once(once, [] {
        // WDG_TRACE=0 turns the ranges off; the library handle is kept until the process ends
        const char* env = std::getenv("WDG_TRACE");
        if (env && env[0] == '0') return;
        for (const char* name : {"librocprofiler-sdk-roctx.so.1", "librocprofiler-sdk-roctx.so"}) {
            void* h = dlopen(name, RTLD_NOW | RTLD_LOCAL);
            if (!h) continue;
            auto push = reinterpret_cast<PushFn>(dlsym(h, "roctxRangePushA"));
            auto pop = reinterpret_cast<PopFn>(dlsym(h, "roctxRangePop"));
            if (push && pop) {
                r.push = push;
                r.pop = pop;
                return;
            }
        }
    });
    return r;
}

}  // namespace

void trace_push(const char* name) {
    const Roctx& r = roctx();
    if (r.push) r.push(name);
}

void trace_pop() {
    const Roctx& r = roctx();
    if (r.pop) r.pop();
}

}  // namespace wdg
