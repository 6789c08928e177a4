// Host-side ranges for a tracer (roctx): one range per library call that steps, and one per step or sweep inside
// it. The roctx runtime is opened at the first range; without it, or without a tracer attached to it, a range
// costs a branch or a call into an idle library. `rocprofv3 --marker-trace` records the ranges.
#pragma once

namespace wdg {

void trace_push(const char* name);
void trace_pop();

struct TraceRange {
    explicit TraceRange(const char* name) { trace_push(name); }
    ~TraceRange() { trace_pop(); }
    TraceRange(const TraceRange&) = delete;
    TraceRange& operator=(const TraceRange&) = delete;
};

}  // namespace wdg
