// roctx ranges around the C ABI calls (start-up, steps, queries), visible to rocprofv3
// --marker-trace and other ROCm tools; a push and a pop per call when no tool listens.
#pragma once

#include <rocprofiler-sdk-roctx/roctx.h>

namespace spfc {

struct TraceRange {
    explicit TraceRange(const char* name) { roctxRangePushA(name); }
    ~TraceRange() { roctxRangePop(); }
    TraceRange(const TraceRange&) = delete;
    TraceRange& operator=(const TraceRange&) = delete;
};

}  // namespace spfc
