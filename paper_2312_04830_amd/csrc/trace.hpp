// Tracing of the C-ABI calls with roctx ranges.
#pragma once

#include <rocprofiler-sdk-roctx/roctx.h>

namespace props {

// A roctx range named after a C-ABI call, open for the call's host-side duration: the
// asynchronous work it enqueues shows up inside it under rocprofv3 --marker-trace.  Without
// a profiler attached the push and pop return at once.
struct ApiRange {
    explicit ApiRange(const char *name) { roctxRangePushA(name); }
    ~ApiRange() { roctxRangePop(); }
    ApiRange(const ApiRange &) = delete;
    ApiRange &operator=(const ApiRange &) = delete;
};

}  // namespace props
