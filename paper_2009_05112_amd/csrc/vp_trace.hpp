// vp_trace.hpp -- ROCTx ranges around the library's host-side phases (problem
// set-up, the enqueueing of iterations, result reads; the serving loop's
// admission, planning, step and retirement), so that a profiler's marker
// trace (rocprofv3 --marker-trace) shows them beside the kernels.  The calls
// cost next to nothing when no profiler is attached.
#pragma once

#include <rocprofiler-sdk-roctx/roctx.h>

namespace vp {

class TraceRange {
public:
    explicit TraceRange(const char* what) { roctxRangePushA(what); }
    ~TraceRange() { roctxRangePop(); }
    TraceRange(const TraceRange&) = delete;
    TraceRange& operator=(const TraceRange&) = delete;
};

}  // namespace vp
