// Named ranges around the library's host-side phases (setup, solve, group
// solves, refinement / restart cycles, far field), recorded by a profiler's
// marker trace (rocprofv3 --marker-trace) and free when none is attached.
#pragma once

#include <rocprofiler-sdk-roctx/roctx.h>

namespace vie {

struct TraceRange {
  explicit TraceRange(const char* name) { roctxRangePushA(name); }
  ~TraceRange() { roctxRangePop(); }
  TraceRange(const TraceRange&) = delete;
  TraceRange& operator=(const TraceRange&) = delete;
};

}  // namespace vie
