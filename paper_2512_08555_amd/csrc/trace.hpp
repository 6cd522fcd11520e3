// Observability of the host side:
//  - roctx ranges around the library's enqueue steps (the plan's setup, a
//    solve and each of its passes, a batch graph launch, a multigrid cycle,
//    the autotuner), visible with `rocprofv3 --marker-trace`; a range spans
//    the host call that enqueues the work, the kernels it launches follow it
//    on the stream;
//  - logging to stderr, chosen by the environment variable UPS_LOG_LEVEL:
//    0 or unset: silent; 1: every failed call with its status and message;
//    2: also plan, batch, cycle and autotuner decisions (kernels, schedule,
//    buffer sizes); 3: also every solve, batch launch and cycle.
#pragma once
#include <rocprofiler-sdk-roctx/roctx.h>

namespace ups {

// UPS_LOG_LEVEL, read once (values outside 0 .. 3 are clamped)
int log_level();
// one line "[ups] ..." on stderr if level <= log_level()
void logf(int level, const char* fmt, ...) __attribute__((format(printf, 2, 3)));

class TraceRange {
 public:
  explicit TraceRange(const char* name) { roctxRangePushA(name); }
  ~TraceRange() { roctxRangePop(); }
  TraceRange(const TraceRange&) = delete;
  TraceRange& operator=(const TraceRange&) = delete;
};

}  // namespace ups
