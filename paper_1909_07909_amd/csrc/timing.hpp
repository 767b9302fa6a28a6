// Optional per-kernel timing: when enabled (hss_timing_enable), every kernel
// launch of the library is bracketed by two HIP events on its stream; the
// report sums the event intervals per kernel name.
#pragma once
#include <hip/hip_runtime.h>

namespace hss {

bool timing_on();
void timing_begin(const char* name, hipStream_t s);
void timing_end(hipStream_t s);

struct TimedLaunch {
  bool on;
  hipStream_t s;
  TimedLaunch(const char* name, hipStream_t st) : on(timing_on()), s(st) {
    if (on) timing_begin(name, s);
  }
  ~TimedLaunch() {
    if (on) timing_end(s);
  }
};

}  // namespace hss
