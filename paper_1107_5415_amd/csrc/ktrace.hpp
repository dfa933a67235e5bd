// Per-launch kernel timing (process-wide, off by default).  When enabled,
// every kernel this library launches is bracketed by two HIP events recorded
// on its own stream, together with the kernel's name and the algorithmic
// bytes of that launch (the minimum the operation must move to/from HBM).
#pragma once
#include <hip/hip_runtime.h>

namespace lfft {

bool trace_on();
// Stable storage for a formatted kernel name (deduplicated, never freed).
const char* kernel_name_intern(const char* fmt, ...);
// Returns a slot index for a launch about to be enqueued on `s`, or -1.
int trace_begin(const char* kernel, double bytes, hipStream_t s);
void trace_end(int slot, hipStream_t s);

struct TraceScope {
  int slot;
  hipStream_t s;
  TraceScope(const char* kernel, double bytes, hipStream_t st) : slot(-1), s(st) {
    if (trace_on()) slot = trace_begin(kernel, bytes, s);
  }
  ~TraceScope() {
    if (slot >= 0) trace_end(slot, s);
  }
};

}  // namespace lfft
