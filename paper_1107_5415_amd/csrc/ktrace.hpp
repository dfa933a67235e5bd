// Per-launch kernel timing (process-wide, off by default).  When enabled,
// every kernel this library launches is bracketed by two HIP events recorded
// on its own stream, together with the kernel's name and two byte counts:
//  - method bytes: the launch's share of the minimum the operation must move
//    to/from HBM (an FFT moves 16 B per complex point once, read and write,
//    however many passes it takes, so each of its np passes is credited
//    16 B / np per point; a split level 20 B per point);
//  - pass bytes: what the launch itself must move at least (16 B per point
//    for every FFT pass; equal to the method bytes for other kernels).
#pragma once
#include <hip/hip_runtime.h>

namespace lfft {

bool trace_on();
// Stable storage for a formatted kernel name (deduplicated, never freed).
const char* kernel_name_intern(const char* fmt, ...);
// Returns a slot index for a launch about to be enqueued on `s`, or -1.
int trace_begin(const char* kernel, double bytes, double pass_bytes, hipStream_t s);
void trace_end(int slot, hipStream_t s);

struct TraceScope {
  int slot;
  hipStream_t s;
  TraceScope(const char* kernel, double bytes, hipStream_t st) : slot(-1), s(st) {
    if (trace_on()) slot = trace_begin(kernel, bytes, bytes, s);
  }
  TraceScope(const char* kernel, double bytes, double pass_bytes, hipStream_t st)
      : slot(-1), s(st) {
    if (trace_on()) slot = trace_begin(kernel, bytes, pass_bytes, s);
  }
  ~TraceScope() {
    if (slot >= 0) trace_end(slot, s);
  }
};

}  // namespace lfft
