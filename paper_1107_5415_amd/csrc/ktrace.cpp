// Per-launch kernel timing; see ktrace.hpp and the lfft_trace_* entry points.
#include "ktrace.hpp"

#include <cstdarg>
#include <cstdio>
#include <mutex>
#include <set>
#include <string>
#include <vector>

#include "lfft.h"

namespace lfft {
namespace {
struct Rec {
  const char* name;
  double bytes, pass_bytes;
  hipEvent_t a, b;
};
struct State {
  std::mutex mu;
  bool on = false;
  std::vector<Rec> recs;
  size_t used = 0;
};
State& st() {
  static State s;
  return s;
}
}  // namespace

bool trace_on() { return st().on; }

const char* kernel_name_intern(const char* fmt, ...) {
  static std::mutex mu;
  static std::set<std::string> names;
  char buf[256];
  va_list ap;
  va_start(ap, fmt);
  vsnprintf(buf, sizeof buf, fmt, ap);
  va_end(ap);
  std::lock_guard<std::mutex> g(mu);
  return names.insert(buf).first->c_str();
}

int trace_begin(const char* kernel, double bytes, double pass_bytes, hipStream_t s) {
  State& S = st();
  std::lock_guard<std::mutex> g(S.mu);
  if (!S.on || S.used >= S.recs.size()) return -1;
  int i = (int)S.used++;
  S.recs[i].name = kernel;
  S.recs[i].bytes = bytes;
  S.recs[i].pass_bytes = pass_bytes;
  if (hipEventRecord(S.recs[i].a, s) != hipSuccess) return -1;
  return i;
}

void trace_end(int slot, hipStream_t s) {
  State& S = st();
  (void)hipEventRecord(S.recs[slot].b, s);
}

}  // namespace lfft

extern "C" {

int lfft_trace_begin(int capacity) {
  using namespace lfft;
  if (capacity <= 0) return LFFT_E_ARG;
  State& S = st();
  std::lock_guard<std::mutex> g(S.mu);
  if ((int)S.recs.size() < capacity) {
    size_t old = S.recs.size();
    S.recs.resize(capacity);
    for (size_t i = old; i < S.recs.size(); ++i) {
      if (hipEventCreate(&S.recs[i].a) != hipSuccess) return LFFT_E_HIP;
      if (hipEventCreate(&S.recs[i].b) != hipSuccess) return LFFT_E_HIP;
    }
  }
  S.used = 0;
  S.on = true;
  return LFFT_OK;
}

int lfft_trace_end(int* count) {
  using namespace lfft;
  State& S = st();
  std::lock_guard<std::mutex> g(S.mu);
  S.on = false;
  if (count) *count = (int)S.used;
  return LFFT_OK;
}

int lfft_trace_get(int i, const char** name, double* bytes, double* pass_bytes, float* ms) {
  using namespace lfft;
  State& S = st();
  std::lock_guard<std::mutex> g(S.mu);
  if (i < 0 || (size_t)i >= S.used) return LFFT_E_ARG;
  if (name) *name = S.recs[i].name;
  if (bytes) *bytes = S.recs[i].bytes;
  if (pass_bytes) *pass_bytes = S.recs[i].pass_bytes;
  if (ms) {
    if (hipEventSynchronize(S.recs[i].b) != hipSuccess) return LFFT_E_HIP;
    if (hipEventElapsedTime(ms, S.recs[i].a, S.recs[i].b) != hipSuccess) return LFFT_E_HIP;
  }
  return LFFT_OK;
}

}  // extern "C"
