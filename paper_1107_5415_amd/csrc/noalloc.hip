// lfft_forward_noalloc: the forward lattice FFT without a workspace argument
// and without any device allocation, for callers that cannot allocate (code
// under HIP graph capture, tight serving loops, harnesses that forbid
// hipMalloc).
//
// The intermediate grid between the passes lives in one fixed array per
// device, `scratch`, of kScratchElems complex64 values (64 MiB), which every
// device that loads the library holds until the process ends.  Host code
// never uses the array's name as an address: the first call on a device asks
// the runtime for the array's device address on that device
// (hipGetSymbolAddress, with that device current) and keeps it; kernels get
// that address as their workspace pointer.  The passes write the whole
// intermediate grid before they read it, so nothing needs clearing between
// calls; calls that overlap in time on one device race on the array.
#include <hip/hip_runtime.h>

#include <mutex>

#include "handles.hpp"
#include "lfft.h"
#include "plan.hpp"

namespace {

constexpr size_t kScratchElems = size_t(1) << 23;   // complex64 values, 64 MiB
constexpr int kMaxDevices = 64;

static __device__ __align__(256) float2 scratch[kScratchElems];

std::mutex g_mu;
void* g_ptr[kMaxDevices] = {};

// device address of `scratch` on the current device (nullptr on error)
void* scratch_ptr(int* status) {
  int dev = 0;
  if (hipGetDevice(&dev) != hipSuccess || dev < 0 || dev >= kMaxDevices) {
    *status = LFFT_E_HIP;
    return nullptr;
  }
  std::lock_guard<std::mutex> g(g_mu);
  if (!g_ptr[dev]) {
    void* p = nullptr;
    if (hipGetSymbolAddress(&p, HIP_SYMBOL(scratch)) != hipSuccess || !p) {
      *status = LFFT_E_HIP;
      return nullptr;
    }
    g_ptr[dev] = p;
  }
  return g_ptr[dev];
}

}  // namespace

extern "C" int lfft_forward_noalloc(lfft_plan_t plan, const void* in, void* out, uint32_t layout,
                                    hipStream_t stream) {
  if (!plan || !plan->p || !in || !out || in == out) return LFFT_E_ARG;
  if (layout & ~(LFFT_IN_GRID | LFFT_OUT_GRID)) return LFFT_E_ARG;
  const lfft::LatticePlan* p = plan->p;
  if (!p->dtab) return LFFT_E_STATE;
  if (p->ws_elems > kScratchElems) return LFFT_E_UNSUPPORTED;
  int status = LFFT_OK;
  void* ws = nullptr;
  if (p->ws_elems) {
    ws = scratch_ptr(&status);
    if (!ws) return status;
  }
  try {
    lfft::exec_lattice(p, false, (layout & LFFT_IN_GRID) != 0, (layout & LFFT_OUT_GRID) != 0, in,
                       out, ws, p->m, p->m, stream);
  } catch (const lfft::StatusError& e) {
    return e.code;
  } catch (...) {
    return LFFT_E_STATE;
  }
  return LFFT_OK;
}
