// One-launch-per-pass driver of the register-resident power-of-two FFT pass
// (device body in fast_tile.hpp).
//
// Each thread keeps P complex values in VGPRs for the whole pass; a
// workgroup owns W pencils: W consecutive columns (inner index s) when the
// pencil axis is strided, so the HBM accesses of a wavefront are W*8-byte
// contiguous segments, or W consecutive rows when the pencils are contiguous.
//
// The first pass gathers from the natural sample order and the last pass
// scatters to the natural frequency order with the Hermite-box group
// arithmetic of the planner's tables (Section 3 bases, Theorem 1 of
// Section 4.1); a thread's R inputs of one butterfly are an arithmetic
// progression in one digit, so their natural coordinates follow by repeated
// group addition of one constant.
#include <hip/hip_runtime.h>

#include <atomic>

#include "fast_tile.hpp"
#include "kernels.hpp"
#include "ktrace.hpp"

namespace lfft {
namespace {
using namespace dev;

template <int P, bool COLS, bool SPLIT, int MIN, int MOUT>
__global__ void __launch_bounds__(1024) fft_fast_kernel(PassDesc p, const float2* __restrict__ in,
                                                        float2* __restrict__ out) {
  extern __shared__ float2 lds_raw[];
  fastk::fast_tile<P, COLS, SPLIT, MIN, MOUT>(p, xcd_tile(blockIdx.x, gridDim.x), threadIdx.x, in,
                                              out, lds_raw);
}

template <int P, bool COLS, bool SPLIT, int MIN, int MOUT>
hipError_t launch_t(const PassDesc& p, const float2* in, float2* out, hipStream_t s) {
  auto k = fft_fast_kernel<P, COLS, SPLIT, MIN, MOUT>;
  // set once; threads that race here all write the same attribute
  static std::atomic<bool> attr{false};
  if (!attr.load(std::memory_order_acquire)) {
    hipError_t e = hipFuncSetAttribute((const void*)k, hipFuncAttributeMaxDynamicSharedMemorySize,
                                       160 * 1024);
    if (e != hipSuccess) return e;
    attr.store(true, std::memory_order_release);
  }
  const long long npen = p.batch * (long long)p.O * p.S;
  const long long tiles = (npen + p.W - 1) / p.W;
  const int nt = p.W * (p.L / P);
  const int tile = p.W * p.L;
  const size_t lds = (size_t)(tile + tile / 16 + 1) * (SPLIT ? sizeof(float) : sizeof(float2));
  hipLaunchKernelGGL(k, dim3((unsigned)tiles), dim3(nt), lds, s, p, in, out);
  return hipGetLastError();
}

template <int P, bool COLS, bool SPLIT, int MIN>
hipError_t launch_out(const PassDesc& p, const float2* in, float2* out, hipStream_t s) {
  switch (p.out.mode) {
    case MAP_IDENTITY: return launch_t<P, COLS, SPLIT, MIN, MAP_IDENTITY>(p, in, out, s);
    case MAP_LINEAR: return launch_t<P, COLS, SPLIT, MIN, MAP_LINEAR>(p, in, out, s);
    default: return launch_t<P, COLS, SPLIT, MIN, MAP_NATURAL>(p, in, out, s);
  }
}

template <int P, bool COLS, bool SPLIT>
hipError_t launch_in(const PassDesc& p, const float2* in, float2* out, hipStream_t s) {
  if (p.in.mode == MAP_NATURAL) return launch_out<P, COLS, SPLIT, MAP_NATURAL>(p, in, out, s);
  return launch_out<P, COLS, SPLIT, MAP_IDENTITY>(p, in, out, s);
}

}  // namespace

const char* fast_kernel_name(const PassDesc& p) {
  const int min = p.in.mode == MAP_NATURAL ? 2 : 0;
  return kernel_name_intern("fft_fast_kernel<16, %s, %s, %d, %d>", p.S > 1 ? "true" : "false",
                            p.split ? "true" : "false", min, p.out.mode);
}

hipError_t launch_fast_pass(const PassDesc& p, const float2* in, float2* out, hipStream_t s) {
  if (p.P != 16) return hipErrorInvalidValue;
  if (p.S > 1) return p.split ? launch_in<16, true, true>(p, in, out, s) : launch_in<16, true, false>(p, in, out, s);
  return p.split ? launch_in<16, false, true>(p, in, out, s) : launch_in<16, false, false>(p, in, out, s);
}

}  // namespace lfft
