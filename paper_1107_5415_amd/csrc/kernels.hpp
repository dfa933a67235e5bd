// Kernel launchers (gfx950).  Every launcher only enqueues work on the given
// stream and returns the launch status.
#pragma once
#include <hip/hip_runtime.h>

#include "device.hpp"

namespace lfft {

// One FFT pass (gather -> Stockham stages -> optional four-step twiddle ->
// scatter) over every tile of the batch.
hipError_t launch_pass(const PassDesc& p, const float2* in, float2* out, hipStream_t s);
// Name of the kernel launch_pass uses for this descriptor (for tracing).
const char* pass_kernel_name(const PassDesc& p);
// Register-resident power-of-two pass (descriptor kind 1).
hipError_t launch_fast_pass(const PassDesc& p, const float2* in, float2* out, hipStream_t s);
const char* fast_kernel_name(const PassDesc& p);
// Persistent double-buffered pass for single-digit power-of-two pencils
// (descriptor kind 2) and the (L, W) shapes it is compiled for.
hipError_t launch_stream_pass(const PassDesc& p, const float2* in, float2* out, hipStream_t s);
bool stream_supported(int L, int W, bool cols);
const char* stream_kernel_name(const PassDesc& p);

// Fourier-domain wavelet split of one level (Section 5.3, step 4).
hipError_t launch_split(const SplitDesc& sd, long long batch, const float2* ahat, long long ah_bs,
                        const float* mask, float2* d1, float2* d2, long long d_bs, hipStream_t s);
// Its inverse (synthesis).
hipError_t launch_unsplit(const SplitDesc& sd, long long batch, const float2* d1, const float2* d2,
                          long long d_bs, const float* mask, float2* ahat, long long ah_bs,
                          hipStream_t s);
// d loss / d mask of the split, summed over the batch.
hipError_t launch_split_mask_grad(const SplitDesc& sd, long long batch, const float2* ahat,
                                  long long ah_bs, const float2* g1, const float2* g2,
                                  long long g_bs, float* gmask, hipStream_t s);
// d loss / d mask of the unsplit, summed over the batch.
hipError_t launch_unsplit_mask_grad(const SplitDesc& sd, long long batch, const float2* d1,
                                    const float2* d2, long long d_bs, const float2* g,
                                    long long g_bs, float* gmask, hipStream_t s);

}  // namespace lfft
