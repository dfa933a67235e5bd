// Device execution of the multi-level wavelet pyramid and its adjoints.
#pragma once
#include "plan.hpp"

namespace lfft {

size_t wave_saved_elems(const WavePlan* w);
void wave_decompose(const WavePlan* w, const float2* x, const float* const* masks, float2* coeffs,
                    float2* saved, void* ws, hipStream_t s);
void wave_reconstruct(const WavePlan* w, const float2* coeffs, const float* const* masks,
                      float2* x, float2* saved, void* ws, hipStream_t s);
void wave_decompose_backward(const WavePlan* w, const float2* gc, const float2* saved,
                             const float* const* masks, float2* gx, float* const* gmasks, void* ws,
                             hipStream_t s);
void wave_reconstruct_backward(const WavePlan* w, const float2* gx, const float2* saved,
                               const float* const* masks, float2* gc, float* const* gmasks,
                               void* ws, hipStream_t s);

}  // namespace lfft
