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
// Split-BF16 MFMA pass (descriptor kind 3): tiles of W * L = 4096 elements.
hipError_t launch_mfma_pass(const PassDesc& p, const float2* in, float2* out, hipStream_t s);
const char* mfma_kernel_name(const PassDesc& p);

// One phase of the batched persistent launch (tile_lg 11..13: tiles of
// 2^tile_lg elements, 2^tile_lg / 16 threads per workgroup).  qbeg[0..8]
// bounds the eight queues of the phase in `items`; the heads
// heads[kHeadStride * q], q < 8, must be zero (launch_batch_clear) before the
// launch.
constexpr int kHeadStride = 32;
hipError_t launch_batch(int tile_lg, const BatchPass* passes, const int2* items, const int* qbeg,
                        int* heads, const float2* in, float2* out, float2* ws, int grid,
                        hipStream_t s);
hipError_t launch_batch_clear(int* heads, int n, hipStream_t s);
size_t batch_lds_bytes(int tile);
int batch_occupancy(int tile_lg);        // resident workgroups per CU (0 on error)
const char* batch_kernel_name(int tile_lg);

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

// Levels l .. l+K-1 (2 <= K <= kMaxChain, every level narrow) of the q = 2
// split in one launch: ahat [B][m_l] -> d2 of every level (c.d2) and the
// low-pass d1 of level l+K-1 [B][m_{l+K-1}/2]; and the inverse.
hipError_t launch_split_chain(int K, const SplitChain& c, long long batch, const float2* ahat,
                              long long ah_bs, float2* d1, long long d1_bs, hipStream_t s);
hipError_t launch_unsplit_chain(int K, const SplitChain& c, long long batch, const float2* d1,
                                long long d1_bs, float2* ahat, long long ah_bs, hipStream_t s);

// q-channel split of one level, q = |det J| > 2: ahat [B][m_l] (batch stride
// ah_bs) -> channel 0 into d0 [B][m_l/q] (stride d0_bs) and channels
// 1 .. q-1 into dw [B][q-1][m_l/q] (batch stride dw_bs, channel stride m_l/q).
hipError_t launch_split_q(const SplitQDesc& sd, long long batch, const float2* ahat, long long ah_bs,
                          const float* mask, float2* d0, long long d0_bs, float2* dw,
                          long long dw_bs, hipStream_t s);
// Its inverse (synthesis), same layouts.
hipError_t launch_unsplit_q(const SplitQDesc& sd, long long batch, const float2* d0,
                            long long d0_bs, const float2* dw, long long dw_bs, const float* mask,
                            float2* ahat, long long ah_bs, hipStream_t s);

// d loss / d mask of the q-channel split (x = ahat [B][m_l], incoming
// gradients g0 of channel 0 [B][m_l/q] and gw of channels 1 .. q-1, layouts
// as in launch_split_q) and of its synthesis (saved inputs d0, dw as in
// launch_unsplit_q, incoming gradient g of ahat [B][m_l]); summed over the
// batch, one writer per mask entry.
hipError_t launch_split_q_mask_grad(const SplitQDesc& sd, long long batch, const float2* ahat,
                                    long long ah_bs, const float* mask, const float2* g0,
                                    long long g0_bs, const float2* gw, long long gw_bs,
                                    float* gmask, hipStream_t s);
hipError_t launch_unsplit_q_mask_grad(const SplitQDesc& sd, long long batch, const float2* d0,
                                      long long d0_bs, const float2* dw, long long dw_bs,
                                      const float* mask, const float2* g, long long g_bs,
                                      float* gmask, hipStream_t s);

// Chirp-z pass (kind 4), three steps around the inner FFTs of length p.bN:
// A[pen][j] = x(pen, j) chirp[j] for j < L, 0 up to bN (gather through p.in);
// B[pen][k] *= bhat[k]; out(pen, k) = A[pen][k] chirp[k] scale (scatter
// through p.out).  npen = batch * O * S pencils.
hipError_t launch_blue_pre(const PassDesc& p, const float2* in, float2* A, hipStream_t s);
hipError_t launch_blue_mul(const PassDesc& p, float2* B, hipStream_t s);
hipError_t launch_blue_post(const PassDesc& p, const float2* A, float2* out, hipStream_t s);

// data[b * bstride + idx[i]] *= fac[r[i]] for every listed class i < n and
// signal b < batch (the Dirichlet kernel's boundary classes, Section 6.2).
hipError_t launch_boundary_scale(const long long* idx, const int* r, long long n, const float* fac,
                                 float2* data, long long batch, long long bstride, hipStream_t s);

}  // namespace lfft
