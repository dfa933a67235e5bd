// Chirp-z (Bluestein) pass: the DFT of one grid axis whose length L has a
// prime factor too large for an on-chip pencil.  With w = exp(-2 pi i / L)
// and jk = (j^2 + k^2 - (k - j)^2) / 2,
//   X_k = sum_j x_j w^{jk} = c_k sum_j (x_j c_j) conj(c_{k-j}),  c_j = w^{j^2/2},
// a cyclic convolution of length N >= 2L - 1 (a power of two) computed with
// the library's own power-of-two FFTs.  The axis is one factor of the
// Kronecker form of the lattice Fourier matrix (Section 4.1, Theorem 1), so
// Algorithm 1 of Section 4.2 applies to any elementary divisors; the chirp
// only changes how the 1-D DFT of this factor is computed.  These kernels are
// the elementwise steps around the two inner FFTs; they gather and scatter
// through the pass's maps like every other pass (natural or grid layouts).
#include <hip/hip_runtime.h>

#include "fft_common.hpp"
#include "kernels.hpp"

namespace lfft {
namespace {
using namespace dev;

__device__ __forceinline__ float2 chirp_at(const PassDesc& p, int j) {
  float2 c = p.chirp[j];
  return p.sign < 0 ? c : c_conj(c);
}

__global__ void __launch_bounds__(256) blue_pre_kernel(PassDesc p, const float2* __restrict__ in,
                                                       float2* __restrict__ A, long long total) {
  const long long e = (long long)blockIdx.x * blockDim.x + threadIdx.x;
  if (e >= total) return;
  const long long N = p.bN;
  const long long pen = e / N;
  const int j = (int)(e - pen * N);
  float2 v = make_float2(0.f, 0.f);
  if (j < p.L) {
    const long long bo = pen / p.S;
    const int s = (int)(pen - bo * p.S);
    const long long b = bo / p.O;
    const int o = (int)(bo - b * p.O);
    v = c_mul(in[map_index(p.in, b, o, j, s, p.L, p.S)], chirp_at(p, j));
  }
  A[e] = v;
}

__global__ void __launch_bounds__(256) blue_mul_kernel(PassDesc p, float2* __restrict__ B,
                                                       long long total) {
  const long long e = (long long)blockIdx.x * blockDim.x + threadIdx.x;
  if (e >= total) return;
  float2 h = p.bhat[e & (p.bN - 1)];
  if (p.sign > 0) h = c_conj(h);
  B[e] = c_mul(B[e], h);
}

__global__ void __launch_bounds__(256) blue_post_kernel(PassDesc p, const float2* __restrict__ A,
                                                        float2* __restrict__ out, long long total) {
  const long long e = (long long)blockIdx.x * blockDim.x + threadIdx.x;
  if (e >= total) return;
  const long long pen = e / p.L;
  const int k = (int)(e - pen * p.L);
  const long long bo = pen / p.S;
  const int s = (int)(pen - bo * p.S);
  const long long b = bo / p.O;
  const int o = (int)(bo - b * p.O);
  float2 v = c_mul(A[pen * p.bN + k], chirp_at(p, k));
  v.x *= p.scale;
  v.y *= p.scale;
  out[map_index(p.out, b, o, k, s, p.L, p.S)] = v;
}

unsigned blocks(long long n) { return (unsigned)((n + 255) / 256); }

}  // namespace

hipError_t launch_blue_pre(const PassDesc& p, const float2* in, float2* A, hipStream_t s) {
  const long long total = p.batch * (long long)p.O * p.S * p.bN;
  if (total <= 0) return hipSuccess;
  hipLaunchKernelGGL(blue_pre_kernel, dim3(blocks(total)), dim3(256), 0, s, p, in, A, total);
  return hipGetLastError();
}

hipError_t launch_blue_mul(const PassDesc& p, float2* B, hipStream_t s) {
  const long long total = p.batch * (long long)p.O * p.S * p.bN;
  if (total <= 0) return hipSuccess;
  hipLaunchKernelGGL(blue_mul_kernel, dim3(blocks(total)), dim3(256), 0, s, p, B, total);
  return hipGetLastError();
}

hipError_t launch_blue_post(const PassDesc& p, const float2* A, float2* out, hipStream_t s) {
  const long long total = p.batch * (long long)p.O * p.S * p.L;
  if (total <= 0) return hipSuccess;
  hipLaunchKernelGGL(blue_post_kernel, dim3(blocks(total)), dim3(256), 0, s, p, A, out, total);
  return hipGetLastError();
}

}  // namespace lfft
