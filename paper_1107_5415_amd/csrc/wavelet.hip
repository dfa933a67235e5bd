// Fourier-domain wavelet split for |det J| = 2 (Section 5.3, steps 3-4 with
// the Dirichlet wavelet symbol of Section 6.2), its inverse and the mask
// gradients, all in natural order.
//
// One thread owns one fiber {h0, h0 + s} of G(M^T) over k in G(N^T)
// (eq. decomposition applied to G(M^T)): h0 is k reduced into the Hermite box
// of M^T, s = N^T g0.  With a0 = a(h0), a1 = a(h0 + s) and
// phi0 = exp(-2 pi i h0^T M^{-1} v), v = J y0:
//   d1 = (a0 x0 + a1 x1)/sqrt2,   d2 = conj(phi0) (a1 x0 - a0 x1)/sqrt2.
// The batch loop runs inside the thread, so the index arithmetic is paid once
// per fiber and the mask gradient needs no atomics: each mask entry has
// exactly one writer.
#include <hip/hip_runtime.h>

#include "fft_common.hpp"
#include "kernels.hpp"

namespace lfft {
namespace {

constexpr float kInvSqrt2 = 0.70710678118654752440f;

__device__ __forceinline__ float2 cmul(float2 a, float2 b) {
  return make_float2(a.x * b.x - a.y * b.y, a.x * b.y + a.y * b.x);
}
__device__ __forceinline__ float2 cconj(float2 a) { return make_float2(a.x, -a.y); }
__device__ __forceinline__ float2 axpby(float a, float2 x, float b, float2 y) {
  return make_float2(a * x.x + b * y.x, a * x.y + b * y.y);
}
__device__ __forceinline__ float2 scale(float2 a, float s) { return make_float2(a.x * s, a.y * s); }

struct Fiber {
  long long i0, i1;   // natural indices of h0 and h0 + s in G(M^T)
  float2 phi;         // phi(h0)
};

__device__ __forceinline__ long long floordiv_ll(long long a, long long b) {
  long long q = a / b;
  if ((a % b != 0) && ((a < 0) != (b < 0))) --q;
  return q;
}

__device__ __forceinline__ void reduce_hm(const SplitDesc& sd, long long* v) {
  for (int i = sd.d - 1; i >= 0; --i) {
    long long q = floordiv_ll(v[i], sd.HM[i][i]);
    if (q)
      for (int r = 0; r <= i; ++r) v[r] -= q * sd.HM[r][i];
  }
}

__device__ __forceinline__ Fiber fiber_of(const SplitDesc& sd, long long klin) {
  long long k[4] = {0, 0, 0, 0};
  long long r = klin;
  for (int i = sd.d - 1; i >= 0; --i) {
    k[i] = r % sd.KN[i];
    r /= sd.KN[i];
  }
  long long h0[4] = {k[0], k[1], k[2], k[3]};
  reduce_hm(sd, h0);
  long long h1[4] = {h0[0] + sd.s[0], h0[1] + sd.s[1], h0[2] + sd.s[2], h0[3] + sd.s[3]};
  reduce_hm(sd, h1);
  Fiber f;
  f.i0 = 0;
  f.i1 = 0;
  long long rho = 0;
  for (int i = 0; i < sd.d; ++i) {
    f.i0 += h0[i] * sd.hstride[i];
    f.i1 += h1[i] * sd.hstride[i];
    rho = (rho + (h0[i] % sd.E) * (long long)sd.w[i]) % sd.E;
  }
  f.phi = sd.tw[rho];
  return f;
}

// 32-bit fiber maps (sd.narrow): the same arithmetic with invariant-divisor
// multiplications instead of 64-bit divisions.
__device__ __forceinline__ void reduce_hm32(const SplitDesc& sd, int* v) {
#pragma unroll
  for (int i = 3; i >= 0; --i) {
    if (i < sd.d) {
      // floor(v / h) for |v| < 2^30 (bounded on the host)
      const int h = sd.HM[i][i];
      const int x = v[i];
      const int q = x >= 0 ? (int)fast_div((unsigned)x, sd.fHM[i])
                           : -(int)fast_div((unsigned)(h - 1 - x), sd.fHM[i]);
#pragma unroll
      for (int r = 0; r <= i; ++r) v[r] -= q * sd.HM[r][i];
    }
  }
}

__device__ __forceinline__ Fiber fiber_of32(const SplitDesc& sd, long long klin) {
  int k[4] = {0, 0, 0, 0};
  unsigned r = (unsigned)klin;
#pragma unroll
  for (int i = 3; i >= 0; --i) {
    if (i < sd.d) {
      const unsigned q = fast_div(r, sd.fKN[i]);
      k[i] = (int)(r - q * (unsigned)sd.KN[i]);
      r = q;
    }
  }
  int h0[4] = {k[0], k[1], k[2], k[3]};
  reduce_hm32(sd, h0);
  int h1[4] = {h0[0] + sd.s[0], h0[1] + sd.s[1], h0[2] + sd.s[2], h0[3] + sd.s[3]};
  reduce_hm32(sd, h1);
  int i0 = 0, i1 = 0, acc = 0;
#pragma unroll
  for (int i = 0; i < 4; ++i) {
    if (i < sd.d) {
      i0 += h0[i] * (int)sd.hstride[i];
      i1 += h1[i] * (int)sd.hstride[i];
      acc += h0[i] * sd.w[i];
    }
  }
  const unsigned q = fast_div((unsigned)acc, sd.fE);
  Fiber f;
  f.i0 = i0;
  f.i1 = i1;
  f.phi = sd.tw[(unsigned)acc - q * (unsigned)sd.E];
  return f;
}

__device__ __forceinline__ Fiber fiber_at(const SplitDesc& sd, long long k) {
  return sd.narrow ? fiber_of32(sd, k) : fiber_of(sd, k);
}

__global__ void split_kernel(SplitDesc sd, long long batch, const float2* __restrict__ ah,
                             long long ah_bs, const float* __restrict__ mask, float2* __restrict__ d1,
                             float2* __restrict__ d2, long long d_bs) {
  long long k = lfft::dev::xcd_tile(blockIdx.x, gridDim.x) * blockDim.x + threadIdx.x;
  if (k >= sd.mN) return;
  Fiber f = fiber_at(sd, k);
  const float a0 = mask[f.i0] * kInvSqrt2, a1 = mask[f.i1] * kInvSqrt2;
  const float2 cphi = cconj(f.phi);
  for (long long b = 0; b < batch; ++b) {
    float2 x0 = ah[b * ah_bs + f.i0];
    float2 x1 = ah[b * ah_bs + f.i1];
    d1[b * d_bs + k] = axpby(a0, x0, a1, x1);
    d2[b * d_bs + k] = cmul(cphi, axpby(a1, x0, -a0, x1));
  }
}

__global__ void unsplit_kernel(SplitDesc sd, long long batch, const float2* __restrict__ d1,
                               const float2* __restrict__ d2, long long d_bs,
                               const float* __restrict__ mask, float2* __restrict__ ah,
                               long long ah_bs) {
  long long k = lfft::dev::xcd_tile(blockIdx.x, gridDim.x) * blockDim.x + threadIdx.x;
  if (k >= sd.mN) return;
  Fiber f = fiber_at(sd, k);
  const float a0 = mask[f.i0] * kInvSqrt2, a1 = mask[f.i1] * kInvSqrt2;
  for (long long b = 0; b < batch; ++b) {
    float2 y1 = d1[b * d_bs + k];
    float2 y2 = cmul(f.phi, d2[b * d_bs + k]);
    ah[b * ah_bs + f.i0] = axpby(a0, y1, a1, y2);
    ah[b * ah_bs + f.i1] = axpby(a1, y1, -a0, y2);
  }
}

// Re(conj(g) * x)
__device__ __forceinline__ float re_dot(float2 g, float2 x) { return g.x * x.x + g.y * x.y; }

__global__ void split_mask_grad_kernel(SplitDesc sd, long long batch, const float2* __restrict__ ah,
                                       long long ah_bs, const float2* __restrict__ g1,
                                       const float2* __restrict__ g2, long long g_bs,
                                       float* __restrict__ gmask) {
  long long k = lfft::dev::xcd_tile(blockIdx.x, gridDim.x) * blockDim.x + threadIdx.x;
  if (k >= sd.mN) return;
  Fiber f = fiber_at(sd, k);
  const float2 c = cconj(f.phi);
  float s0 = 0.f, s1 = 0.f;
  for (long long b = 0; b < batch; ++b) {
    float2 x0 = ah[b * ah_bs + f.i0];
    float2 x1 = ah[b * ah_bs + f.i1];
    float2 G1 = g1[b * g_bs + k];
    float2 G2 = g2[b * g_bs + k];
    // d1 = (a0 x0 + a1 x1)/sqrt2, d2 = c (a1 x0 - a0 x1)/sqrt2
    s0 += re_dot(G1, x0) - re_dot(G2, cmul(c, x1));
    s1 += re_dot(G1, x1) + re_dot(G2, cmul(c, x0));
  }
  gmask[f.i0] = s0 * kInvSqrt2;
  gmask[f.i1] = s1 * kInvSqrt2;
}

__global__ void unsplit_mask_grad_kernel(SplitDesc sd, long long batch, const float2* __restrict__ d1,
                                         const float2* __restrict__ d2, long long d_bs,
                                         const float2* __restrict__ g, long long g_bs,
                                         float* __restrict__ gmask) {
  long long k = lfft::dev::xcd_tile(blockIdx.x, gridDim.x) * blockDim.x + threadIdx.x;
  if (k >= sd.mN) return;
  Fiber f = fiber_at(sd, k);
  float s0 = 0.f, s1 = 0.f;
  for (long long b = 0; b < batch; ++b) {
    float2 y1 = d1[b * d_bs + k];
    float2 y2 = cmul(f.phi, d2[b * d_bs + k]);
    float2 G0 = g[b * g_bs + f.i0];
    float2 G1 = g[b * g_bs + f.i1];
    // ah0 = (a0 y1 + a1 y2)/sqrt2, ah1 = (a1 y1 - a0 y2)/sqrt2
    s0 += re_dot(G0, y1) - re_dot(G1, y2);
    s1 += re_dot(G0, y2) + re_dot(G1, y1);
  }
  gmask[f.i0] = s0 * kInvSqrt2;
  gmask[f.i1] = s1 * kInvSqrt2;
}

inline unsigned blocks_for(long long n, int bs) { return (unsigned)((n + bs - 1) / bs); }

}  // namespace

hipError_t launch_split(const SplitDesc& sd, long long batch, const float2* ah, long long ah_bs,
                        const float* mask, float2* d1, float2* d2, long long d_bs, hipStream_t s) {
  hipLaunchKernelGGL(split_kernel, dim3(blocks_for(sd.mN, 256)), dim3(256), 0, s, sd, batch, ah,
                     ah_bs, mask, d1, d2, d_bs);
  return hipGetLastError();
}

hipError_t launch_unsplit(const SplitDesc& sd, long long batch, const float2* d1, const float2* d2,
                          long long d_bs, const float* mask, float2* ah, long long ah_bs,
                          hipStream_t s) {
  hipLaunchKernelGGL(unsplit_kernel, dim3(blocks_for(sd.mN, 256)), dim3(256), 0, s, sd, batch, d1,
                     d2, d_bs, mask, ah, ah_bs);
  return hipGetLastError();
}

hipError_t launch_split_mask_grad(const SplitDesc& sd, long long batch, const float2* ah,
                                  long long ah_bs, const float2* g1, const float2* g2,
                                  long long g_bs, float* gmask, hipStream_t s) {
  hipLaunchKernelGGL(split_mask_grad_kernel, dim3(blocks_for(sd.mN, 256)), dim3(256), 0, s, sd,
                     batch, ah, ah_bs, g1, g2, g_bs, gmask);
  return hipGetLastError();
}

hipError_t launch_unsplit_mask_grad(const SplitDesc& sd, long long batch, const float2* d1,
                                    const float2* d2, long long d_bs, const float2* g,
                                    long long g_bs, float* gmask, hipStream_t s) {
  hipLaunchKernelGGL(unsplit_mask_grad_kernel, dim3(blocks_for(sd.mN, 256)), dim3(256), 0, s, sd,
                     batch, d1, d2, d_bs, g, g_bs, gmask);
  return hipGetLastError();
}

}  // namespace lfft
