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
//
// For q = |det J| > 2 (split_q_kernel / unsplit_q_kernel) a thread owns the
// q-point fiber {k + N^T g_l} and applies the orthogonal q x q channel matrix
// built from the scaling mask (first row a / sqrt q, the other rows from a
// Householder reflection).
#include <hip/hip_runtime.h>

#include "fft_common.hpp"
#include "fiber.hpp"
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

__device__ __forceinline__ Fiber with_phase(const SplitDesc& sd, const fib::FiberIdx& x) {
  Fiber f;
  f.i0 = x.i0;
  f.i1 = x.i1;
  f.phi = sd.tw[x.rho];
  return f;
}

__device__ __forceinline__ Fiber fiber_of32(const SplitDesc& sd, long long klin) {
  return with_phase(sd, fib::fiber_index32(sd, klin));
}

__device__ __forceinline__ Fiber fiber_at(const SplitDesc& sd, long long k) {
  return with_phase(sd, sd.narrow ? fib::fiber_index32(sd, k) : fib::fiber_index64(sd, k));
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

// ---------------------------------------------------------------------------
// K consecutive levels of the q = 2 split in one launch.  The fibers form a
// binary tree in heap order: node 0 is the fiber of the coarsest level at
// k = t, and the children of node n (2n+1 and 2n+2) are the fibers of the
// next finer level whose outputs k are node n's inputs i0 and i1 (G(M_{j+1}^T)
// and G(N_j^T) are the same group in the same natural order).  Every node
// does exactly the arithmetic of split_kernel / unsplit_kernel, so the chain
// gives the same bits as K single-level launches.
__host__ __device__ constexpr int node_depth(int n) {
  return n == 0 ? 0 : 1 + node_depth((n - 1) / 2);
}

template <int K>
__global__ void __launch_bounds__(256) split_chain_kernel(SplitChain c, long long batch,
                                                          const float2* __restrict__ ah,
                                                          long long ah_bs, float2* __restrict__ d1,
                                                          long long d1_bs) {
  constexpr int NF = (1 << K) - 1;
  constexpr int LEAF0 = (1 << (K - 1)) - 1;   // first node of the finest level
  const long long t = lfft::dev::xcd_tile(blockIdx.x, gridDim.x) * blockDim.x + threadIdx.x;
  if (t >= c.sd[K - 1].mN) return;
  int kk[NF], i0[NF], i1[NF];
  float2 cphi[NF];
  float a0[NF], a1[NF];
  kk[0] = (int)t;
#pragma unroll
  for (int n = 0; n < NF; ++n) {
    const int j = K - 1 - node_depth(n);
    const Fiber f = fiber_of32(c.sd[j], kk[n]);
    i0[n] = (int)f.i0;
    i1[n] = (int)f.i1;
    cphi[n] = cconj(f.phi);
    if (n < LEAF0) {
      kk[2 * n + 1] = i0[n];
      kk[2 * n + 2] = i1[n];
    }
    a0[n] = c.mask[j][i0[n]] * kInvSqrt2;
    a1[n] = c.mask[j][i1[n]] * kInvSqrt2;
  }
  for (long long b = 0; b < batch; ++b) {
    float2 x0[NF - LEAF0], x1[NF - LEAF0];
#pragma unroll
    for (int n = LEAF0; n < NF; ++n) {
      // the finest input is dead once read
      x0[n - LEAF0] = lfft::dev::load_stream(&ah[b * ah_bs + i0[n]]);
      x1[n - LEAF0] = lfft::dev::load_stream(&ah[b * ah_bs + i1[n]]);
    }
    float2 lo[NF];
#pragma unroll
    for (int n = NF - 1; n >= 0; --n) {
      const int j = K - 1 - node_depth(n);
      const float2 u = n >= LEAF0 ? x0[n - LEAF0] : lo[2 * n + 1];
      const float2 v = n >= LEAF0 ? x1[n - LEAF0] : lo[2 * n + 2];
      lo[n] = axpby(a0[n], u, a1[n], v);
      c.d2[j][b * c.d2_bs[j] + kk[n]] = cmul(cphi[n], axpby(a1[n], u, -a0[n], v));
    }
    d1[b * d1_bs + t] = lo[0];
  }
}

template <int K>
__global__ void __launch_bounds__(256) unsplit_chain_kernel(SplitChain c, long long batch,
                                                            const float2* __restrict__ d1,
                                                            long long d1_bs,
                                                            float2* __restrict__ ah,
                                                            long long ah_bs) {
  constexpr int NF = (1 << K) - 1;
  constexpr int LEAF0 = (1 << (K - 1)) - 1;
  const long long t = lfft::dev::xcd_tile(blockIdx.x, gridDim.x) * blockDim.x + threadIdx.x;
  if (t >= c.sd[K - 1].mN) return;
  int kk[NF], i0[NF], i1[NF];
  float2 phi[NF];
  float a0[NF], a1[NF];
  kk[0] = (int)t;
#pragma unroll
  for (int n = 0; n < NF; ++n) {
    const int j = K - 1 - node_depth(n);
    const Fiber f = fiber_of32(c.sd[j], kk[n]);
    i0[n] = (int)f.i0;
    i1[n] = (int)f.i1;
    phi[n] = f.phi;
    if (n < LEAF0) {
      kk[2 * n + 1] = i0[n];
      kk[2 * n + 2] = i1[n];
    }
    a0[n] = c.mask[j][i0[n]] * kInvSqrt2;
    a1[n] = c.mask[j][i1[n]] * kInvSqrt2;
  }
  for (long long b = 0; b < batch; ++b) {
    float2 y2[NF];
#pragma unroll
    for (int n = 0; n < NF; ++n) {
      const int j = K - 1 - node_depth(n);
      // the channels and the coarsest low-pass are dead once read
      y2[n] = lfft::dev::load_stream(&c.d2[j][b * c.d2_bs[j] + kk[n]]);
    }
    float2 lo[NF];
    lo[0] = lfft::dev::load_stream(&d1[b * d1_bs + t]);
#pragma unroll
    for (int n = 0; n < NF; ++n) {
      const float2 y1 = lo[n];
      const float2 w = cmul(phi[n], y2[n]);
      const float2 o0 = axpby(a0[n], y1, a1[n], w);
      const float2 o1 = axpby(a1[n], y1, -a0[n], w);
      if (n < LEAF0) {
        lo[2 * n + 1] = o0;
        lo[2 * n + 2] = o1;
      } else {
        ah[b * ah_bs + i0[n]] = o0;
        ah[b * ah_bs + i1[n]] = o1;
      }
    }
  }
}

// ---------------------------------------------------------------------------
// q-channel split, q = |det J| > 2 (Section 5.3 step 4 for general |det J|).
// Per fiber u_l = a(h_l) / sqrt q; the channel matrix has first row u and the
// other rows from the reflection H = I - c v v^T, v = u + sigma e_0,
// sigma = sign(u_0) (+1 at 0), c = 2 / (v^T v); v^T v >= 1, so c needs no
// guard and the rows lose no accuracy near u = e_0:
//   dhat_0 = sum_l u_l x_l,  t = dhat_0 + sigma x_0,
//   dhat_j = x_j - c u_j t                                (j >= 1)
// and the synthesis (its transpose), with tau = sum_{j>=1} u_j y_j:
//   x_0 = u_0 y_0 - c v_0 tau,  x_l = u_l y_0 + y_l - c u_l tau   (l >= 1).
// Q > 0 fixes q at compile time; Q = 0 reads it from the descriptor.
template <int Q>
__device__ __forceinline__ void fiber_q(const SplitQDesc& sd, long long klin, long long* idx) {
  fib::fiber_q_index<Q>(sd, klin, idx, sd.narrow != 0);
}

// u_l, sigma, v_0 and c of one fiber
template <int Q>
__device__ __forceinline__ void reflector(const SplitQDesc& sd, const float* __restrict__ mask,
                                          const long long* idx, float* u, float& sigma,
                                          float& v0, float& c) {
  constexpr int QM = Q ? Q : kMaxQ;
  const int q = Q ? Q : sd.q;
  float perp = 0.f;
#pragma unroll
  for (int l = 0; l < QM; ++l) {
    if (l < q) {
      u[l] = mask[idx[l]] * sd.rsq;
      if (l) perp += u[l] * u[l];
    }
  }
  sigma = u[0] >= 0.f ? 1.f : -1.f;
  v0 = u[0] + sigma;
  c = 2.f / (v0 * v0 + perp);
}

template <int Q>
__global__ void __launch_bounds__(256) split_q_kernel(SplitQDesc sd, long long batch,
                                                      const float2* __restrict__ ah, long long ah_bs,
                                                      const float* __restrict__ mask,
                                                      float2* __restrict__ d0, long long d0_bs,
                                                      float2* __restrict__ dw, long long dw_bs) {
  constexpr int QM = Q ? Q : kMaxQ;
  const int q = Q ? Q : sd.q;
  const long long k = lfft::dev::xcd_tile(blockIdx.x, gridDim.x) * blockDim.x + threadIdx.x;
  if (k >= sd.mN) return;
  long long idx[QM];
  fiber_q<Q>(sd, k, idx);
  float u[QM], sigma, v0, c;
  reflector<Q>(sd, mask, idx, u, sigma, v0, c);
  for (long long b = 0; b < batch; ++b) {
    float2 x[QM];
#pragma unroll
    for (int l = 0; l < QM; ++l)
      if (l < q) x[l] = lfft::dev::load_stream(&ah[b * ah_bs + idx[l]]);  // dead once read
    float2 y0 = make_float2(0.f, 0.f);
#pragma unroll
    for (int l = 0; l < QM; ++l)
      if (l < q) y0 = axpby(1.f, y0, u[l], x[l]);
    const float2 t = axpby(1.f, y0, sigma, x[0]);
    d0[b * d0_bs + k] = y0;
    float2* o = dw + b * dw_bs + k;
#pragma unroll
    for (int j = 1; j < QM; ++j)
      if (j < q) o[(j - 1) * sd.mN] = axpby(1.f, x[j], -c * u[j], t);
  }
}

template <int Q>
__global__ void __launch_bounds__(256) unsplit_q_kernel(SplitQDesc sd, long long batch,
                                                        const float2* __restrict__ d0,
                                                        long long d0_bs,
                                                        const float2* __restrict__ dw,
                                                        long long dw_bs,
                                                        const float* __restrict__ mask,
                                                        float2* __restrict__ ah, long long ah_bs) {
  constexpr int QM = Q ? Q : kMaxQ;
  const int q = Q ? Q : sd.q;
  const long long k = lfft::dev::xcd_tile(blockIdx.x, gridDim.x) * blockDim.x + threadIdx.x;
  if (k >= sd.mN) return;
  long long idx[QM];
  fiber_q<Q>(sd, k, idx);
  float u[QM], sigma, v0, c;
  reflector<Q>(sd, mask, idx, u, sigma, v0, c);
  for (long long b = 0; b < batch; ++b) {
    float2 y[QM];
    // the channels are dead once read
    y[0] = lfft::dev::load_stream(&d0[b * d0_bs + k]);
    const float2* in = dw + b * dw_bs + k;
#pragma unroll
    for (int j = 1; j < QM; ++j)
      if (j < q) y[j] = lfft::dev::load_stream(&in[(j - 1) * sd.mN]);
    float2 tau = make_float2(0.f, 0.f);
#pragma unroll
    for (int j = 1; j < QM; ++j)
      if (j < q) tau = axpby(1.f, tau, u[j], y[j]);
    float2* o = ah + b * ah_bs;
    o[idx[0]] = axpby(u[0], y[0], -c * v0, tau);
#pragma unroll
    for (int l = 1; l < QM; ++l)
      if (l < q) o[idx[l]] = axpby(1.f, axpby(u[l], y[0], 1.f, y[l]), -c * u[l], tau);
  }
}

// d loss / d mask of the q-channel split and synthesis, summed over the batch
// (one thread per fiber, one writer per mask entry).  Incoming gradients
// follow the convention G = dL/dRe + i dL/dIm, so dL = sum Re(conj(G) dz);
// re(g, z) = Re(conj(g) z).  With u_l = a_l / sqrt q, v_l = u_l + sigma [l = 0],
// c = 2 / v^T v (sigma constant on the fiber, so dc/du_l = -c^2 v_l):
//  split, x -> dhat (G_0 on dhat_0, G_j on dhat_j), t = sum_l v_l x_l,
//  Gs = sum_{j>=1} u_j G_j:
//    dL/du_l = re(G_0, x_l) + c^2 v_l re(Gs, t) - c [l >= 1] re(G_l, t) - c re(Gs, x_l);
//  synthesis, y -> x (G_l on x_l), tau = sum_{j>=1} u_j y_j, T = sum_l v_l G_l:
//    dL/du_l = re(G_l, y_0) + c^2 v_l re(T, tau) - c re(G_l, tau) - c [l >= 1] re(T, y_l);
// and dL/da_l = dL/du_l / sqrt q.
__device__ __forceinline__ float re_of(float2 g, float2 z) { return g.x * z.x + g.y * z.y; }

template <int Q>
__global__ void __launch_bounds__(256) split_q_mask_grad_kernel(
    SplitQDesc sd, long long batch, const float2* __restrict__ ah, long long ah_bs,
    const float* __restrict__ mask, const float2* __restrict__ g0, long long g0_bs,
    const float2* __restrict__ gw, long long gw_bs, float* __restrict__ gmask) {
  constexpr int QM = Q ? Q : kMaxQ;
  const int q = Q ? Q : sd.q;
  const long long k = lfft::dev::xcd_tile(blockIdx.x, gridDim.x) * blockDim.x + threadIdx.x;
  if (k >= sd.mN) return;
  long long idx[QM];
  fiber_q<Q>(sd, k, idx);
  float u[QM], sigma, v0, c;
  reflector<Q>(sd, mask, idx, u, sigma, v0, c);
  float acc[QM];
#pragma unroll
  for (int l = 0; l < QM; ++l) acc[l] = 0.f;
  for (long long b = 0; b < batch; ++b) {
    float2 x[QM], G[QM];
#pragma unroll
    for (int l = 0; l < QM; ++l)
      if (l < q) x[l] = ah[b * ah_bs + idx[l]];
    G[0] = g0[b * g0_bs + k];
    const float2* gin = gw + b * gw_bs + k;
#pragma unroll
    for (int j = 1; j < QM; ++j)
      if (j < q) G[j] = gin[(j - 1) * sd.mN];
    float2 t = make_float2(v0 * x[0].x, v0 * x[0].y);
    float2 Gs = make_float2(0.f, 0.f);
#pragma unroll
    for (int l = 1; l < QM; ++l) {
      if (l < q) {
        t = axpby(1.f, t, u[l], x[l]);
        Gs = axpby(1.f, Gs, u[l], G[l]);
      }
    }
    const float rt = re_of(Gs, t);
#pragma unroll
    for (int l = 0; l < QM; ++l) {
      if (l < q) {
        const float vl = l ? u[l] : v0;
        float d = re_of(G[0], x[l]) + c * c * vl * rt - c * re_of(Gs, x[l]);
        if (l) d -= c * re_of(G[l], t);
        acc[l] += d;
      }
    }
  }
#pragma unroll
  for (int l = 0; l < QM; ++l)
    if (l < q) gmask[idx[l]] = acc[l] * sd.rsq;
}

template <int Q>
__global__ void __launch_bounds__(256) unsplit_q_mask_grad_kernel(
    SplitQDesc sd, long long batch, const float2* __restrict__ d0, long long d0_bs,
    const float2* __restrict__ dw, long long dw_bs, const float* __restrict__ mask,
    const float2* __restrict__ g, long long g_bs, float* __restrict__ gmask) {
  constexpr int QM = Q ? Q : kMaxQ;
  const int q = Q ? Q : sd.q;
  const long long k = lfft::dev::xcd_tile(blockIdx.x, gridDim.x) * blockDim.x + threadIdx.x;
  if (k >= sd.mN) return;
  long long idx[QM];
  fiber_q<Q>(sd, k, idx);
  float u[QM], sigma, v0, c;
  reflector<Q>(sd, mask, idx, u, sigma, v0, c);
  float acc[QM];
#pragma unroll
  for (int l = 0; l < QM; ++l) acc[l] = 0.f;
  for (long long b = 0; b < batch; ++b) {
    float2 y[QM], G[QM];
    y[0] = d0[b * d0_bs + k];
    const float2* in = dw + b * dw_bs + k;
#pragma unroll
    for (int j = 1; j < QM; ++j)
      if (j < q) y[j] = in[(j - 1) * sd.mN];
#pragma unroll
    for (int l = 0; l < QM; ++l)
      if (l < q) G[l] = g[b * g_bs + idx[l]];
    float2 tau = make_float2(0.f, 0.f);
    float2 T = make_float2(v0 * G[0].x, v0 * G[0].y);
#pragma unroll
    for (int l = 1; l < QM; ++l) {
      if (l < q) {
        tau = axpby(1.f, tau, u[l], y[l]);
        T = axpby(1.f, T, u[l], G[l]);
      }
    }
    const float rt = re_of(T, tau);
#pragma unroll
    for (int l = 0; l < QM; ++l) {
      if (l < q) {
        const float vl = l ? u[l] : v0;
        float d = re_of(G[l], y[0]) + c * c * vl * rt - c * re_of(G[l], tau);
        if (l) d -= c * re_of(T, y[l]);
        acc[l] += d;
      }
    }
  }
#pragma unroll
  for (int l = 0; l < QM; ++l)
    if (l < q) gmask[idx[l]] = acc[l] * sd.rsq;
}

template <int Q>
hipError_t launch_q_mask_grad(const SplitQDesc& sd, bool synthesis, long long batch,
                              const float2* a, long long a_bs, const float* mask,
                              const float2* d0, long long d0_bs, const float2* dw,
                              long long dw_bs, float* gmask, hipStream_t s) {
  const unsigned grid = (unsigned)((sd.mN + 255) / 256);
  if (synthesis)
    hipLaunchKernelGGL(unsplit_q_mask_grad_kernel<Q>, dim3(grid), dim3(256), 0, s, sd, batch, d0,
                       d0_bs, dw, dw_bs, mask, a, a_bs, gmask);
  else
    hipLaunchKernelGGL(split_q_mask_grad_kernel<Q>, dim3(grid), dim3(256), 0, s, sd, batch, a,
                       a_bs, mask, d0, d0_bs, dw, dw_bs, gmask);
  return hipGetLastError();
}

hipError_t dispatch_q_mask_grad(const SplitQDesc& sd, bool synthesis, long long batch,
                                const float2* a, long long a_bs, const float* mask,
                                const float2* d0, long long d0_bs, const float2* dw,
                                long long dw_bs, float* gmask, hipStream_t s) {
  if (sd.q < 3 || sd.q > kMaxQ) return hipErrorInvalidValue;
  switch (sd.q) {
    case 3: return launch_q_mask_grad<3>(sd, synthesis, batch, a, a_bs, mask, d0, d0_bs, dw, dw_bs, gmask, s);
    case 4: return launch_q_mask_grad<4>(sd, synthesis, batch, a, a_bs, mask, d0, d0_bs, dw, dw_bs, gmask, s);
    case 8: return launch_q_mask_grad<8>(sd, synthesis, batch, a, a_bs, mask, d0, d0_bs, dw, dw_bs, gmask, s);
    default: return launch_q_mask_grad<0>(sd, synthesis, batch, a, a_bs, mask, d0, d0_bs, dw, dw_bs, gmask, s);
  }
}

template <int Q>
hipError_t launch_q(const SplitQDesc& sd, bool inverse, long long batch, const float2* a,
                    long long a_bs, const float* mask, const float2* d0c, float2* d0,
                    long long d0_bs, const float2* dwc, float2* dw, long long dw_bs, float2* ah,
                    hipStream_t s) {
  const unsigned grid = (unsigned)((sd.mN + 255) / 256);
  if (inverse)
    hipLaunchKernelGGL(unsplit_q_kernel<Q>, dim3(grid), dim3(256), 0, s, sd, batch, d0c, d0_bs,
                       dwc, dw_bs, mask, ah, a_bs);
  else
    hipLaunchKernelGGL(split_q_kernel<Q>, dim3(grid), dim3(256), 0, s, sd, batch, a, a_bs, mask,
                       d0, d0_bs, dw, dw_bs);
  return hipGetLastError();
}

hipError_t dispatch_q(const SplitQDesc& sd, bool inverse, long long batch, const float2* a,
                      long long a_bs, const float* mask, const float2* d0c, float2* d0,
                      long long d0_bs, const float2* dwc, float2* dw, long long dw_bs, float2* ah,
                      hipStream_t s) {
  if (sd.q < 3 || sd.q > kMaxQ) return hipErrorInvalidValue;
  switch (sd.q) {
    case 3: return launch_q<3>(sd, inverse, batch, a, a_bs, mask, d0c, d0, d0_bs, dwc, dw, dw_bs, ah, s);
    case 4: return launch_q<4>(sd, inverse, batch, a, a_bs, mask, d0c, d0, d0_bs, dwc, dw, dw_bs, ah, s);
    case 8: return launch_q<8>(sd, inverse, batch, a, a_bs, mask, d0c, d0, d0_bs, dwc, dw, dw_bs, ah, s);
    default: return launch_q<0>(sd, inverse, batch, a, a_bs, mask, d0c, d0, d0_bs, dwc, dw, dw_bs, ah, s);
  }
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

hipError_t launch_split_q(const SplitQDesc& sd, long long batch, const float2* ahat, long long ah_bs,
                          const float* mask, float2* d0, long long d0_bs, float2* dw,
                          long long dw_bs, hipStream_t s) {
  return dispatch_q(sd, false, batch, ahat, ah_bs, mask, nullptr, d0, d0_bs, nullptr, dw, dw_bs,
                    nullptr, s);
}

hipError_t launch_unsplit_q(const SplitQDesc& sd, long long batch, const float2* d0,
                            long long d0_bs, const float2* dw, long long dw_bs, const float* mask,
                            float2* ahat, long long ah_bs, hipStream_t s) {
  return dispatch_q(sd, true, batch, nullptr, ah_bs, mask, d0, nullptr, d0_bs, dw, nullptr, dw_bs,
                    ahat, s);
}

hipError_t launch_split_q_mask_grad(const SplitQDesc& sd, long long batch, const float2* ahat,
                                    long long ah_bs, const float* mask, const float2* g0,
                                    long long g0_bs, const float2* gw, long long gw_bs,
                                    float* gmask, hipStream_t s) {
  return dispatch_q_mask_grad(sd, false, batch, ahat, ah_bs, mask, g0, g0_bs, gw, gw_bs, gmask, s);
}

hipError_t launch_unsplit_q_mask_grad(const SplitQDesc& sd, long long batch, const float2* d0,
                                      long long d0_bs, const float2* dw, long long dw_bs,
                                      const float* mask, const float2* g, long long g_bs,
                                      float* gmask, hipStream_t s) {
  return dispatch_q_mask_grad(sd, true, batch, g, g_bs, mask, d0, d0_bs, dw, dw_bs, gmask, s);
}

hipError_t launch_split_chain(int K, const SplitChain& c, long long batch, const float2* ahat,
                              long long ah_bs, float2* d1, long long d1_bs, hipStream_t s) {
  const unsigned grid = blocks_for(c.sd[K - 1].mN, 256);
  switch (K) {
    case 2: hipLaunchKernelGGL(split_chain_kernel<2>, dim3(grid), dim3(256), 0, s, c, batch, ahat, ah_bs, d1, d1_bs); break;
    case 3: hipLaunchKernelGGL(split_chain_kernel<3>, dim3(grid), dim3(256), 0, s, c, batch, ahat, ah_bs, d1, d1_bs); break;
    case 4: hipLaunchKernelGGL(split_chain_kernel<4>, dim3(grid), dim3(256), 0, s, c, batch, ahat, ah_bs, d1, d1_bs); break;
    default: return hipErrorInvalidValue;
  }
  return hipGetLastError();
}

hipError_t launch_unsplit_chain(int K, const SplitChain& c, long long batch, const float2* d1,
                                long long d1_bs, float2* ahat, long long ah_bs, hipStream_t s) {
  const unsigned grid = blocks_for(c.sd[K - 1].mN, 256);
  switch (K) {
    case 2: hipLaunchKernelGGL(unsplit_chain_kernel<2>, dim3(grid), dim3(256), 0, s, c, batch, d1, d1_bs, ahat, ah_bs); break;
    case 3: hipLaunchKernelGGL(unsplit_chain_kernel<3>, dim3(grid), dim3(256), 0, s, c, batch, d1, d1_bs, ahat, ah_bs); break;
    case 4: hipLaunchKernelGGL(unsplit_chain_kernel<4>, dim3(grid), dim3(256), 0, s, c, batch, d1, d1_bs, ahat, ah_bs); break;
    default: return hipErrorInvalidValue;
  }
  return hipGetLastError();
}

}  // namespace lfft

namespace lfft {
namespace {
struct Fac5 {
  float f[5];
};

// One thread per boundary class, the batch loop inside.
__global__ void __launch_bounds__(256) boundary_scale_kernel(const long long* __restrict__ idx,
                                                             const int* __restrict__ r, long long n,
                                                             Fac5 fac, float2* __restrict__ data,
                                                             long long batch, long long bstride) {
  const long long i = (long long)blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= n) return;
  const long long k = idx[i];
  const float f = fac.f[r[i]];
  for (long long b = 0; b < batch; ++b) {
    float2 v = data[b * bstride + k];
    data[b * bstride + k] = make_float2(v.x * f, v.y * f);
  }
}
}  // namespace

hipError_t launch_boundary_scale(const long long* idx, const int* r, long long n, const float* fac,
                                 float2* data, long long batch, long long bstride, hipStream_t s) {
  Fac5 f;
  for (int i = 0; i < 5; ++i) f.f[i] = fac[i];
  hipLaunchKernelGGL(boundary_scale_kernel, dim3((unsigned)((n + 255) / 256)), dim3(256), 0, s, idx,
                     r, n, f, data, batch, bstride);
  return hipGetLastError();
}

}  // namespace lfft
