// Generic FFT pass for gfx950: any pencil length up to 8192 with any
// factorisation (radices 2, 3, 4, 8, 16 in registers, every other prime by a
// direct sum read from LDS).  One workgroup owns a tile of TP pencils; the
// tile lives in LDS in two ping-pong buffers between Stockham stages.
//
// The pass realises one factor group of the Kronecker form of the lattice
// Fourier matrix (Section 4.1, eqs. FourierKronecker2 and KroneckerFFT): the
// first pass gathers samples from their natural order through the pattern
// basis, the last pass scatters frequencies through the generating-group
// basis (Section 3), so neither order is ever materialised separately.
#include <hip/hip_runtime.h>

#include "kernels.hpp"

namespace lfft {
namespace {

__device__ __forceinline__ float2 c_mul(float2 a, float2 b) {
  return make_float2(a.x * b.x - a.y * b.y, a.x * b.y + a.y * b.x);
}
__device__ __forceinline__ float2 c_add(float2 a, float2 b) { return make_float2(a.x + b.x, a.y + b.y); }
__device__ __forceinline__ float2 c_sub(float2 a, float2 b) { return make_float2(a.x - b.x, a.y - b.y); }
__device__ __forceinline__ float2 c_conj(float2 a) { return make_float2(a.x, -a.y); }
// a * (sign * i)
__device__ __forceinline__ float2 c_muli(float2 a, int sign) {
  return sign < 0 ? make_float2(a.y, -a.x) : make_float2(-a.y, a.x);
}
__device__ __forceinline__ float2 tw_lookup(const float2* tw, long long k, int sign) {
  float2 w = tw[k];
  return sign < 0 ? w : c_conj(w);
}

// In-register DFT of power-of-two length R with exponent sign `sign`.
template <int R>
__device__ __forceinline__ void dft_pow2(float2* v, int sign);

template <>
__device__ __forceinline__ void dft_pow2<1>(float2*, int) {}

template <>
__device__ __forceinline__ void dft_pow2<2>(float2* v, int) {
  float2 a = v[0], b = v[1];
  v[0] = c_add(a, b);
  v[1] = c_sub(a, b);
}

template <>
__device__ __forceinline__ void dft_pow2<4>(float2* v, int sign) {
  float2 s02 = c_add(v[0], v[2]), d02 = c_sub(v[0], v[2]);
  float2 s13 = c_add(v[1], v[3]), d13 = c_muli(c_sub(v[1], v[3]), sign);
  v[0] = c_add(s02, s13);
  v[2] = c_sub(s02, s13);
  v[1] = c_add(d02, d13);
  v[3] = c_sub(d02, d13);
}

// exp(sign * 2 pi i k / 16) for k in [0, 8): cos and sin of multiples of pi/8
__device__ __forceinline__ float2 root16(int k, int sign) {
  constexpr float C[8] = {1.0f, 0.92387953251128675613f, 0.70710678118654752440f,
                          0.38268343236508977173f, 0.0f, -0.38268343236508977173f,
                          -0.70710678118654752440f, -0.92387953251128675613f};
  constexpr float Sn[8] = {0.0f, 0.38268343236508977173f, 0.70710678118654752440f,
                           0.92387953251128675613f, 1.0f, 0.92387953251128675613f,
                           0.70710678118654752440f, 0.38268343236508977173f};
  return make_float2(C[k], sign < 0 ? -Sn[k] : Sn[k]);
}

template <int R>
__device__ __forceinline__ void dft_pow2(float2* v, int sign) {
  static_assert(R <= 16, "radix above 16");
  // even/odd split: X[k] = E[k] + w^k O[k], X[k + R/2] = E[k] - w^k O[k]
  float2 e[R / 2], o[R / 2];
#pragma unroll
  for (int i = 0; i < R / 2; ++i) {
    e[i] = v[2 * i];
    o[i] = v[2 * i + 1];
  }
  dft_pow2<R / 2>(e, sign);
  dft_pow2<R / 2>(o, sign);
#pragma unroll
  for (int k = 0; k < R / 2; ++k) {
    float2 t = c_mul(root16(k * (16 / R), sign), o[k]);
    v[k] = c_add(e[k], t);
    v[k + R / 2] = c_sub(e[k], t);
  }
}

__device__ __forceinline__ void dft3(float2* v, int sign) {
  const float h = 0.86602540378443864676f;  // sqrt(3)/2
  float2 t1 = c_add(v[1], v[2]);
  float2 t2 = c_sub(v[1], v[2]);
  float2 x0 = v[0];
  v[0] = c_add(x0, t1);
  float2 mm = make_float2(x0.x - 0.5f * t1.x, x0.y - 0.5f * t1.y);
  float2 nn = c_muli(make_float2(h * t2.x, h * t2.y), sign);
  v[1] = c_add(mm, nn);
  v[2] = c_sub(mm, nn);
}

struct Coords {
  long long c[4];
};

__device__ __forceinline__ void group_add(const MapDesc& m, long long* c, int4 b) {
  c[0] += b.x;
  c[1] += b.y;
  c[2] += b.z;
  c[3] += b.w;
  for (int i = m.d - 1; i >= 0; --i) {
    const long long hii = m.H[i][i];
    while (c[i] >= hii)
      for (int r = 0; r <= i; ++r) c[r] -= m.H[r][i];
    while (c[i] < 0)
      for (int r = 0; r <= i; ++r) c[r] += m.H[r][i];
  }
}

__device__ __forceinline__ long long map_index(const MapDesc& m, long long b, int o, int l, int s,
                                               int L, int S) {
  if (m.mode == MAP_IDENTITY) return b * m.bstride + ((long long)o * L + l) * (long long)S + s;
  if (m.mode == MAP_LINEAR)
    return b * m.bstride + (long long)m.To[o].x + (long long)m.Tl[l].x + (long long)m.Ts[s].x;
  long long c[4] = {0, 0, 0, 0};
  group_add(m, c, m.To[o]);
  group_add(m, c, m.Tl[l]);
  group_add(m, c, m.Ts[s]);
  long long idx = b * m.bstride;
  for (int i = 0; i < m.d; ++i) idx += c[i] * m.box_stride[i];
  return idx;
}

template <int R>
__device__ __forceinline__ void stage_reg(const StageDesc& st, int sign, const float2* A, float2* B,
                                          int TP, bool colmajor, int L, int bf) {
  const int n = st.n, stride = st.stride, Ns = st.Ns;
  const int nr = n / R;
  int pp = bf % TP;
  int q = bf / TP;
  int l_lo = q % stride;
  q /= stride;
  int j = q % nr;
  int l_hi = q / nr;
  int base = l_hi * n * stride + l_lo;
  float2 v[R];
  const int jm = j % Ns;
  const long long tstep = (long long)(n / (Ns * R)) * jm;
#pragma unroll
  for (int i = 0; i < R; ++i) {
    int l = base + (j + i * nr) * stride;
    float2 x = colmajor ? A[l * TP + pp] : A[pp * L + l];
    if (i > 0 && jm > 0) x = c_mul(x, tw_lookup(st.tw, (tstep * i) % n, sign));
    v[i] = x;
  }
  if constexpr (R == 3) {
    dft3(v, sign);
  } else {
    dft_pow2<R>(v, sign);
  }
  int idxD = (j / Ns) * Ns * R + jm;
#pragma unroll
  for (int i = 0; i < R; ++i) {
    int l = base + (idxD + i * Ns) * stride;
    if (colmajor)
      B[l * TP + pp] = v[i];
    else
      B[pp * L + l] = v[i];
  }
}

__device__ void stage_generic(const StageDesc& st, int sign, const float2* A, float2* B, int TP,
                              bool colmajor, int L, int bf) {
  const int R = st.radix;
  const int n = st.n, stride = st.stride, Ns = st.Ns;
  const int nr = n / R;
  int pp = bf % TP;
  int q = bf / TP;
  int l_lo = q % stride;
  q /= stride;
  int j = q % nr;
  int l_hi = q / nr;
  int base = l_hi * n * stride + l_lo;
  const int jm = j % Ns;
  const long long tstep = (long long)(n / (Ns * R)) * jm;
  int idxD = (j / Ns) * Ns * R + jm;
  for (int k = 0; k < R; ++k) {
    float2 acc = make_float2(0.f, 0.f);
    for (int i = 0; i < R; ++i) {
      int l = base + (j + i * nr) * stride;
      float2 x = colmajor ? A[l * TP + pp] : A[pp * L + l];
      long long e = (tstep * i + (long long)nr * ((long long)i * k % R)) % n;
      acc = c_add(acc, c_mul(x, tw_lookup(st.tw, e, sign)));
    }
    int l = base + (idxD + k * Ns) * stride;
    if (colmajor)
      B[l * TP + pp] = acc;
    else
      B[pp * L + l] = acc;
  }
}

__global__ void __launch_bounds__(256) pass_generic_kernel(PassDesc p, const float2* __restrict__ in,
                                                           float2* __restrict__ out) {
  extern __shared__ float2 lds[];
  const int TP = p.TP, L = p.L, S = p.S, O = p.O;
  const int tile = TP * L;
  float2* A = lds;
  float2* B = lds + tile;
  const long long npen = p.batch * (long long)O * S;
  const long long pen0 = (long long)blockIdx.x * TP;
  const bool colmajor = S > 1;
  const int tid = threadIdx.x, NT = blockDim.x;

  for (int e = tid; e < tile; e += NT) {
    int pp, l;
    if (colmajor) {
      l = e / TP;
      pp = e % TP;
    } else {
      pp = e / L;
      l = e % L;
    }
    long long pen = pen0 + pp;
    float2 v = make_float2(0.f, 0.f);
    if (pen < npen) {
      long long bo = pen / S;
      int s = (int)(pen % S);
      long long b = bo / O;
      int o = (int)(bo % O);
      v = in[map_index(p.in, b, o, l, s, L, S)];
    }
    A[e] = v;
  }
  __syncthreads();

  for (int si = 0; si < p.nst; ++si) {
    const StageDesc st = p.st[si];
    const int nb = tile / st.radix;
    for (int bf = tid; bf < nb; bf += NT) {
      switch (st.radix) {
        case 2: stage_reg<2>(st, p.sign, A, B, TP, colmajor, L, bf); break;
        case 3: stage_reg<3>(st, p.sign, A, B, TP, colmajor, L, bf); break;
        case 4: stage_reg<4>(st, p.sign, A, B, TP, colmajor, L, bf); break;
        case 8: stage_reg<8>(st, p.sign, A, B, TP, colmajor, L, bf); break;
        case 16: stage_reg<16>(st, p.sign, A, B, TP, colmajor, L, bf); break;
        default: stage_generic(st, p.sign, A, B, TP, colmajor, L, bf); break;
      }
    }
    __syncthreads();
    float2* t = A;
    A = B;
    B = t;
  }

  for (int e = tid; e < tile; e += NT) {
    int pp, l;
    if (colmajor) {
      l = e / TP;
      pp = e % TP;
    } else {
      pp = e / L;
      l = e % L;
    }
    long long pen = pen0 + pp;
    if (pen >= npen) continue;
    long long bo = pen / S;
    int s = (int)(pen % S);
    long long b = bo / O;
    int o = (int)(bo % O);
    float2 v = A[e];
    if (p.post) {
      long long lo = (s / p.lo_div) % p.lo_n;
      long long x = ((long long)l * lo) % p.postN;
      float2 w = c_mul(p.tw_hi[x >> 12], p.tw_lo[x & 4095]);
      if (p.sign > 0) w = c_conj(w);
      v = c_mul(v, w);
    }
    v.x *= p.scale;
    v.y *= p.scale;
    out[map_index(p.out, b, o, l, s, L, S)] = v;
  }
}

}  // namespace

hipError_t launch_pass(const PassDesc& p, const float2* in, float2* out, hipStream_t s) {
  static bool attr = false;
  if (!attr) {
    hipError_t e = hipFuncSetAttribute((const void*)pass_generic_kernel,
                                       hipFuncAttributeMaxDynamicSharedMemorySize, 160 * 1024);
    if (e != hipSuccess) return e;
    attr = true;
  }
  const long long npen = p.batch * (long long)p.O * p.S;
  const long long tiles = (npen + p.TP - 1) / p.TP;
  const size_t lds = (size_t)2 * p.TP * p.L * sizeof(float2);
  if (tiles <= 0) return hipSuccess;
  if (tiles > 0x7fffffffLL) return hipErrorInvalidValue;
  hipLaunchKernelGGL(pass_generic_kernel, dim3((unsigned)tiles), dim3(256), lds, s, p, in, out);
  return hipGetLastError();
}

}  // namespace lfft
