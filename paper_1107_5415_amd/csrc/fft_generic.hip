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

#include <atomic>

#include "fft_common.hpp"
#include "kernels.hpp"

namespace lfft {
namespace {
using namespace dev;

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
  const long long pen0 = xcd_tile(blockIdx.x, gridDim.x) * TP;
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
      long long x = ((long long)(l % p.post_lmod) * lo) % p.postN;
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

const char* pass_kernel_name(const PassDesc& p) {
  if (p.kind == 3) return mfma_kernel_name(p);
  if (p.kind == 2) return stream_kernel_name(p);
  return p.kind == 1 ? fast_kernel_name(p) : "pass_generic_kernel";
}

hipError_t launch_pass(const PassDesc& p, const float2* in, float2* out, hipStream_t s) {
  if (p.kind == 3) return launch_mfma_pass(p, in, out, s);
  if (p.kind == 2) return launch_stream_pass(p, in, out, s);
  if (p.kind == 1) return launch_fast_pass(p, in, out, s);
  static std::atomic<bool> attr{false};
  if (!attr.load(std::memory_order_acquire)) {
    hipError_t e = hipFuncSetAttribute((const void*)pass_generic_kernel,
                                       hipFuncAttributeMaxDynamicSharedMemorySize, 160 * 1024);
    if (e != hipSuccess) return e;
    attr.store(true, std::memory_order_release);
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
