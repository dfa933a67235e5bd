// Split-BF16 MFMA FFT pass for gfx950 (descriptor kind 3).
//
// A workgroup of 256 threads owns a tile of T = 4096 complex values (W
// pencils of length L, W * L = T) staged in LDS.  The gather from the input
// order and the scatter to the output order (natural orders through the
// planner's Hermite-box tables, Section 3 bases and Theorem 1 of Section 4.1)
// happen in the load and store phases; in between, every Stockham stage
// reads its butterfly inputs from LDS, applies the twiddles in FP32 and
// writes the outputs back.
//
// Radix-16 stages are dense products: for 32 butterflies at a time, the real
// 32 x 32 matrix W = [[C, -S], [S, C]] of the 16-point DFT (C + iS with
// entries exp(sign 2 pi i k j / 16)) multiplies the 32 x 32 block X whose
// columns are [Re x_0..15, Im x_0..15] of one butterfly each.  Both operands
// are split into bf16 pairs, v = hi + lo with hi = bf16_rne(v) and
// lo = bf16_rne(v - hi), and W X is accumulated in FP32 by
// v_mfma_f32_32x32x16_bf16 as W_hi X_hi + W_hi X_lo + W_lo X_hi (the
// W_lo X_lo term is below FP32 rounding of the result).  Other radices run
// in FP32 on the vector ALUs.
//
// MFMA 32x32x16 operand layout (lane l, element j; checked on the device):
// A[l % 32][8 (l / 32) + j], B[8 (l / 32) + j][l % 32], and result element v
// of lane l is D[8 (v / 4) + 4 (l / 32) + v % 4][l % 32].
#include <hip/hip_runtime.h>

#include "fft_common.hpp"
#include "kernels.hpp"
#include "ktrace.hpp"

namespace lfft {
namespace {
using namespace dev;

typedef __bf16 bf16x8 __attribute__((ext_vector_type(8)));
typedef float f32x16 __attribute__((ext_vector_type(16)));

constexpr int kT = 4096;        // tile elements
constexpr int kNT = 256;        // threads
constexpr int kPer = kT / kNT;  // complex values per thread and stage

__device__ __forceinline__ int phys(int e) { return e + (e >> 4); }

template <bool COLS>
__device__ __forceinline__ int lds_pos(int l, int w, int W, int L) {
  return COLS ? l * W + w : w * L + l;
}

struct Geo {
  int in0, in_step, out0, out_step, jm;
};

// Stockham geometry of pencil-local butterfly bl (power-of-two stage).
__device__ __forceinline__ Geo geo(const StageDesc& st, int bl) {
  Geo g;
  const int lg_nr = st.lg_n - st.lg_r;
  const int l_lo = bl & (st.stride - 1);
  const int q = bl >> st.lg_stride;
  const int j = q & ((1 << lg_nr) - 1);
  const int l_hi = q >> lg_nr;
  const int base = (l_hi << (st.lg_n + st.lg_stride)) + l_lo;
  g.in0 = base + (j << st.lg_stride);
  g.in_step = 1 << (lg_nr + st.lg_stride);
  g.jm = j & (st.Ns - 1);
  const int idxD = ((j >> st.lg_Ns) << (st.lg_Ns + st.lg_r)) + g.jm;
  g.out0 = base + (idxD << st.lg_stride);
  g.out_step = 1 << (st.lg_Ns + st.lg_stride);
  return g;
}

// butterfly b of the tile -> (pencil w, pencil-local butterfly bl); for
// strided pencils consecutive b are consecutive pencils (consecutive LDS words)
template <bool COLS>
__device__ __forceinline__ void bf_split(int b, int W, int nbl, int& w, int& bl) {
  if (COLS) {
    w = b % W;
    bl = b / W;
  } else {
    w = b / nbl;
    bl = b - w * nbl;
  }
}

__device__ __forceinline__ float2 twiddle(const StageDesc& st, int jm, int i, int sign) {
  const int tstep = jm << (st.lg_n - st.lg_Ns - st.lg_r);
  float2 w = st.tw[(tstep * i) & (st.n - 1)];
  if (sign > 0) w.y = -w.y;
  return w;
}

__device__ __forceinline__ void split_bf16(float v, __bf16& hi, __bf16& lo) {
  hi = (__bf16)v;
  lo = (__bf16)(v - (float)hi);
}

// The four A operands of the radix-16 product for this lane: K block kb
// (0: multiplies Re x, 1: multiplies Im x), hi and lo parts.
struct WOps {
  bf16x8 hi[2], lo[2];
};

__device__ __forceinline__ WOps make_w(int lane, int sign) {
  WOps o;
  const int r = lane & 31, h = lane >> 5;
  const int k = r & 15;
  const bool imrow = r >= 16;
#pragma unroll
  for (int j = 0; j < 8; ++j) {
    const int i = 8 * h + j;
    // exp(sign 2 pi i t / 16) with t = k i mod 16; root16 covers t < 8 and
    // the upper half is its negative
    const int t = (k * i) & 15;
    float2 f = root16(t & 7, sign);
    if (t >= 8) f = make_float2(-f.x, -f.y);
    // rows 0-15 (Re y): [C, -S]; rows 16-31 (Im y): [S, C]
    const float a0 = imrow ? f.y : f.x;
    const float a1 = imrow ? f.x : -f.y;
    __bf16 h0, l0, h1, l1;
    split_bf16(a0, h0, l0);
    split_bf16(a1, h1, l1);
    o.hi[0][j] = h0;
    o.lo[0][j] = l0;
    o.hi[1][j] = h1;
    o.lo[1][j] = l1;
  }
  return o;
}

template <bool COLS>
__device__ __forceinline__ void stage_mfma(const StageDesc& st, const WOps& Wm, int sign,
                                           float2* lds, int W, int L, float2* y, int* ypos) {
  const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
  const int c = lane & 31, h = lane >> 5;
  const int nbl = L >> 4;
#pragma unroll
  for (int rd = 0; rd < kT / 16 / 32 / (kNT / 64); ++rd) {
    const int b = (wave + (kNT / 64) * rd) * 32 + c;
    int w, bl;
    bf_split<COLS>(b, W, nbl, w, bl);
    const Geo g = geo(st, bl);
    bf16x8 rh, rl, ih, il;
    // twiddles w^i, i = 8h .. 8h+7, from two table entries: w^(8h) and w,
    // then successive products (a few ulp, far inside this path's bound)
    float2 tcur = twiddle(st, g.jm, 8 * h, sign);
    const float2 tstep = twiddle(st, g.jm, 1, sign);
#pragma unroll
    for (int j = 0; j < 8; ++j) {
      const int i = 8 * h + j;
      float2 x = lds[phys(lds_pos<COLS>(g.in0 + i * g.in_step, w, W, L))];
      x = c_mul(x, tcur);
      tcur = c_mul(tcur, tstep);
      __bf16 a, e;
      split_bf16(x.x, a, e);
      rh[j] = a;
      rl[j] = e;
      split_bf16(x.y, a, e);
      ih[j] = a;
      il[j] = e;
    }
    f32x16 acc = {0};
    acc = __builtin_amdgcn_mfma_f32_32x32x16_bf16(Wm.hi[0], rh, acc, 0, 0, 0);
    acc = __builtin_amdgcn_mfma_f32_32x32x16_bf16(Wm.hi[0], rl, acc, 0, 0, 0);
    acc = __builtin_amdgcn_mfma_f32_32x32x16_bf16(Wm.lo[0], rh, acc, 0, 0, 0);
    acc = __builtin_amdgcn_mfma_f32_32x32x16_bf16(Wm.hi[1], ih, acc, 0, 0, 0);
    acc = __builtin_amdgcn_mfma_f32_32x32x16_bf16(Wm.hi[1], il, acc, 0, 0, 0);
    acc = __builtin_amdgcn_mfma_f32_32x32x16_bf16(Wm.lo[1], ih, acc, 0, 0, 0);
#pragma unroll
    for (int v = 0; v < 8; ++v) {
      const int k = 8 * (v >> 2) + 4 * h + (v & 3);
      y[rd * 8 + v] = make_float2(acc[v], acc[v + 8]);
      ypos[rd * 8 + v] = phys(lds_pos<COLS>(g.out0 + k * g.out_step, w, W, L));
    }
  }
}

template <bool COLS, int R>
__device__ __forceinline__ void stage_valu(const StageDesc& st, int sign, float2* lds, int W,
                                           int L, float2* y, int* ypos) {
  const int nbl = L / R;
#pragma unroll
  for (int q = 0; q < kPer / R; ++q) {
    const int b = threadIdx.x + kNT * q;
    int w, bl;
    bf_split<COLS>(b, W, nbl, w, bl);
    const Geo g = geo(st, bl);
    float2 v[R];
    const float2 tstep = twiddle(st, g.jm, 1, sign);
    float2 tcur = tstep;
#pragma unroll
    for (int i = 0; i < R; ++i) {
      float2 x = lds[phys(lds_pos<COLS>(g.in0 + i * g.in_step, w, W, L))];
      if (i > 0) {
        x = c_mul(x, tcur);
        tcur = c_mul(tcur, tstep);
      }
      v[i] = x;
    }
    dft_pow2<R>(v, sign);
#pragma unroll
    for (int i = 0; i < R; ++i) {
      y[q * R + i] = v[i];
      ypos[q * R + i] = phys(lds_pos<COLS>(g.out0 + i * g.out_step, w, W, L));
    }
  }
}

// index of tile element (pencil w, position l) on one side
template <int MODE>
__device__ __forceinline__ long long side_index(const MapDesc& m, long long b, int o, int l, int s,
                                                int L, int S) {
  if constexpr (MODE == MAP_IDENTITY) {
    return b * m.bstride + ((long long)o * L + l) * (long long)S + s;
  } else if constexpr (MODE == MAP_LINEAR) {
    return b * m.bstride + (long long)m.To[o].x + (long long)m.Tl[l].x + (long long)m.Ts[s].x;
  } else {
    int c[4] = {0, 0, 0, 0};
    if (m.d == 2) {
      gadd2(m, c[0], c[1], m.To[o]);
      gadd2(m, c[0], c[1], m.Tl[l]);
      gadd2(m, c[0], c[1], m.Ts[s]);
      return b * m.bstride + c[0] * m.H[1][1] + c[1];
    }
    if (m.d == 3) {
      gadd3(m, c, m.To[o]);
      gadd3(m, c, m.Tl[l]);
      gadd3(m, c, m.Ts[s]);
      return b * m.bstride + nat_index3(m, c);
    }
    gadd32(m, c, m.To[o]);
    gadd32(m, c, m.Tl[l]);
    gadd32(m, c, m.Ts[s]);
    return b * m.bstride + nat_index32(m, c);
  }
}

template <bool COLS, int MIN, int MOUT>
__global__ void __launch_bounds__(kNT) fft_mfma_kernel(PassDesc p, const float2* __restrict__ in,
                                                       float2* __restrict__ out) {
  extern __shared__ float2 lds[];
  const int L = p.L, S = p.S, O = p.O, W = p.W;
  const int tid = threadIdx.x;
  const long long npen = p.batch * (long long)O * S;
  const long long tile = xcd_tile(blockIdx.x, gridDim.x);
  // load: element e -> (w, l); consecutive e are consecutive HBM words of
  // the identity layout on both pencil orientations.  All loads are issued
  // before the first LDS write, so their latencies overlap.
  {
    float2 v[kPer];
#pragma unroll
    for (int k = 0; k < kPer; ++k) {
      const int e = tid + kNT * k;
      const int w = COLS ? e % W : e / L;
      const int l = COLS ? e / W : e % L;
      const long long pen = tile * W + w;
      v[k] = make_float2(0.f, 0.f);
      if (pen < npen) {
        const long long bo = pen / S;
        const int s = (int)(pen - bo * S);
        const long long b = bo / O;
        const int o = (int)(bo - b * O);
        v[k] = in[side_index<MIN>(p.in, b, o, l, s, L, S)];
      }
    }
#pragma unroll
    for (int k = 0; k < kPer; ++k) {
      const int e = tid + kNT * k;
      const int w = COLS ? e % W : e / L;
      const int l = COLS ? e / W : e % L;
      lds[phys(lds_pos<COLS>(l, w, W, L))] = v[k];
    }
  }
  __syncthreads();
  const WOps Wm = make_w(tid & 63, p.sign);
  float2 y[kPer];
  int ypos[kPer];
  for (int si = 0; si < p.nst; ++si) {
    const StageDesc& st = p.st[si];
    switch (st.radix) {
      case 16: stage_mfma<COLS>(st, Wm, p.sign, lds, W, L, y, ypos); break;
      case 8: stage_valu<COLS, 8>(st, p.sign, lds, W, L, y, ypos); break;
      case 4: stage_valu<COLS, 4>(st, p.sign, lds, W, L, y, ypos); break;
      default: stage_valu<COLS, 2>(st, p.sign, lds, W, L, y, ypos); break;
    }
    __syncthreads();
#pragma unroll
    for (int k = 0; k < kPer; ++k) lds[ypos[k]] = y[k];
    __syncthreads();
  }
  // store: four-step twiddle, 1/sqrt(m) scale, scatter
#pragma unroll
  for (int k = 0; k < kPer; ++k) {
    const int e = tid + kNT * k;
    const int w = COLS ? e % W : e / L;
    const int l = COLS ? e / W : e % L;
    const long long pen = tile * W + w;
    if (pen >= npen) continue;
    const long long bo = pen / S;
    const int s = (int)(pen - bo * S);
    const long long b = bo / O;
    const int o = (int)(bo - b * O);
    float2 x = lds[phys(lds_pos<COLS>(l, w, W, L))];
    if (p.post) {
      const long long lo = (s / p.lo_div) % p.lo_n;
      const long long t = ((long long)(l % p.post_lmod) * lo) % p.postN;
      float2 tw = c_mul(p.tw_hi[t >> 12], p.tw_lo[t & 4095]);
      if (p.sign > 0) tw.y = -tw.y;
      x = c_mul(x, tw);
    }
    x.x *= p.scale;
    x.y *= p.scale;
    out[side_index<MOUT>(p.out, b, o, l, s, L, S)] = x;
  }
}

template <bool COLS, int MIN, int MOUT>
hipError_t launch_t(const PassDesc& p, const float2* in, float2* out, hipStream_t s) {
  const long long npen = p.batch * (long long)p.O * p.S;
  const long long tiles = (npen + p.W - 1) / p.W;
  if (tiles <= 0) return hipSuccess;
  if (tiles > 0x7fffffffLL) return hipErrorInvalidValue;
  const size_t lds = (size_t)(kT + kT / 16 + 1) * sizeof(float2);
  hipLaunchKernelGGL((fft_mfma_kernel<COLS, MIN, MOUT>), dim3((unsigned)tiles), dim3(kNT), lds, s,
                     p, in, out);
  return hipGetLastError();
}

template <bool COLS, int MIN>
hipError_t launch_out(const PassDesc& p, const float2* in, float2* out, hipStream_t s) {
  switch (p.out.mode) {
    case MAP_IDENTITY: return launch_t<COLS, MIN, MAP_IDENTITY>(p, in, out, s);
    case MAP_LINEAR: return launch_t<COLS, MIN, MAP_LINEAR>(p, in, out, s);
    default: return launch_t<COLS, MIN, MAP_NATURAL>(p, in, out, s);
  }
}

template <bool COLS>
hipError_t launch_in(const PassDesc& p, const float2* in, float2* out, hipStream_t s) {
  if (p.in.mode == MAP_NATURAL) return launch_out<COLS, MAP_NATURAL>(p, in, out, s);
  return launch_out<COLS, MAP_IDENTITY>(p, in, out, s);
}

}  // namespace

const char* mfma_kernel_name(const PassDesc& p) {
  const int min = p.in.mode == MAP_NATURAL ? 2 : 0;
  return kernel_name_intern("fft_mfma_kernel<%s, %d, %d>", p.S > 1 ? "true" : "false", min,
                            p.out.mode);
}

hipError_t launch_mfma_pass(const PassDesc& p, const float2* in, float2* out, hipStream_t s) {
  if ((long long)p.W * p.L != kT || p.L < 32) return hipErrorInvalidValue;
  return p.S > 1 ? launch_in<true>(p, in, out, s) : launch_in<false>(p, in, out, s);
}

}  // namespace lfft
