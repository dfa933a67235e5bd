// Device body of the register-resident power-of-two FFT pass: one tile of
// W pencils of length L, P = 16 points per thread, Stockham stages of radix
// 2/4/8/16 in registers with padded LDS transposes between them, the natural
// gather fused into the first load and the natural scatter (plus the optional
// four-step twiddle and the 1/sqrt(m) scale) fused into the last store.
//
// Used by the one-launch-per-pass kernel and by the batched persistent kernel.
#pragma once
#include <hip/hip_runtime.h>

#include "fft_common.hpp"

namespace lfft {
namespace fastk {
using namespace dev;

__device__ __forceinline__ int phys(int e) { return e + (e >> 4); }

struct Pencil {
  long long b;
  int o, s;
  bool active;
};

// Butterfly geometry of pencil-local butterfly index bl in a stage.
struct BfGeom {
  int in0, in_step;    // positions of input i: in0 + i * in_step
  int out0, out_step;  // positions of output i: out0 + i * out_step
  int jm;              // j mod Ns (twiddle exponent)
};

__device__ __forceinline__ BfGeom geom(const StageDesc& st, int bl) {
  BfGeom g;
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

// One side of a pencil: the signal's base pointer and 32-bit element
// offsets inside the signal (the planner keeps these lattices below 2^30
// points).
template <int MODE>
struct Addr {
  const float2* base;
  int lin;              // IDENTITY: o*L*S + s; LINEAR: To[o] + Ts[s]
  int cbase[4];         // NATURAL: To[o] (+) Ts[s]
};

template <int MODE>
__device__ __forceinline__ void addr_init(Addr<MODE>& A, const MapDesc& m, const float2* buf,
                                          const Pencil& pc, int L, int S) {
  A.base = buf + pc.b * m.bstride;
  if constexpr (MODE == MAP_IDENTITY) {
    A.lin = pc.o * L * S + pc.s;
  } else if constexpr (MODE == MAP_LINEAR) {
    A.lin = m.To[pc.o].x + m.Ts[pc.s].x;
  } else {
    A.cbase[0] = A.cbase[1] = A.cbase[2] = A.cbase[3] = 0;
    if (m.d == 2) {
      gadd2(m, A.cbase[0], A.cbase[1], m.To[pc.o]);
      gadd2(m, A.cbase[0], A.cbase[1], m.Ts[pc.s]);
    } else if (m.d == 3) {
      gadd3(m, A.cbase, m.To[pc.o]);
      gadd3(m, A.cbase, m.Ts[pc.s]);
    } else {
      gadd32(m, A.cbase, m.To[pc.o]);
      gadd32(m, A.cbase, m.Ts[pc.s]);
    }
  }
}

// Visit the element offsets of positions l0 + i*step, i < R.
template <int MODE, int R, class F>
__device__ __forceinline__ void for_positions(const Addr<MODE>& A, const MapDesc& m, int S, int l0,
                                              int step, F&& f) {
  if constexpr (MODE == MAP_IDENTITY) {
    const int a = A.lin + l0 * S;
#pragma unroll
    for (int i = 0; i < R; ++i) f(i, a + i * step * S);
  } else if constexpr (MODE == MAP_LINEAR) {
#pragma unroll
    for (int i = 0; i < R; ++i) f(i, A.lin + m.Tl[l0 + i * step].x);
  } else {
    const int4 D = m.Tl[step];
    if (m.d == 2) {
      int c0 = A.cbase[0], c1 = A.cbase[1];
      gadd2(m, c0, c1, m.Tl[l0]);
      const int h11 = m.H[1][1];
#pragma unroll
      for (int i = 0; i < R; ++i) {
        f(i, c0 * h11 + c1);
        if (i + 1 < R) gadd2(m, c0, c1, D);
      }
    } else if (m.d == 3) {
      int c[4] = {A.cbase[0], A.cbase[1], A.cbase[2], 0};
      gadd3(m, c, m.Tl[l0]);
#pragma unroll
      for (int i = 0; i < R; ++i) {
        f(i, nat_index3(m, c));
        if (i + 1 < R) gadd3(m, c, D);
      }
    } else {
      int c[4] = {A.cbase[0], A.cbase[1], A.cbase[2], A.cbase[3]};
      gadd32(m, c, m.Tl[l0]);
#pragma unroll
      for (int i = 0; i < R; ++i) {
        f(i, nat_index_i(m, c));
        if (i + 1 < R) gadd32(m, c, D);
      }
    }
  }
}

template <int R>
__device__ __forceinline__ void dftR(float2* v, int sign) {
  dft_pow2<R>(v, sign);
}

template <int P, int R, int MIN>
__device__ __forceinline__ void load_first(float2* v, const PassDesc& p, const Addr<MIN>& A,
                                           int jt, int TPP, bool active) {
  const StageDesc& st = p.st[0];
#pragma unroll
  for (int q = 0; q < P / R; ++q) {
    BfGeom g = geom(st, jt + TPP * q);
    if (active) {
      for_positions<MIN, R>(A, p.in, p.S, g.in0, g.in_step,
                            [&](int i, int off) { v[q * R + i] = A.base[(unsigned)off]; });
    } else {
#pragma unroll
      for (int i = 0; i < R; ++i) v[q * R + i] = make_float2(0.f, 0.f);
    }
  }
}

// Base twiddles of a stage: for every butterfly of the thread, w^(2^k) for
// 2^k < R with w = exp(-2 pi i jm / (Ns R)), read from the FP64-built table
// of the digit.  Issued one stage ahead so their latency hides behind the
// LDS exchange.
template <int P, int R>
__device__ __forceinline__ void prefetch_tw(float2* twb, const StageDesc& st, int jt, int TPP) {
  constexpr int LG = R == 16 ? 4 : R == 8 ? 3 : R == 4 ? 2 : 1;
#pragma unroll
  for (int q = 0; q < P / R; ++q) {
    BfGeom g = geom(st, jt + TPP * q);
    const int tstep = g.jm << (st.lg_n - st.lg_Ns - st.lg_r);
#pragma unroll
    for (int k = 0; k < LG; ++k) twb[q * LG + k] = st.tw[tstep << k];
  }
}

// Multiply input i of one butterfly by w^i, i = 1..R-1, building every power
// from the base powers w, w^2, w^4, w^8 with at most three products.
template <int R>
__device__ __forceinline__ void apply_tw(float2* x, const float2* b, int sign) {
  float2 pw[R];
  float2 b0 = b[0];
  if (sign > 0) b0.y = -b0.y;
  pw[1] = b0;
  if constexpr (R >= 4) {
    float2 b1 = b[1];
    if (sign > 0) b1.y = -b1.y;
    pw[2] = b1;
    pw[3] = c_mul(b0, b1);
  }
  if constexpr (R >= 8) {
    float2 b2 = b[2];
    if (sign > 0) b2.y = -b2.y;
    pw[4] = b2;
#pragma unroll
    for (int i = 5; i < 8; ++i) pw[i] = c_mul(pw[i - 4], b2);
  }
  if constexpr (R >= 16) {
    float2 b3 = b[3];
    if (sign > 0) b3.y = -b3.y;
    pw[8] = b3;
#pragma unroll
    for (int i = 9; i < 16; ++i) pw[i] = c_mul(pw[i - 8], b3);
  }
#pragma unroll
  for (int i = 1; i < R; ++i) x[i] = c_mul(x[i], pw[i]);
}

// tw: the stage has twiddles (Ns > 1; the first stage of a digit has none)
template <int P, int R>
__device__ __forceinline__ void compute_stage(float2* v, const float2* twb, int sign, bool tw) {
  constexpr int LG = R == 16 ? 4 : R == 8 ? 3 : R == 4 ? 2 : 1;
#pragma unroll
  for (int q = 0; q < P / R; ++q) {
    if (tw) apply_tw<R>(&v[q * R], &twb[q * LG], sign);
    dftR<R>(&v[q * R], sign);
  }
}

// LDS element index of pencil-local position l of tile pencil w
template <bool COLS>
__device__ __forceinline__ int lds_e(int l, int w, int W, int L) {
  return COLS ? l * W + w : w * L + l;
}

template <int P, int R, bool COLS, int PART>
__device__ __forceinline__ void lds_write(const float2* v, void* lds, const StageDesc& st, int jt,
                                          int TPP, int w, int W, int L) {
#pragma unroll
  for (int q = 0; q < P / R; ++q) {
    BfGeom g = geom(st, jt + TPP * q);
#pragma unroll
    for (int i = 0; i < R; ++i) {
      int e = phys(lds_e<COLS>(g.out0 + i * g.out_step, w, W, L));
      if constexpr (PART == 0)
        static_cast<float2*>(lds)[e] = v[q * R + i];
      else if constexpr (PART == 1)
        static_cast<float*>(lds)[e] = v[q * R + i].x;
      else
        static_cast<float*>(lds)[e] = v[q * R + i].y;
    }
  }
}

template <int P, int R, bool COLS, int PART>
__device__ __forceinline__ void lds_read(float2* v, const void* lds, const StageDesc& st, int jt,
                                         int TPP, int w, int W, int L) {
#pragma unroll
  for (int q = 0; q < P / R; ++q) {
    BfGeom g = geom(st, jt + TPP * q);
#pragma unroll
    for (int i = 0; i < R; ++i) {
      int e = phys(lds_e<COLS>(g.in0 + i * g.in_step, w, W, L));
      if constexpr (PART == 0)
        v[q * R + i] = static_cast<const float2*>(lds)[e];
      else if constexpr (PART == 1)
        v[q * R + i].x = static_cast<const float*>(lds)[e];
      else
        v[q * R + i].y = static_cast<const float*>(lds)[e];
    }
  }
}

#define LFFT_RADIX_SWITCH(R_, ...)                         \
  switch (R_) {                                            \
    case 2: { constexpr int RR = 2; __VA_ARGS__; } break;   \
    case 4: { constexpr int RR = 4; __VA_ARGS__; } break;   \
    case 8: { constexpr int RR = 8; __VA_ARGS__; } break;   \
    default: { constexpr int RR = 16; __VA_ARGS__; } break; \
  }

template <int P, int R, int MOUT>
__device__ __forceinline__ void store_last_r(const float2* v, const PassDesc& p,
                                             const Addr<MOUT>& A, int jt, int TPP,
                                             const Pencil& pc) {
  const StageDesc& st = p.st[p.nst - 1];
  float2* out = const_cast<float2*>(A.base);
  const bool scaled = p.scale != 1.0f;
  // four-step twiddle exponent ((l mod post_lmod) * lo) mod postN, lo fixed
  // per pencil
  const long long lo = p.post ? (pc.s / p.lo_div) % p.lo_n : 0;
#pragma unroll
  for (int q = 0; q < P / R; ++q) {
    BfGeom g = geom(st, jt + TPP * q);
    for_positions<MOUT, R>(A, p.out, p.S, g.out0, g.out_step, [&](int i, int off) {
      float2 x = v[q * R + i];
      if (p.post) {
        const int l = (g.out0 + i * g.out_step) % p.post_lmod;
        const long long t = ((long long)l * lo) % p.postN;
        float2 w = c_mul(p.tw_hi[t >> 12], p.tw_lo[t & 4095]);
        if (p.sign > 0) w.y = -w.y;
        x = c_mul(x, w);
      }
      if (scaled) {
        x.x *= p.scale;
        x.y *= p.scale;
      }
      out[(unsigned)off] = x;
    });
  }
}

template <int P, int MOUT>
__device__ __forceinline__ void store_last(const float2* v, const PassDesc& p, const Addr<MOUT>& A,
                                           int jt, int TPP, const Pencil& pc) {
  LFFT_RADIX_SWITCH(p.st[p.nst - 1].radix, (store_last_r<P, RR, MOUT>(v, p, A, jt, TPP, pc)));
}

// Process tile `tile` of pass p with NT = W * L / P threads (tid < NT);
// lds holds (W*L + W*L/16 + 1) float2 (SPLIT: floats).
template <int P, bool COLS, bool SPLIT, int MIN, int MOUT>
__device__ __forceinline__ void fast_tile(const PassDesc& p, long long tile, int tid,
                                          const float2* __restrict__ in,
                                          float2* __restrict__ out, void* lds) {
  const int L = p.L, S = p.S, O = p.O, W = p.W;
  const int TPP = L / P;
  int w, jt;
  if (COLS) {
    w = tid % W;
    jt = tid / W;
  } else {
    w = tid / TPP;
    jt = tid - w * TPP;
  }
  Pencil pc;
  const long long npen = p.batch * (long long)O * S;
  const long long pen = tile * W + w;
  pc.active = pen < npen;
  {
    const long long pp = pc.active ? pen : 0;
    const long long bo = pp / S;
    pc.s = (int)(pp - bo * S);
    pc.b = bo / O;
    pc.o = (int)(bo - pc.b * O);
  }
  float2 v[P];
  {
    Addr<MIN> A;
    addr_init<MIN>(A, p.in, in, pc, L, S);
    LFFT_RADIX_SWITCH(p.st[0].radix, (load_first<P, RR, MIN>(v, p, A, jt, TPP, pc.active)));
  }
  float2 twb[8];
  if (p.st[0].Ns > 1)
    LFFT_RADIX_SWITCH(p.st[0].radix, (prefetch_tw<P, RR>(twb, p.st[0], jt, TPP)));
  for (int si = 0; si < p.nst; ++si) {
    const StageDesc& st = p.st[si];
    LFFT_RADIX_SWITCH(st.radix, (compute_stage<P, RR>(v, twb, p.sign, st.Ns > 1)));
    if (si + 1 < p.nst) {
      const StageDesc& nx = p.st[si + 1];
      if (nx.Ns > 1) LFFT_RADIX_SWITCH(nx.radix, (prefetch_tw<P, RR>(twb, nx, jt, TPP)));
      if constexpr (!SPLIT) {
        LFFT_RADIX_SWITCH(st.radix, (lds_write<P, RR, COLS, 0>(v, lds, st, jt, TPP, w, W, L)));
        __syncthreads();
        LFFT_RADIX_SWITCH(nx.radix, (lds_read<P, RR, COLS, 0>(v, lds, nx, jt, TPP, w, W, L)));
        __syncthreads();
      } else {
        LFFT_RADIX_SWITCH(st.radix, (lds_write<P, RR, COLS, 1>(v, lds, st, jt, TPP, w, W, L)));
        __syncthreads();
        LFFT_RADIX_SWITCH(nx.radix, (lds_read<P, RR, COLS, 1>(v, lds, nx, jt, TPP, w, W, L)));
        __syncthreads();
        LFFT_RADIX_SWITCH(st.radix, (lds_write<P, RR, COLS, 2>(v, lds, st, jt, TPP, w, W, L)));
        __syncthreads();
        LFFT_RADIX_SWITCH(nx.radix, (lds_read<P, RR, COLS, 2>(v, lds, nx, jt, TPP, w, W, L)));
        __syncthreads();
      }
    }
  }
  if (pc.active) {
    Addr<MOUT> A;
    addr_init<MOUT>(A, p.out, out, pc, L, S);
    store_last<P, MOUT>(v, p, A, jt, TPP, pc);
  }
}

}  // namespace fastk
}  // namespace lfft
