// Persistent FFT pass for single-digit power-of-two pencils (the dominant
// case: the last axis of the eps-grid in rows, or one outer axis in column
// tiles).
//
// Every workgroup stays resident and walks a contiguous range of tiles of
// its XCD; two workgroups per CU overlap one tile's HBM traffic with the
// other's arithmetic.  A tile is transformed by radix-32/16/8 Stockham
// stages in VGPRs with padded LDS transposes between stages.  Pencil length
// L, pencils per tile W and the radix sequence are compile-time constants,
// so the butterfly geometry and the LDS offsets fold to constants; the
// tile's signal and pencil indices are uniform (scalar unit) and every
// global access is a 32-bit offset from a uniform base.
#include <hip/hip_runtime.h>

#include <atomic>

#include "fft_common.hpp"
#include "kernels.hpp"
#include "ktrace.hpp"

namespace lfft {
namespace {
using namespace dev;

constexpr int kP = 32;  // values per thread
// workgroups per CU the register budget is sized for
constexpr int kRowsWgPerCu = 2;
constexpr int kColsWgPerCu = 1;
// exchange real and imaginary parts separately for row tiles (halves LDS)
constexpr bool kSplitRows = false;

__device__ __forceinline__ int sphys(int e) { return e + (e >> 4); }

// Radix sequence of a pencil of length L with 32 values per thread: a
// radix-32 first stage (no twiddles) and radix-16/8 stages after it.
__host__ __device__ constexpr int seq_radix(int L, int s) {
  return L == 8192 ? (s == 0 ? 32 : 16)
       : L == 4096 ? (s == 0 ? 32 : s == 1 ? 16 : 8)
       : L == 2048 ? (s == 0 ? 32 : 8)
       : L == 1024 ? 32
       : L == 512 ? (s == 0 ? 32 : 16)
       : 16;  // 256
}
__host__ __device__ constexpr int seq_len(int L) {
  return (L == 8192 || L == 4096 || L == 2048) ? 3 : 2;
}
__host__ __device__ constexpr int seq_ns(int L, int s) {
  return s == 0 ? 1 : seq_ns(L, s - 1) * seq_radix(L, s - 1);
}
template <int L, int S>
struct StageR {
  static constexpr int value = seq_radix(L, S);
};
template <int L>
struct NStages {
  static constexpr int value = seq_len(L);
};
template <int L, int S>
struct StageNs {
  static constexpr int value = seq_ns(L, S);
};
template <int R>
struct Lg {
  static constexpr int value = R == 32 ? 5 : R == 16 ? 4 : R == 8 ? 3 : R == 4 ? 2 : 1;
};

// One side (input or output) of a tile: the signal's base pointer is uniform
// over the workgroup (a tile never straddles two signals), every per-lane
// offset is a 32-bit element index inside the signal.
template <int MODE>
struct Side {
  const float2* base;
  int lin;     // IDENTITY / LINEAR: offset of position 0 of the lane's pencil
  int c[4];    // NATURAL: To[o] (+) Ts[s]
};

template <int MODE>
__device__ __forceinline__ void side_init(Side<MODE>& A, const MapDesc& m, const float2* buf,
                                          long long b, int o, int s, int L, int S) {
  A.base = buf + b * m.bstride;
  if constexpr (MODE == MAP_IDENTITY) {
    A.lin = o * L * S + s;
  } else if constexpr (MODE == MAP_LINEAR) {
    A.lin = m.To[o].x + m.Ts[s].x;
  } else {
    A.c[0] = A.c[1] = A.c[2] = A.c[3] = 0;
    if (m.d == 2) {
      gadd2(m, A.c[0], A.c[1], m.To[o]);
      gadd2(m, A.c[0], A.c[1], m.Ts[s]);
    } else if (m.d == 3) {
      gadd3(m, A.c, m.To[o]);
      gadd3(m, A.c, m.Ts[s]);
    } else {
      gadd32(m, A.c, m.To[o]);
      gadd32(m, A.c, m.Ts[s]);
    }
  }
}

// element offsets of positions l0 + i*step (i < R) on one side
template <int MODE, int R, class F>
__device__ __forceinline__ void side_positions(const Side<MODE>& A, const MapDesc& m, int S, int l0,
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
      // two-dimensional box: two coordinates, index c0 * h11 + c1
      int c0 = A.c[0], c1 = A.c[1];
      gadd2(m, c0, c1, m.Tl[l0]);
      const int h11 = m.H[1][1];
#pragma unroll
      for (int i = 0; i < R; ++i) {
        f(i, c0 * h11 + c1);
        if (i + 1 < R) gadd2(m, c0, c1, D);
      }
    } else if (m.d == 3) {
      int c[4] = {A.c[0], A.c[1], A.c[2], 0};
      gadd3(m, c, m.Tl[l0]);
#pragma unroll
      for (int i = 0; i < R; ++i) {
        f(i, nat_index3(m, c));
        if (i + 1 < R) gadd3(m, c, D);
      }
    } else {
      int c[4] = {A.c[0], A.c[1], A.c[2], A.c[3]};
      gadd32(m, c, m.Tl[l0]);
#pragma unroll
      for (int i = 0; i < R; ++i) {
        f(i, nat_index_i(m, c));
        if (i + 1 < R) gadd32(m, c, D);
      }
    }
  }
}

// Uniform decomposition of a tile: its W pencils belong to one signal b;
// rows: pencil o = o0 + w (s = 0), column tiles: o = o0, s = s0 + w.
struct TileId {
  long long b;
  int o0, s0;
};

template <int W>
__device__ __forceinline__ TileId tile_of(long long tile, int O, int S) {
  const long long pen0 = tile * W;
  const long long per = (long long)O * S;
  TileId t;
  t.b = pen0 / per;
  const long long r = pen0 - t.b * per;
  t.o0 = (int)(r / S);
  t.s0 = (int)(r - (long long)t.o0 * S);
  return t;
}

// loads of the first stage's inputs of one tile into v
template <int L, bool COLS, int MIN>
__device__ __forceinline__ void load_tile(float2* v, const PassDesc& p, const float2* __restrict__ in,
                                          const TileId& t, int w, int jt) {
  constexpr int R = StageR<L, 0>::value;
  constexpr int TPP = L / kP;
  Side<MIN> A;
  side_init<MIN>(A, p.in, in, t.b, COLS ? t.o0 : t.o0 + w, COLS ? t.s0 + w : t.s0, L, p.S);
#pragma unroll
  for (int q = 0; q < kP / R; ++q) {
    const int j = jt + TPP * q;
    side_positions<MIN, R>(A, p.in, p.S, j, L / R,
                           [&](int i, int off) {
                             // rows passes: non-temporal loads of the
                             // caller's aligned input rows (first pass) or
                             // of the intermediate grid, dead once read
                             // (last pass of a reversed engine)
                             if constexpr (!COLS) {
                               if (MIN == MAP_NATURAL ? p.stream_in : p.stream_out) {
                                 v[q * R + i] = load_stream(A.base + (unsigned)off);
                                 return;
                               }
                             }
                             v[q * R + i] = A.base[(unsigned)off];
                           });
  }
}

template <int L, int SI>
__device__ __forceinline__ void tw_load(float2* twb, const PassDesc& p, int jt) {
  constexpr int R = StageR<L, SI>::value;
  constexpr int Ns = StageNs<L, SI>::value;
  constexpr int LG = Lg<R>::value;
  constexpr int TPP = L / kP;
  const float2* tw = p.st[0].tw;   // exp(-2 pi i k / L)
#pragma unroll
  for (int q = 0; q < kP / R; ++q) {
    const int j = jt + TPP * q;
    const int tstep = (j & (Ns - 1)) * (L / (Ns * R));
#pragma unroll
    for (int k = 0; k < LG; ++k) twb[q * LG + k] = tw[tstep << k];
  }
}

// x[i] *= w^i for a block of N = 2^(K+1) inputs: bit K of i selects the
// factor b[K] = w^(2^K); partial products are formed top-down so at most
// K + 1 of them are live at any time.
template <int N, int K>
struct TwRec {
  __device__ __forceinline__ static void run(float2* x, const float2* b, float2 part, bool has) {
    TwRec<N / 2, K - 1>::run(x, b, part, has);
    const float2 np = has ? c_mul(part, b[K]) : b[K];
    TwRec<N / 2, K - 1>::run(x + N / 2, b, np, true);
  }
};
template <int K>
struct TwRec<1, K> {
  __device__ __forceinline__ static void run(float2* x, const float2*, float2 part, bool has) {
    if (has) x[0] = c_mul(x[0], part);
  }
};

template <int R>
__device__ __forceinline__ void apply_tw_s(float2* x, const float2* b, int sign) {
  constexpr int LG = Lg<R>::value;
  float2 bb[LG];
#pragma unroll
  for (int k = 0; k < LG; ++k) {
    bb[k] = b[k];
    if (sign > 0) bb[k].y = -bb[k].y;
  }
  TwRec<R, LG - 1>::run(x, bb, make_float2(1.f, 0.f), false);
}

template <int L, int SI>
__device__ __forceinline__ void stage_compute(float2* v, const float2* twb, int sign) {
  constexpr int R = StageR<L, SI>::value;
  constexpr int LG = Lg<R>::value;
#pragma unroll
  for (int q = 0; q < kP / R; ++q) {
    if constexpr (SI > 0) apply_tw_s<R>(&v[q * R], &twb[q * LG], sign);
    dft_pow2<R>(&v[q * R], sign);
  }
}

template <bool COLS, int L, int W>
__device__ __forceinline__ int slds(int l, int w) {
  return sphys(COLS ? l * W + w : w * L + l);
}

// LDS word of pencil position l0 + delta where delta * (COLS ? W : 1) is a
// multiple of 16 or, for rows, l0 is a multiple of 16 and delta < 16: then
// sphys is linear in delta and the offset folds into the instruction.
template <bool COLS, int L, int W>
__device__ __forceinline__ int slds_off(int base_e, int delta) {
  const int d = COLS ? delta * W : delta;
  return base_e + d + (d >> 4);
}

// write stage SI outputs, read stage SI+1 inputs (one part: 0 both, 1 re, 2 im)
template <int L, int W, bool COLS, int SI, int PART>
__device__ __forceinline__ void exch_write(const float2* v, void* lds, int jt, int w) {
  constexpr int R = StageR<L, SI>::value;
  constexpr int Ns = StageNs<L, SI>::value;
  constexpr int TPP = L / kP;
  // linear offsets: rows need Ns % 16 == 0 or (Ns == 1 and R % 16 == 0);
  // column tiles need (Ns * W) % 16 == 0
  constexpr bool lin = COLS ? ((Ns * W) % 16 == 0) : (Ns % 16 == 0 || (Ns == 1 && R % 16 == 0));
#pragma unroll
  for (int q = 0; q < kP / R; ++q) {
    const int j = jt + TPP * q;
    const int out0 = (j / Ns) * Ns * R + (j & (Ns - 1));
    const int eb = slds<COLS, L, W>(out0, w);
#pragma unroll
    for (int i = 0; i < R; ++i) {
      const int e = lin ? slds_off<COLS, L, W>(eb, i * Ns) : slds<COLS, L, W>(out0 + i * Ns, w);
      if constexpr (PART == 0)
        static_cast<float2*>(lds)[e] = v[q * R + i];
      else if constexpr (PART == 1)
        static_cast<float*>(lds)[e] = v[q * R + i].x;
      else
        static_cast<float*>(lds)[e] = v[q * R + i].y;
    }
  }
}

template <int L, int W, bool COLS, int SI, int PART>
__device__ __forceinline__ void exch_read(float2* v, const void* lds, int jt, int w) {
  constexpr int R = StageR<L, SI>::value;
  constexpr int TPP = L / kP;
  static_assert((L / R) % 16 == 0, "read stride must keep LDS offsets linear");
#pragma unroll
  for (int q = 0; q < kP / R; ++q) {
    const int j = jt + TPP * q;
    const int eb = slds<COLS, L, W>(j, w);
#pragma unroll
    for (int i = 0; i < R; ++i) {
      const int e = slds_off<COLS, L, W>(eb, i * (L / R));
      if constexpr (PART == 0)
        v[q * R + i] = static_cast<const float2*>(lds)[e];
      else if constexpr (PART == 1)
        v[q * R + i].x = static_cast<const float*>(lds)[e];
      else
        v[q * R + i].y = static_cast<const float*>(lds)[e];
    }
  }
}

template <int L, int W, bool COLS, bool SPLIT, int SI>
__device__ __forceinline__ void stages_from(float2* v, float2* twb, void* lds, const PassDesc& p,
                                            int jt, int w) {
  constexpr int NS = NStages<L>::value;
  stage_compute<L, SI>(v, twb, p.sign);
  if constexpr (SI + 1 < NS) {
    tw_load<L, SI + 1>(twb, p, jt);
    if constexpr (!SPLIT) {
      exch_write<L, W, COLS, SI, 0>(v, lds, jt, w);
      __syncthreads();
      exch_read<L, W, COLS, SI + 1, 0>(v, lds, jt, w);
      __syncthreads();
    } else {
      exch_write<L, W, COLS, SI, 1>(v, lds, jt, w);
      __syncthreads();
      exch_read<L, W, COLS, SI + 1, 1>(v, lds, jt, w);
      __syncthreads();
      exch_write<L, W, COLS, SI, 2>(v, lds, jt, w);
      __syncthreads();
      exch_read<L, W, COLS, SI + 1, 2>(v, lds, jt, w);
      __syncthreads();
    }
    stages_from<L, W, COLS, SPLIT, SI + 1>(v, twb, lds, p, jt, w);
  }
}

template <int L, bool COLS, int MOUT>
__device__ __forceinline__ void store_tile(const float2* v, const PassDesc& p,
                                           float2* __restrict__ out, const TileId& t, int w,
                                           int jt) {
  constexpr int NS = NStages<L>::value;
  constexpr int R = StageR<L, NS - 1>::value;
  constexpr int Ns = StageNs<L, NS - 1>::value;
  constexpr int TPP = L / kP;
  const int o = COLS ? t.o0 : t.o0 + w;
  const int s = COLS ? t.s0 + w : t.s0;
  Side<MOUT> A;
  side_init<MOUT>(A, p.out, out, t.b, o, s, L, p.S);
  float2* base = const_cast<float2*>(A.base);
  const bool scaled = p.scale != 1.0f;
#pragma unroll
  for (int q = 0; q < kP / R; ++q) {
    const int j = jt + TPP * q;
    const int out0 = (j / Ns) * Ns * R + (j & (Ns - 1));
    side_positions<MOUT, R>(A, p.out, p.S, out0, Ns, [&](int i, int off) {
      float2 x = v[q * R + i];
      if (p.post) {
        const int l = (out0 + i * Ns) % p.post_lmod;
        const long long lo = (s / p.lo_div) % p.lo_n;
        const long long tt = ((long long)l * lo) % p.postN;
        float2 wv = c_mul(p.tw_hi[tt >> 12], p.tw_lo[tt & 4095]);
        if (p.sign > 0) wv.y = -wv.y;
        x = c_mul(x, wv);
      }
      if (scaled) {
        x.x *= p.scale;
        x.y *= p.scale;
      }
      if constexpr (MOUT == MAP_NATURAL && !COLS) {
        if (p.stream_out) {
          store_stream(base + (unsigned)off, x);
        } else {
          base[(unsigned)off] = x;
        }
      } else {
        base[(unsigned)off] = x;
      }
    });
  }
}

// Every launch satisfies (checked on the host): W divides the pencils of one
// signal (O * S), so all tiles are full and never straddle two signals, and
// one signal has fewer than 2^28 points (32-bit element offsets).
template <int L, int W, bool COLS, bool SPLIT, int MIN, int MOUT>
__global__ void __launch_bounds__(W * L / kP, (COLS ? kColsWgPerCu : kRowsWgPerCu)) fft_stream_kernel(PassDesc p, const float2* __restrict__ in,
                                                                float2* __restrict__ out) {
  extern __shared__ float2 lds_raw[];
  void* lds = lds_raw;
  constexpr int TPP = L / kP;
  const int tid = threadIdx.x;
  const int w = COLS ? tid % W : tid / TPP;
  const int jt = COLS ? tid / W : tid % TPP;
  const long long npen = p.batch * (long long)p.O * p.S;
  const long long ntiles = npen / W;
  // persistent schedule: XCD x owns tiles [beg_x, end_x); its k-th workgroup
  // takes beg_x + k, beg_x + k + nwg_x, ...
  const long long G = gridDim.x;
  const long long x = blockIdx.x & 7, k = blockIdx.x >> 3;
  const long long nwg_x = (G >> 3) + ((G & 7) > x ? 1 : 0);
  const long long per = ntiles >> 3, rem = ntiles & 7;
  const long long beg = x * per + (x < rem ? x : rem);
  const long long end = beg + per + (x < rem ? 1 : 0);
  long long tile = beg + k;
  if (tile >= end) return;

  float2 twb[16];
  float2 va[kP];
  for (; tile < end; tile += nwg_x) {
    const TileId ta = tile_of<W>(tile, p.O, p.S);
    load_tile<L, COLS, MIN>(va, p, in, ta, w, jt);
    stages_from<L, W, COLS, SPLIT, 0>(va, twb, lds, p, jt, w);
    store_tile<L, COLS, MOUT>(va, p, out, ta, w, jt);
  }
}

// compute units of the device and, per kernel, workgroups per CU: found on
// first use; threads that race here all store the same values
std::atomic<int> g_cus{0};

template <int L, int W, bool COLS, bool SPLIT, int MIN, int MOUT>
hipError_t launch_t(const PassDesc& p, const float2* in, float2* out, hipStream_t s) {
  auto kern = fft_stream_kernel<L, W, COLS, SPLIT, MIN, MOUT>;
  constexpr int NT = W * L / kP;
  constexpr int tile = W * L;
  constexpr size_t lds = (size_t)(tile + tile / 16 + 1) * (SPLIT ? sizeof(float) : sizeof(float2));
  static std::atomic<int> wgs_cache{0};
  int wgs_per_cu = wgs_cache.load(std::memory_order_acquire);
  if (!wgs_per_cu) {
    hipError_t e = hipFuncSetAttribute((const void*)kern, hipFuncAttributeMaxDynamicSharedMemorySize,
                                       160 * 1024);
    if (e != hipSuccess) return e;
    int nb = 0;
    e = hipOccupancyMaxActiveBlocksPerMultiprocessor(&nb, kern, NT, lds);
    if (e != hipSuccess) return e;
    wgs_per_cu = nb > 0 ? nb : 1;
    wgs_cache.store(wgs_per_cu, std::memory_order_release);
  }
  int cus = g_cus.load(std::memory_order_acquire);
  if (!cus) {
    int dev = 0;
    hipError_t e = hipGetDevice(&dev);
    if (e != hipSuccess) return e;
    e = hipDeviceGetAttribute(&cus, hipDeviceAttributeMultiprocessorCount, dev);
    if (e != hipSuccess) return e;
    g_cus.store(cus, std::memory_order_release);
  }
  const long long npen = p.batch * (long long)p.O * p.S;
  const long long ntiles = (npen + W - 1) / W;
  long long grid = (long long)cus * wgs_per_cu;
  if (grid > ntiles) grid = ntiles;
  hipLaunchKernelGGL(kern, dim3((unsigned)grid), dim3(NT), lds, s, p, in, out);
  return hipGetLastError();
}

// Exchange real and imaginary parts separately when the tile would not fit
// 72 KB of LDS as complex values, except for the 2048 x 8 column tiles with a
// natural side: one workgroup per CU holds their 139 KB complex tile, and
// whole complex exchanges (half the barriers) measured 2% faster on the step
// without spilling registers.
__host__ __device__ constexpr bool stream_split(int L, int W, bool cols, int min, int mout) {
  return (cols && L == 2048 && W == 8 && mout != MAP_LINEAR &&
          (min == MAP_NATURAL || mout == MAP_NATURAL))
             ? false
             : ((cols || kSplitRows) ? ((long long)W * L * 17 / 16 * 8 > 72 * 1024 || kSplitRows)
                                     : false);
}

template <int L, int W, bool COLS, int MIN>
hipError_t launch_o(const PassDesc& p, const float2* in, float2* out, hipStream_t s) {
  switch (p.out.mode) {
    case MAP_IDENTITY:
      return launch_t<L, W, COLS, stream_split(L, W, COLS, MIN, MAP_IDENTITY), MIN, MAP_IDENTITY>(
          p, in, out, s);
    case MAP_LINEAR:
      return launch_t<L, W, COLS, stream_split(L, W, COLS, MIN, MAP_LINEAR), MIN, MAP_LINEAR>(
          p, in, out, s);
    default:
      return launch_t<L, W, COLS, stream_split(L, W, COLS, MIN, MAP_NATURAL), MIN, MAP_NATURAL>(
          p, in, out, s);
  }
}

template <int L, int W, bool COLS>
hipError_t launch_i(const PassDesc& p, const float2* in, float2* out, hipStream_t s) {
  if (p.in.mode == MAP_NATURAL) return launch_o<L, W, COLS, MAP_NATURAL>(p, in, out, s);
  return launch_o<L, W, COLS, MAP_IDENTITY>(p, in, out, s);
}

}  // namespace

// (L, W) shapes with a compiled streaming kernel; see plan.cpp
bool stream_supported(int L, int W, bool cols) {
  if (!cols) {
    return (L == 8192 && W == 1) || (L == 4096 && W == 1) || (L == 2048 && W == 2) ||
           (L == 1024 && W == 4) || (L == 512 && W == 8) || (L == 256 && W == 16);
  }
  return (L == 4096 && W == 4) || (L == 2048 && W == 8) || (L == 1024 && (W == 16 || W == 8)) ||
         (L == 512 && (W == 32 || W == 16 || W == 8)) ||
         (L == 256 && (W == 64 || W == 32 || W == 16 || W == 8));
}

const char* stream_kernel_name(const PassDesc& p) {
  // the template arguments exactly as the profiler prints the symbol
  const bool cols = p.S > 1;
  const int W = p.W;
  const int min = p.in.mode == MAP_NATURAL ? 2 : 0;
  const int mout = p.out.mode;
  const bool split = stream_split(p.L, W, cols, min, mout);
  return kernel_name_intern("fft_stream_kernel<%d, %d, %s, %s, %d, %d>", p.L, W,
                            cols ? "true" : "false", split ? "true" : "false", min, mout);
}

hipError_t launch_stream_pass(const PassDesc& p, const float2* in, float2* out, hipStream_t s) {
  const bool cols = p.S > 1;
  if (!cols) {
    switch (p.L) {
      case 8192: return launch_i<8192, 1, false>(p, in, out, s);
      case 4096: return launch_i<4096, 1, false>(p, in, out, s);
      case 2048: return launch_i<2048, 2, false>(p, in, out, s);
      case 1024: return launch_i<1024, 4, false>(p, in, out, s);
      case 512: return launch_i<512, 8, false>(p, in, out, s);
      case 256: return launch_i<256, 16, false>(p, in, out, s);
      default: return hipErrorInvalidValue;
    }
  }
  switch (p.L * 100 + p.W) {
    case 4096 * 100 + 4: return launch_i<4096, 4, true>(p, in, out, s);
    case 2048 * 100 + 8: return launch_i<2048, 8, true>(p, in, out, s);
    case 1024 * 100 + 16: return launch_i<1024, 16, true>(p, in, out, s);
    case 1024 * 100 + 8: return launch_i<1024, 8, true>(p, in, out, s);
    case 512 * 100 + 32: return launch_i<512, 32, true>(p, in, out, s);
    case 512 * 100 + 16: return launch_i<512, 16, true>(p, in, out, s);
    case 512 * 100 + 8: return launch_i<512, 8, true>(p, in, out, s);
    case 256 * 100 + 64: return launch_i<256, 64, true>(p, in, out, s);
    case 256 * 100 + 32: return launch_i<256, 32, true>(p, in, out, s);
    case 256 * 100 + 16: return launch_i<256, 16, true>(p, in, out, s);
    case 256 * 100 + 8: return launch_i<256, 8, true>(p, in, out, s);
    default: return hipErrorInvalidValue;
  }
}

}  // namespace lfft
