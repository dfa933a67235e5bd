// Device helpers shared by the FFT pass kernels: complex arithmetic,
// in-register DFTs of small lengths and the natural-order group arithmetic
// of the gather/scatter maps.
#pragma once
#include <hip/hip_runtime.h>

#include "device.hpp"

namespace lfft {
namespace dev {

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

// exp(sign * 2 pi i k / 32) for k in [0, 16): cos and sin of multiples of pi/16
__device__ __forceinline__ float2 root32(int k, int sign) {
  constexpr float C[16] = {1.0f, 0.98078528040323044913f, 0.92387953251128675613f,
                           0.83146961230254523708f, 0.70710678118654752440f,
                           0.55557023301960222474f, 0.38268343236508977173f,
                           0.19509032201612826785f, 0.0f, -0.19509032201612826785f,
                           -0.38268343236508977173f, -0.55557023301960222474f,
                           -0.70710678118654752440f, -0.83146961230254523708f,
                           -0.92387953251128675613f, -0.98078528040323044913f};
  constexpr float Sn[16] = {0.0f, 0.19509032201612826785f, 0.38268343236508977173f,
                            0.55557023301960222474f, 0.70710678118654752440f,
                            0.83146961230254523708f, 0.92387953251128675613f,
                            0.98078528040323044913f, 1.0f, 0.98078528040323044913f,
                            0.92387953251128675613f, 0.83146961230254523708f,
                            0.70710678118654752440f, 0.55557023301960222474f,
                            0.38268343236508977173f, 0.19509032201612826785f};
  return make_float2(C[k], sign < 0 ? -Sn[k] : Sn[k]);
}

// o * exp(sign 2 pi i K / R) for a compile-time K < R / 2: the factors 1
// and sign * i cost no multiplication (IEEE semantics keep the compiler
// from dropping products with the constant 0 by itself).
template <int R, int K>
__device__ __forceinline__ float2 rot_k(float2 o, int sign) {
  if constexpr (K == 0) {
    return o;
  } else if constexpr (4 * K == R) {
    return c_muli(o, sign);
  } else if constexpr (R == 32) {
    return c_mul(root32(K, sign), o);
  } else {
    return c_mul(root16(K * (16 / R), sign), o);
  }
}

// butterflies k = K .. R/2 - 1 of the last combining step
template <int R, int K>
struct Combine {
  __device__ __forceinline__ static void run(float2* v, const float2* e, const float2* o, int sign) {
    if constexpr (K < R / 2) {
      const float2 t = rot_k<R, K>(o[K], sign);
      v[K] = c_add(e[K], t);
      v[K + R / 2] = c_sub(e[K], t);
      Combine<R, K + 1>::run(v, e, o, sign);
    }
  }
};

template <int R>
__device__ __forceinline__ void dft_pow2(float2* v, int sign) {
  static_assert(R <= 32, "radix above 32");
  // even/odd split: X[k] = E[k] + w^k O[k], X[k + R/2] = E[k] - w^k O[k]
  float2 e[R / 2], o[R / 2];
#pragma unroll
  for (int i = 0; i < R / 2; ++i) {
    e[i] = v[2 * i];
    o[i] = v[2 * i + 1];
  }
  dft_pow2<R / 2>(e, sign);
  dft_pow2<R / 2>(o, sign);
  Combine<R, 0>::run(v, e, o, sign);
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


}  // namespace dev
}  // namespace lfft

namespace lfft {
namespace dev {

// Group sum in Z^d / H Z^d of two reduced coordinate vectors (int32; the
// planner routes lattices with m >= 2^30 to the generic kernel).
__device__ __forceinline__ void gadd32(const MapDesc& m, int* c, int4 b) {
  c[0] += b.x;
  c[1] += b.y;
  c[2] += b.z;
  c[3] += b.w;
  // Both operands are reduced.  Processing coordinates from the last one,
  // coordinate i has received at most k = d - 1 - i corrections of size
  // below H_ii from the later columns, so it lies in (-k H_ii, (2 + k) H_ii)
  // and needs at most k + 1 subtractions or k additions of column i.
  // Branch-free selects, fully unrolled so that c stays in registers.
#pragma unroll
  for (int i = 3; i >= 0; --i) {
    if (i < m.d) {
      const int k = m.d - 1 - i;
#pragma unroll
      for (int t = 0; t < 4 - i; ++t) {
        if (t <= k) {
          const bool over = c[i] >= m.H[i][i];
#pragma unroll
          for (int r = 0; r <= i; ++r) c[r] -= over ? m.H[r][i] : 0;
        }
      }
#pragma unroll
      for (int t = 0; t < 3 - i; ++t) {
        if (t < k) {
          const bool under = c[i] < 0;
#pragma unroll
          for (int r = 0; r <= i; ++r) c[r] += under ? m.H[r][i] : 0;
        }
      }
    }
  }
}

// Workgroups are dispatched round-robin over the 8 XCDs of the MI355X.  Map
// dispatch index i to a logical tile so that every XCD works on one
// contiguous range of tiles: concurrently running neighbours share cache
// lines in that XCD's L2 (partial-line reads hit, partial-line writes merge).
__device__ __forceinline__ long long xcd_tile(long long i, long long n) {
  const long long per = n >> 3, rem = n & 7;
  const long long x = i & 7, k = i >> 3;
  return x * per + (x < rem ? x : rem) + k;
}

// Non-temporal 8-byte load and store: the line is not kept for reuse.  For
// data read or written once by a call (whole lines, so that no other wave
// has to fetch the same line again), which leaves the caches to the data
// that is read again.
typedef float stream_f2 __attribute__((ext_vector_type(2)));
__device__ __forceinline__ float2 load_stream(const float2* p) {
  const stream_f2 t = __builtin_nontemporal_load(reinterpret_cast<const stream_f2*>(p));
  return make_float2(t.x, t.y);
}
__device__ __forceinline__ void store_stream(float2* p, float2 v) {
  const stream_f2 t = {v.x, v.y};
  __builtin_nontemporal_store(t, reinterpret_cast<stream_f2*>(p));
}

// Natural box of a 2-D lattice, column Hermite form [[h00, h01], [0, h11]]:
// c += b for reduced c and b.  c1 + b1 < 2 h11 needs at most one column-1
// subtraction; c0 then lies in (-h00, 2 h00 - 1) and needs at most one
// correction by h00.
__device__ __forceinline__ void gadd2(const MapDesc& m, int& c0, int& c1, int4 b) {
  c0 += b.x;
  c1 += b.y;
  const bool o1 = c1 >= m.H[1][1];
  c1 -= o1 ? m.H[1][1] : 0;
  c0 -= o1 ? m.H[0][1] : 0;
  c0 += c0 < 0 ? m.H[0][0] : 0;
  c0 -= c0 >= m.H[0][0] ? m.H[0][0] : 0;
}

// Natural box of a 3-D lattice (upper-triangular H): c += b for reduced c
// and b.  Coordinate 2 needs at most one subtraction of column 2, which
// leaves coordinate 1 in (-h11, 2 h11 - 1): one correction by column 1;
// coordinate 0 then lies in (-2 h00, 3 h00 - 2): at most two corrections.
__device__ __forceinline__ void gadd3(const MapDesc& m, int* c, int4 b) {
  c[0] += b.x;
  c[1] += b.y;
  c[2] += b.z;
  const bool o2 = c[2] >= m.H[2][2];
  c[2] -= o2 ? m.H[2][2] : 0;
  c[1] -= o2 ? m.H[1][2] : 0;
  c[0] -= o2 ? m.H[0][2] : 0;
  const bool u1 = c[1] < 0, o1 = c[1] >= m.H[1][1];
  c[1] += u1 ? m.H[1][1] : (o1 ? -m.H[1][1] : 0);
  c[0] += u1 ? m.H[0][1] : (o1 ? -m.H[0][1] : 0);
  const int h00 = m.H[0][0];
  c[0] += c[0] < 0 ? h00 : 0;
  c[0] += c[0] < 0 ? h00 : 0;
  c[0] -= c[0] >= h00 ? h00 : 0;
  c[0] -= c[0] >= h00 ? h00 : 0;
}

__device__ __forceinline__ int nat_index3(const MapDesc& m, const int* c) {
  return c[0] * (int)m.box_stride[0] + c[1] * (int)m.box_stride[1] + c[2];
}

// linear natural index (int: the planner keeps these lattices below 2^30 points)
__device__ __forceinline__ int nat_index_i(const MapDesc& m, const int* c) {
  int idx = 0;
#pragma unroll
  for (int i = 0; i < 4; ++i)
    if (i < m.d) idx += c[i] * (int)m.box_stride[i];
  return idx;
}

__device__ __forceinline__ long long nat_index32(const MapDesc& m, const int* c) {
  long long idx = 0;
#pragma unroll
  for (int i = 0; i < 4; ++i)
    if (i < m.d) idx += (long long)c[i] * m.box_stride[i];
  return idx;
}

}  // namespace dev
}  // namespace lfft
