// Fiber index arithmetic of the wavelet split (Section 5.3, steps 2-3; the
// unique decomposition eq. decomposition applied to G(M^T) = G(N^T) + N^T G(J^T)).
//
// For a natural index k of G(N_l^T) the fiber is {k + N_l^T g : g in G(J^T)},
// every member reduced into the Hermite box of M_l^T and addressed by its
// natural index.  For q = 2 the second member is h0 + s (s = N^T g0) and the
// fiber also carries the residue rho of the wavelet phase
// phi(h0) = exp(-2 pi i rho / E) (Section 6.2 wavelet symbol; E the largest
// elementary divisor of M_l).
//
// These functions are compiled for both the host and the device: the kernels
// of wavelet.hip call them per thread, and the host export of the maps
// (lwt_fiber_map) calls the very same code, so what the host reports is what
// the kernels address.
#pragma once
#include <hip/hip_runtime.h>

#include "device.hpp"

namespace lfft {
namespace fib {

struct FiberIdx {
  long long i0, i1;   // natural indices of h0 and h0 + s in G(M^T)
  long long rho;      // phase residue modulo sd.E
};

__host__ __device__ __forceinline__ long long floordiv_ll(long long a, long long b) {
  long long q = a / b;
  if ((a % b != 0) && ((a < 0) != (b < 0))) --q;
  return q;
}

// reduce v into the Hermite box of M^T (64-bit path)
template <class SD>
__host__ __device__ __forceinline__ void reduce_hm(const SD& sd, long long* v) {
  for (int i = sd.d - 1; i >= 0; --i) {
    long long q = floordiv_ll(v[i], sd.HM[i][i]);
    if (q)
      for (int r = 0; r <= i; ++r) v[r] -= q * sd.HM[r][i];
  }
}

// the same with 32-bit intermediates and invariant-divisor multiplications
// (every intermediate below 2^30 in magnitude, bounded on the host)
template <class SD>
__host__ __device__ __forceinline__ void reduce_hm32(const SD& sd, int* v) {
#pragma unroll
  for (int i = 3; i >= 0; --i) {
    if (i < sd.d) {
      const int h = sd.HM[i][i];
      const int x = v[i];
      const int q = x >= 0 ? (int)fast_div((unsigned)x, sd.fHM[i])
                           : -(int)fast_div((unsigned)(h - 1 - x), sd.fHM[i]);
#pragma unroll
      for (int r = 0; r <= i; ++r) v[r] -= q * sd.HM[r][i];
    }
  }
}

// q = 2, 64-bit path
__host__ __device__ __forceinline__ FiberIdx fiber_index64(const SplitDesc& sd, long long klin) {
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
  FiberIdx f;
  f.i0 = 0;
  f.i1 = 0;
  long long rho = 0;
  for (int i = 0; i < sd.d; ++i) {
    f.i0 += h0[i] * sd.hstride[i];
    f.i1 += h1[i] * sd.hstride[i];
    rho = (rho + (h0[i] % sd.E) * (long long)sd.w[i]) % sd.E;
  }
  f.rho = rho;
  return f;
}

// q = 2, 32-bit path (sd.narrow)
__host__ __device__ __forceinline__ FiberIdx fiber_index32(const SplitDesc& sd, long long klin) {
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
  FiberIdx f;
  f.i0 = i0;
  f.i1 = i1;
  f.rho = (long long)((unsigned)acc - q * (unsigned)sd.E);
  return f;
}

// q > 2: natural indices idx[l] of h_l = k + s_l, l < q (s_0 = 0); Q > 0
// fixes q at compile time, Q = 0 reads it from the descriptor
template <int Q>
__host__ __device__ __forceinline__ void fiber_q_index(const SplitQDesc& sd, long long klin,
                                                       long long* idx, bool narrow) {
  constexpr int QM = Q ? Q : kMaxQ;
  const int q = Q ? Q : sd.q;
  if (narrow) {
    int k[4] = {0, 0, 0, 0};
    unsigned r = (unsigned)klin;
#pragma unroll
    for (int i = 3; i >= 0; --i) {
      if (i < sd.d) {
        const unsigned t = fast_div(r, sd.fKN[i]);
        k[i] = (int)(r - t * (unsigned)sd.KN[i]);
        r = t;
      }
    }
    reduce_hm32(sd, k);
#pragma unroll
    for (int l = 0; l < QM; ++l) {
      if (l < q) {
        int h[4] = {k[0] + sd.s[l][0], k[1] + sd.s[l][1], k[2] + sd.s[l][2], k[3] + sd.s[l][3]};
        if (l) reduce_hm32(sd, h);
        int o = 0;
#pragma unroll
        for (int i = 0; i < 4; ++i)
          if (i < sd.d) o += h[i] * (int)sd.hstride[i];
        idx[l] = o;
      }
    }
  } else {
    long long k[4] = {0, 0, 0, 0};
    long long r = klin;
    for (int i = sd.d - 1; i >= 0; --i) {
      k[i] = r % sd.KN[i];
      r /= sd.KN[i];
    }
    reduce_hm(sd, k);
#pragma unroll
    for (int l = 0; l < QM; ++l) {
      if (l < q) {
        long long h[4] = {k[0] + sd.s[l][0], k[1] + sd.s[l][1], k[2] + sd.s[l][2],
                          k[3] + sd.s[l][3]};
        if (l) reduce_hm(sd, h);
        long long o = 0;
        for (int i = 0; i < sd.d; ++i) o += h[i] * sd.hstride[i];
        idx[l] = o;
      }
    }
  }
}

}  // namespace fib
}  // namespace lfft
