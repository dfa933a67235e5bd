// Plain-old-data descriptors handed from the host planner to the gfx950
// kernels by value.  All pointers are device pointers into the plan's table
// blob.
#pragma once
#include <hip/hip_runtime.h>
#include <cstdint>

namespace lfft {

constexpr int kMaxStages = 24;

// How a pass addresses the buffer on one side.
//   IDENTITY : the internal grid layout, index = ((b*O + o)*L + l)*S + s
//   LINEAR   : separable offsets, index = b*bstride + To[o].x + Tl[l].x + Ts[s].x
//   NATURAL  : natural residue box of a lattice (column Hermite form H):
//              coords = To[o] (+) Tl[l] (+) Ts[s]  (group sum in Z^d / H Z^d),
//              index  = b*bstride + sum_i coords_i * box_stride_i
enum MapMode : int { MAP_IDENTITY = 0, MAP_LINEAR = 1, MAP_NATURAL = 2 };

struct MapDesc {
  int mode;
  int d;
  int H[4][4];
  long long box_stride[4];
  long long bstride;          // batch stride in elements (LINEAR / NATURAL)
  const int4* To;
  const int4* Tl;
  const int4* Ts;
};

// One Stockham stage: radix r on the pass digit of length n whose stride
// inside the pencil index l is `stride`; Ns is the product of the radices
// already applied to that digit.  tw[k] = exp(-2 pi i k / n), k in [0, n).
struct StageDesc {
  int radix;
  int n;
  int stride;
  int Ns;
  const float2* tw;
  // base-2 logarithms (power-of-two stages only, used by the fast kernel)
  int lg_r, lg_n, lg_stride, lg_Ns;
};

struct PassDesc {
  int kind;                   // 0 generic, 1 register-resident power-of-two, 2 streaming,
                              // 3 split-BF16 MFMA, 4 chirp-z (one whole axis)
  int P;                      // fast kernel: points per thread (16 or 32)
  int W;                      // fast kernel: pencils per workgroup
  int split;                  // fast kernel: exchange real and imaginary parts separately
  long long batch;            // number of signals
  int O, L, S;                // per-signal outer count, pencil length, inner count
  int TP;                     // pencils per tile
  int nst;
  StageDesc st[kMaxStages];
  int sign;                   // -1 forward, +1 inverse
  float scale;                // applied when storing
  // streaming kernel, last pass of a natural-order transform whose rows
  // pencils write whole aligned rows of the caller's output: stores marked
  // non-temporal, so that they do not evict the input and the intermediate
  // grid from the caches; its loads of the intermediate grid (whole rows,
  // dead once read) are non-temporal too
  int stream_out;
  // streaming kernel, first pass reading whole aligned rows of the caller's
  // natural-order input (read once by the call): loads marked non-temporal,
  // so that the intermediate grid stays in the caches for the next pass
  int stream_in;
  // four-step twiddle after the stages: x = ((l mod post_lmod) * lo) mod
  // postN with lo = (s / lo_div) % lo_n, factor exp(sign 2 pi i x / postN)
  // from the two-level table tw_hi[x >> 12] * tw_lo[x & 4095]; the high digit
  // is the last (fastest) digit of the pencil, of length post_lmod
  int post;
  int postN;
  int post_lmod;
  int lo_div;
  int lo_n;
  const float2* tw_hi;
  const float2* tw_lo;
  // chirp-z pass (kind 4): the axis of length L as a cyclic convolution of
  // length bN (a power of two >= 2L - 1); chirp[j] = exp(-pi i j^2 / L),
  // bhat = the DFT of the convolution kernel conj(chirp) (forward sign;
  // both conjugated for sign +1); blue = index of the plan's inner FFT
  int bN;
  int blue;
  const float2* chirp;
  const float2* bhat;
  MapDesc in, out;
};

// One pass of one lattice in the batched persistent launch.  Buffers are
// selected by index (0 caller input, 1 caller output, 2 workspace) so the
// descriptors do not depend on the call's pointers.
struct BatchPass {
  PassDesc pd;                // batch 1, maps and batch strides resolved
  long long in_off, out_off;  // element offsets of the lattice's signal
  int in_buf, out_buf;
  int variant;                // body: BATCH_ROWS_NN .. BATCH_COLS_IN
};

enum BatchVariant : int {
  BATCH_ROWS_NN = 0,          // contiguous pencils, natural in, natural out (one-pass lattice)
  BATCH_ROWS_NI = 1,          // contiguous pencils, natural in, grid out
  BATCH_COLS_NI = 2,          // strided pencils, natural in, grid out
  BATCH_ROWS_IN = 3,          // contiguous pencils, grid in, natural out
  BATCH_COLS_IN = 4,          // strided pencils, grid in, natural out
};

// floor(n / d) for 0 <= n < 2^31 as (n * mag) >> (31 + sh), with
// sh = ceil(log2 d) and mag = floor(2^(31 + sh) / d) + 1 < 2^32 (division by
// an invariant integer through multiplication; the rounding error of the
// scaled reciprocal stays below 1/d for n < 2^31).
struct FastDiv {
  unsigned mag;
  int sh;
};

__host__ __device__ __forceinline__ unsigned fast_div(unsigned n, FastDiv f) {
  return (unsigned)(((unsigned long long)n * f.mag) >> (31 + f.sh));
}

// One level of the Fourier-domain wavelet split (natural orders).
struct SplitDesc {
  long long mM;               // |det M_l| (points of the level)
  long long mN;               // |det N_l| = mM / 2
  int d;
  int KN[4];                  // natural box of N_l^T (Hermite diagonal)
  long long kstride[4];
  int HM[4][4];               // column Hermite form of M_l^T
  long long hstride[4];
  int s[4];                   // s = N_l^T g0 reduced into the M_l^T box
  int w[4];                   // phase weights: phi(h) = exp(-2 pi i (w.h mod E)/E)
  int E;                      // phase modulus (largest elementary divisor of M_l)
  const float2* tw;           // exp(-2 pi i t / E), t in [0, E)
  // 32-bit index path (every intermediate of the fiber maps below 2^30 in
  // magnitude, checked on the host): divisions by the box diagonals and by E
  // through FastDiv
  int narrow;
  FastDiv fKN[4], fHM[4], fE;
};

// Consecutive levels l .. l+K-1 of the q = 2 split run as one launch: a
// thread owns one fiber of the coarsest level and the tree of 2^K - 1 fibers
// below it, so the low-pass data between the levels stays in registers.
constexpr int kMaxChain = 4;

struct SplitChain {
  SplitDesc sd[kMaxChain];          // levels l .. l+K-1 (every one on the 32-bit path)
  const float* mask[kMaxChain];     // scaling masks, natural G(M_j^T)
  float2* d2[kMaxChain];            // wavelet channel of every level, natural G(N_j^T)
  long long d2_bs[kMaxChain];       // batch strides of d2
};

// One level of the q-channel split, q = |det J| > 2 (natural orders).  The
// fiber of k in G(N_l^T) is h_l = k + N_l^T g_l reduced into the Hermite box
// of M_l^T, g_0 = 0, g_1 .. g_{q-1} the other classes of G(J^T) in the natural
// order of the Hermite box of J^T.
constexpr int kMaxQ = 16;

struct SplitQDesc {
  long long mM;               // |det M_l|
  long long mN;               // |det N_l| = mM / q
  int d;
  int q;
  int KN[4];                  // natural box of N_l^T (Hermite diagonal)
  int HM[4][4];               // column Hermite form of M_l^T
  long long hstride[4];
  int s[kMaxQ][4];            // N_l^T g_l reduced into the M_l^T box (s[0] = 0)
  float rsq;                  // 1 / sqrt(q)
  int narrow;                 // 32-bit index path (bounds checked on the host)
  FastDiv fKN[4], fHM[4];
};

}  // namespace lfft
