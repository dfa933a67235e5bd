// Host-side plans: exact integer planning, pass schedules and device tables.
#pragma once
#include <array>
#include <cstddef>
#include <cstdint>
#include <vector>

#include "device.hpp"
#include "intmat.hpp"

namespace lfft {

// Status codes (mirrors include/lfft.h).
enum Status : int {
  OK = 0,
  E_ARG = -1,
  E_SINGULAR = -2,
  E_NOT_INTEGRAL = -3,
  E_OVERFLOW = -4,
  E_UNSUPPORTED = -5,
  E_HIP = -6,
  E_NOMEM = -7,
  E_STATE = -8,
  E_IO = -9,
};

// plan flags (mirrors include/lfft.h)
constexpr uint32_t kPlanHostOnly = 0x1;
constexpr uint32_t kPlanSplitBf16 = 0x2;
constexpr uint32_t kPlanSingleStream = 0x4;
constexpr uint32_t kPlanSamples = 0x8;

struct StatusError {
  int code;
};

using Vec4 = std::array<i64, 4>;

// One side of a transform: the natural residue box of a lattice and the
// natural element reached by a unit step along every non-trivial grid axis.
struct Side {
  Mat H;                    // column Hermite form (upper triangular)
  std::vector<Vec4> unit;   // reduced natural coordinates, one per grid axis
};

struct Digit {
  int axis;                 // non-trivial grid axis
  i64 n;                    // digit length
  int part;                 // 0 whole axis, 1 high digit, 2 low digit, 3 whole axis
                            // by chirp-z (a prime factor too large for one pencil),
                            // 4 middle digit of an axis split in three
  i64 w_in;                 // grid-coordinate weight on the input side
  i64 w_out;                // grid-coordinate weight on the output side
};

struct PassRange {
  int a, b;                 // digits [a, b) are transformed
  bool post;                // four-step twiddle after this pass
  int post_axis;
};

// A transform on one Smith basis with a fixed sign; the first/last pass
// have two map variants (natural or grid layout) chosen at launch.
struct Engine {
  int sign = -1;
  std::vector<PassDesc> passes;
  MapDesc in_nat{}, in_grid{}, out_nat{}, out_grid{};
  bool has_nat_in = false, has_nat_out = false;
};

// Device table staging: offsets are encoded as (offset + 1) in pointer
// fields and patched to device addresses after the upload.
struct Blob {
  std::vector<uint8_t> bytes;
  size_t add(const void* p, size_t n);
  template <class T>
  const T* ref(const std::vector<T>& v) {
    return reinterpret_cast<const T*>(add(v.data(), v.size() * sizeof(T)) + 1);
  }
};

struct LatticePlan {
  int d = 0;
  Mat M;
  i64 m = 0;
  i64 batch = 1;
  uint32_t flags = 0;
  int tile_lg = 0;          // fixed-tile schedule (0: default schedule)
  int order = 0;
  Smith Sf;                 // forward basis (largest cycle along sample key e_d)
  Smith Si;                 // basis of M^T used by the natural->natural inverse
  bool Sf_aligned = false, Si_aligned = false;
  Mat HM, UM, HMT, UMT;     // Hermite forms of M and M^T
  std::vector<i64> eps;     // non-trivial elementary divisors, ascending
  std::vector<Digit> digits;
  std::vector<PassRange> ranges;
  Engine fwd, inv_nat, inv_grid;
  // natural -> natural inverse on the forward basis with the passes in
  // reverse order (built when only the forward basis is aligned and no axis
  // is split four-step): the last pass writes the aligned sample rows; used
  // by exec_lattice and by the batched launch
  Engine inv_rev;
  bool has_inv_rev = false;
  // natural -> natural forward on the inverse basis with the passes in
  // reverse order (built for the default schedule when only the inverse
  // basis is aligned and no axis is split four-step): the last pass writes
  // the frequency rows that basis aligns; used by exec_lattice
  Engine fwd_rev;
  bool has_fwd_rev = false;
  Blob blob;
  void* dtab = nullptr;     // device copy of blob
  size_t ws_elems = 0;      // workspace (complex64 elements) per call
  // Classes h of G(M^T) on the boundary of the cube M^T [-1/2, 1/2]^d
  // (r(h) > 0, Section 6.2), natural indices and r(h): the only frequencies
  // where the Dirichlet kernel's bracket sum differs from m^{-1/2}.  Built on
  // first use (build_boundary); dbnd holds [idx int64 x n][r int32 x n].
  // chirp-z axes: the inner power-of-two FFT plan of each (batch = the
  // axis's pencils), indexed by PassDesc::blue
  std::vector<LatticePlan*> blue;
  size_t blue_ws = 0;       // workspace of the chirp-z steps (after the pass buffer)
  bool bnd_built = false;
  std::vector<i64> bnd_idx;
  std::vector<int> bnd_r;
  void* dbnd = nullptr;
};

// tile_lg > 0 selects the fixed-tile schedule of the batched launch (tiles of
// 2^tile_lg elements, 8 <= tile_lg <= 13); order bit 0: leading chunk first,
// bit 1: smallest radix first, bit 2: chunk boundary mid-axis even where an
// axis boundary fits.
LatticePlan* build_lattice_plan(int d, const i64* M, i64 batch, uint32_t flags, int tile_lg = 0,
                                int order = 0);
void upload_plan(LatticePlan* p);   // allocates device tables (throws StatusError)
// The boundary classes of G(M^T) and their device copy (idempotent,
// thread-safe; allocates on first call unless host-only).
void build_boundary(LatticePlan* p);
void free_plan(LatticePlan* p);

// Natural -> grid index maps for tests (SAMPLES: lambda = Q^{-1} g mod eps,
// FREQS: mu = R^{-T} h mod eps, in the forward basis).
void natural_to_grid(const LatticePlan* p, int which, i64* out);

// Natural keys and symmetric representatives of the points of one side
// (which 0: samples, keys g of G(M) and m M^{-1} g; which 1: frequencies,
// keys h of G(M^T) and m M^{-T} h), coordinates reduced into [-m/2, m/2);
// host arrays of m x d, either may be null.
void points(const LatticePlan* p, int which, i64* keys, i64* sym);

struct WaveLevel {
  Mat Ml, Nl;
  i64 ml = 0;
  LatticePlan* fftN = nullptr;
  SplitDesc sd{};           // q = 2
  SplitQDesc sq{};          // q > 2
  LatticePlan* fftW = nullptr;  // q > 2: the q - 1 wavelet channels (batch q - 1)
};

struct BatchPlan;

struct WavePlan {
  int d = 0;
  Mat M, J;
  int q = 2;                // |det J|: channels per level
  int levels = 0;
  i64 batch = 1;
  i64 m = 0;
  LatticePlan* fftM = nullptr;
  std::vector<WaveLevel> lv;
  Blob blob;
  void* dtab = nullptr;     // device copy of blob (empty for q > 2)
  bool uploaded = false;    // every device table of the pyramid is resident
  size_t ws_elems = 0;
  // Channel FFTs of the small levels (small_from .. levels-1, and the final
  // low-pass channel) run as one batched launch: the splits leave their
  // Fourier channels in a staging area of the workspace, one inverse batched
  // launch writes them to the coefficients (and a forward one reads them back
  // for the reconstruction).  small_from == levels: no batching.
  int small_from = 0;
  BatchPlan* chan_dec = nullptr;
  BatchPlan* chan_rec = nullptr;
  std::vector<i64> stage_lvl;   // staging offset of level l's d2hat ([B][m_l/2])
  i64 stage_d1 = 0;             // staging offset of the final d1hat
  size_t fw_elems = 0;          // FFT workspace region (main stream)
  size_t stage_elems = 0;
  // The channel FFTs of the large levels (0 .. small_from-1) run on a second
  // stream, overlapping the chain of splits (decomposition) or ahead of the
  // unsplits (reconstruction); each has its own d2hat buffer, and the two
  // streams use separate FFT workspaces.
  std::vector<i64> big_d2;      // offset of level l's d2hat in the BD region
  size_t bd_elems = 0;          // BD region
  size_t fw2_elems = 0;         // FFT workspace of the second stream
  hipStream_t s2 = nullptr;
  bool single_stream = false;   // LWT_SINGLE_STREAM: no second stream
  bool samples = false;         // LWT_SAMPLES: point values on the signal side
  std::vector<hipEvent_t> ev;   // one per level
  hipEvent_t ev_join = nullptr;
};

WavePlan* build_wave_plan(int d, const i64* M, const i64* J, int levels, i64 batch, uint32_t flags);
void upload_wave_plan(WavePlan* w);
void free_wave_plan(WavePlan* w);
// Dirichlet scaling mask of level l in natural G(M_l^T) order (Section 6.2)
void dirichlet_mask(const WavePlan* w, int level, float* out);
// Fiber maps of level l for the natural indices k0 .. k0+count-1 of
// G(N_l^T), from the kernels' own index arithmetic: lifts[c*q + l] the
// natural index in G(M_l^T) of the fiber member l; phase[c] (q = 2 only) the
// residue rho with phi(h0) = exp(-2 pi i rho / m_l).  path 0: the kernels'
// choice, 1: the 32-bit path (E_UNSUPPORTED if the level's bounds exclude
// it), 2: the 64-bit path.
void fiber_map(const WavePlan* w, int level, int path, i64 k0, i64 count, i64* lifts, i64* phase);
// Scaling step of level l (Section 5.2, Theorem 3; P(J) cyclic): pattern
// dimensions of M_l and N_l, the natural sample key in G(M_l) of the step's
// direction N_l^{-1} z (z = J^{-1} g, g the first generating key of G(J) in
// natural order) and its grid coordinates in the forward Smith basis of M_l.
// Throws E_UNSUPPORTED when P(J) is not cyclic.
void level_scaling(const WavePlan* w, int level, int& d_M, int& d_N, i64* key, i64* grid);

// Execution (stream ordered).  bstride_in/out: batch strides in elements.
// scale_mul multiplies the last pass's output scale.
void exec_lattice(const LatticePlan* p, bool inverse, bool in_grid, bool out_grid,
                  const void* in, void* out, void* ws, long long bstride_in,
                  long long bstride_out, hipStream_t s, float scale_mul = 1.0f);
// Multiply the boundary classes of natural-frequency data [batch][bstride]
// by pow(2, dir * r(h) / 2) (dir = -1: samples -> coefficients; +1: back),
// on `s`; build_boundary must have run.
void scale_boundary(const LatticePlan* p, int dir, void* data, long long batch,
                    long long bstride, hipStream_t s);

}  // namespace lfft
