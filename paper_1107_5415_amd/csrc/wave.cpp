// Multi-level wavelet pyramid on the device (Section 5.3: one lattice FFT,
// then steps 3-4 on the low-pass Fourier data of every level, and one
// inverse FFT per channel), its inverse and both adjoints (|det J| = 2), and
// the q-channel pyramid for |det J| = q > 2 (adjoints without mask
// gradients).
//
// Layouts (complex64, batch outermost):
//   samples  : [B][m]  natural order of G(M)
//   coeffs   : [B][m]  = [d2^(1) | d2^(2) | ... | d2^(L) | d1^(L)], block l in
//              natural sample order of N_l (m_l/2 points)
//   saved    : decompose: Fourier input of every level, [B][m_l] for
//              l = 1..L back to back; reconstruct: (d1hat, d2hat) of every
//              level, [B][m_l/2] twice per level.
#include "wave.hpp"

#include <cmath>

#include "batch.hpp"
#include "kernels.hpp"
#include "ktrace.hpp"

namespace lfft {

namespace {
void check(hipError_t e) {
  if (e != hipSuccess) throw StatusError{E_HIP};
}

struct Bufs {
  float2* F0;
  float2* F1;
  float2* D2;
  float2* FW;
  float2* ST;   // staging of the batched small-level channels
  float2* BD;   // d2hat of the large levels (channel FFTs on the second stream)
  float2* FW2;  // FFT workspace of the second stream
};

Bufs carve(const WavePlan* w, void* ws) {
  float2* base = static_cast<float2*>(ws);
  Bufs b;
  long long bm = w->batch * w->m;
  b.F0 = base;
  b.F1 = base + bm;
  b.D2 = base + bm + bm / 2;
  b.FW = base + 2 * bm;
  b.ST = b.FW + w->fw_elems;
  b.BD = b.ST + w->stage_elems;
  b.FW2 = b.BD + w->bd_elems;
  return b;
}

// Stream of the large levels' channel FFTs: the plan's second stream, or
// the caller's stream for a single-stream plan (everything in issue order).
hipStream_t side_stream(const WavePlan* w, hipStream_t s) { return w->single_stream ? s : w->s2; }

// the side stream starts after everything enqueued on s so far (event e)
void fork(const WavePlan* w, hipEvent_t e, hipStream_t s) {
  if (w->single_stream) return;
  check(hipEventRecord(e, s));
  check(hipStreamWaitEvent(w->s2, e, 0));
}

// s continues after everything enqueued on the side stream so far
void join(const WavePlan* w, hipStream_t s) {
  if (w->single_stream) return;
  check(hipEventRecord(w->ev_join, w->s2));
  check(hipStreamWaitEvent(s, w->ev_join, 0));
}

// The top-level transforms between the signal and the Fourier data of the
// pyramid.  With LWT_SAMPLES the signal holds point values, and the Fourier
// data are those of the orthonormal-translate coefficients: a real diagonal
// factor on G(M^T), (sqrt(m) 2^{r(h)/2})^basis with basis = -1 from samples
// to coefficients and +1 back (the bracket sum of the Dirichlet kernel,
// lfft_basis_change).  The bulk sqrt(m)^basis rides on the FFT's last pass,
// the boundary classes are fixed up on the Fourier side.  basis = 0 (no
// LWT_SAMPLES): the plain transforms.
void top_forward(const WavePlan* w, const float2* x, float2* ahat, float2* fw, long long bin,
                 long long bout, hipStream_t s, int basis) {
  if (!w->samples) basis = 0;
  const float f = basis ? (float)std::pow((double)w->m, 0.5 * basis) : 1.0f;
  exec_lattice(w->fftM, false, false, false, x, ahat, fw, bin, bout, s, f);
  if (basis) scale_boundary(w->fftM, basis, ahat, w->batch, bout, s);
}

// ahat is scaled in place when basis != 0
void top_inverse(const WavePlan* w, float2* ahat, float2* x, float2* fw, long long bin,
                 long long bout, hipStream_t s, int basis) {
  if (!w->samples) basis = 0;
  if (basis) scale_boundary(w->fftM, basis, ahat, w->batch, bin, s);
  const float f = basis ? (float)std::pow((double)w->m, 0.5 * basis) : 1.0f;
  exec_lattice(w->fftM, true, false, false, ahat, x, fw, bin, bout, s, f);
}

// algorithmic bytes of one split/unsplit level: read 8 B and write 8 B per
// complex point and batch element, plus 4 B of mask per point
double split_bytes(long long B, long long ml) { return (16.0 * (double)B + 4.0) * (double)ml; }

long long coeff_offset(const WavePlan* w, int level) {
  long long off = 0;
  for (int l = 0; l < level; ++l) off += w->lv[l].ml / 2;
  return off;
}

// Levels fused into one split/unsplit launch (at most kMaxChain).
constexpr int kChainLevels = 2;

// Fourier data of level l's wavelet channel in the workspace (no `saved`):
// the batched staging area for small levels, the second stream's buffer for
// large ones, D2 otherwise.
float2* d2_slot(const WavePlan* w, const Bufs& b, int l) {
  const bool batched = w->chan_dec != nullptr;
  if (batched && l >= w->small_from) return b.ST + w->stage_lvl[l];
  if (l < w->small_from) return b.BD + w->big_d2[l];
  return b.D2;
}

// Consecutive runs of levels [l0, l0 + K): a run of K > 1 levels needs the
// 32-bit fiber maps on every level and a private d2 slot for each.
std::vector<std::pair<int, int>> level_runs(const WavePlan* w, const Bufs& b) {
  std::vector<std::pair<int, int>> runs;
  int l = 0;
  while (l < w->levels) {
    int k = 0;
    while (l + k < w->levels && k < kChainLevels && w->lv[l + k].sd.narrow &&
           d2_slot(w, b, l + k) != b.D2)
      ++k;
    if (k < 2) k = 1;
    runs.push_back({l, k});
    l += k;
  }
  return runs;
}

SplitChain make_chain(const WavePlan* w, const Bufs& b, const float* const* masks, int l0, int K) {
  SplitChain c{};
  for (int j = 0; j < K; ++j) {
    c.sd[j] = w->lv[l0 + j].sd;
    c.mask[j] = masks[l0 + j];
    c.d2[j] = d2_slot(w, b, l0 + j);
    c.d2_bs[j] = w->lv[l0 + j].ml / 2;
  }
  return c;
}

// algorithmic bytes of a run: the finest input, every level's mask and d2,
// and the coarsest d1
double chain_bytes(const WavePlan* w, int l0, int K) {
  const double B = (double)w->batch;
  double by = 8.0 * B * (double)w->lv[l0].ml;
  for (int j = l0; j < l0 + K; ++j) by += (4.0 + 4.0 * B) * (double)w->lv[j].ml;
  by += 4.0 * B * (double)w->lv[l0 + K - 1].ml;
  return by;
}

const char* chain_name(bool inverse, int K) {
  static const char* fwd[] = {"", "", "split_chain_kernel<2>", "split_chain_kernel<3>",
                              "split_chain_kernel<4>"};
  static const char* inv[] = {"", "", "unsplit_chain_kernel<2>", "unsplit_chain_kernel<3>",
                              "unsplit_chain_kernel<4>"};
  return inverse ? inv[K] : fwd[K];
}

// Decomposition without `saved`: runs of levels fused, the large channels'
// inverse FFTs on the second stream after their run, the small ones batched.
void decompose_runs(const WavePlan* w, const float2* x, const float* const* masks,
                    float2* coeffs, void* ws, hipStream_t s) {
  Bufs b = carve(w, ws);
  const long long B = w->batch, m = w->m;
  const int L = w->levels;
  const bool batched = w->chan_dec != nullptr;
  float2* cur = b.F0;
  top_forward(w, x, cur, b.FW, m, w->lv[0].ml, s, -1);
  bool forked = false;
  const auto runs = level_runs(w, b);
  for (const auto& r : runs) {
    const int l0 = r.first, K = r.second, lt = l0 + K - 1;
    const long long half_t = w->lv[lt].ml / 2;
    float2* next = (batched && lt + 1 == L) ? b.ST + w->stage_d1 : (cur == b.F0 ? b.F1 : b.F0);
    if (K == 1) {
      TraceScope ts("split_kernel", split_bytes(B, w->lv[l0].ml), s);
      check(launch_split(w->lv[l0].sd, B, cur, w->lv[l0].ml, masks[l0], next, d2_slot(w, b, l0),
                         half_t, s));
    } else {
      SplitChain c = make_chain(w, b, masks, l0, K);
      TraceScope ts(chain_name(false, K), chain_bytes(w, l0, K), s);
      check(launch_split_chain(K, c, B, cur, w->lv[l0].ml, next, half_t, s));
    }
    for (int l = l0; l <= lt; ++l) {
      if (l >= w->small_from) continue;
      // large channel: its inverse FFT overlaps the next runs
      if (l == l0) fork(w, w->ev[l], s);
      forked = true;
      exec_lattice(w->lv[l].fftN, true, false, false, b.BD + w->big_d2[l],
                   coeffs + coeff_offset(w, l), b.FW2, w->lv[l].ml / 2, m, side_stream(w, s));
    }
    cur = next;
  }
  if (batched) {
    exec_batch(w->chan_dec, true, BATCH_PERSISTENT, b.ST, coeffs, b.FW, s);
  } else {
    const WaveLevel& VL = w->lv[L - 1];
    exec_lattice(VL.fftN, true, false, false, cur, coeffs + coeff_offset(w, L), b.FW, VL.ml / 2, m,
                 s);
  }
  if (forked) join(w, s);
}

// Reconstruction without `saved`, runs of levels fused (the inverse walk).
void reconstruct_runs(const WavePlan* w, const float2* coeffs, const float* const* masks,
                      float2* x, void* ws, hipStream_t s) {
  Bufs b = carve(w, ws);
  const long long B = w->batch, m = w->m;
  const int L = w->levels;
  const bool batched = w->chan_rec != nullptr;
  const auto runs = level_runs(w, b);
  const int nr = (int)runs.size();
  // run i (0 = finest) writes F0 or F1 alternately upwards from the finest
  // run, which writes F0 for the final inverse FFT (F1 holds B m / 2, enough
  // for every run above level 0)
  auto out_of = [&](int i) { return (i % 2 == 0) ? b.F0 : b.F1; };
  const WaveLevel& VL = w->lv[L - 1];
  float2* cur = batched ? b.ST + w->stage_d1 : (out_of(nr - 1) == b.F0 ? b.F1 : b.F0);
  const bool ahead = w->small_from > 0;
  if (ahead) {
    fork(w, w->ev_join, s);
    for (int l = w->small_from - 1; l >= 0; --l) {
      const WaveLevel& V = w->lv[l];
      exec_lattice(V.fftN, false, false, false, coeffs + coeff_offset(w, l), b.BD + w->big_d2[l],
                   b.FW2, m, V.ml / 2, side_stream(w, s));
      check(hipEventRecord(w->ev[l], side_stream(w, s)));
    }
  }
  if (batched)
    exec_batch(w->chan_rec, false, BATCH_PERSISTENT, coeffs, b.ST, b.FW, s);
  else
    exec_lattice(VL.fftN, false, false, false, coeffs + coeff_offset(w, L), cur, b.FW, m,
                 VL.ml / 2, s);
  for (int i = nr - 1; i >= 0; --i) {
    const int l0 = runs[i].first, K = runs[i].second, lt = l0 + K - 1;
    // large channels come from the second stream (without the batched
    // launch every level is large)
    for (int l = l0; l <= lt; ++l)
      if (l < w->small_from) check(hipStreamWaitEvent(s, w->ev[l], 0));
    float2* next = out_of(i);
    if (K == 1) {
      TraceScope ts("unsplit_kernel", split_bytes(B, w->lv[l0].ml), s);
      check(launch_unsplit(w->lv[l0].sd, B, cur, d2_slot(w, b, l0), w->lv[l0].ml / 2, masks[l0],
                           next, w->lv[l0].ml, s));
    } else {
      SplitChain c = make_chain(w, b, masks, l0, K);
      TraceScope ts(chain_name(true, K), chain_bytes(w, l0, K), s);
      check(launch_unsplit_chain(K, c, B, cur, w->lv[lt].ml / 2, next, w->lv[l0].ml, s));
    }
    cur = next;
  }
  top_inverse(w, cur, x, b.FW, w->lv[0].ml, m, s, +1);
}
}  // namespace

size_t wave_saved_elems(const WavePlan* w) {
  size_t s = 0;
  for (auto& L : w->lv) s += (size_t)(w->batch * L.ml);
  return s;
}

// ---------------------------------------------------------------------------
// q = |det J| > 2: coefficients [B][m] = [lvl 1: ch 1 | .. | ch q-1] ..
// [lvl L: ch 1 | .. | ch q-1] [ch 0 of lvl L], each block in natural sample
// order of N_l.  Workspace: F0 (B m), F1 (B m / q), D (B (q-1) m / q), FW,
// staging.  The levels run in order on the caller's stream; the channels of
// the small levels and the final low-pass channel go through the staging
// area and one batched launch pair, the others through D one level at a time.
namespace {
struct QBufs {
  float2* F0;
  float2* F1;
  float2* D;
  float2* FW;
  float2* ST;
};

QBufs carve_q(const WavePlan* w, void* ws) {
  float2* base = static_cast<float2*>(ws);
  const long long bm = w->batch * w->m;
  QBufs b;
  b.F0 = base;
  b.F1 = base + bm;
  b.D = b.F1 + bm / w->q;
  b.FW = base + 2 * bm;
  b.ST = b.FW + w->fw_elems;
  return b;
}

long long coeff_offset_q(const WavePlan* w, int level) {
  long long off = 0;
  for (int l = 0; l < level; ++l) off += (w->q - 1) * (w->lv[l].ml / w->q);
  return off;
}

// algorithmic bytes of one q-channel split/unsplit level
double split_q_bytes(long long B, long long ml) { return (16.0 * (double)B + 4.0) * (double)ml; }

// buffer written by level l of the synthesis walk (l = L-1 .. 0)
float2* q_target(const QBufs& b, int l) { return l % 2 == 0 ? b.F0 : b.F1; }

// offset of level l's region in `saved`: sum_{j<l} B m_j
std::vector<long long> saved_offsets(const WavePlan* w) {
  std::vector<long long> soff(w->levels, 0);
  long long o = 0;
  for (int l = 0; l < w->levels; ++l) {
    soff[l] = o;
    o += w->batch * w->lv[l].ml;
  }
  return soff;
}

// The analysis walk.  keep: NULL or `saved`, receiving every level's Fourier
// input ahat_l [B][m_l] (for the mask gradients of the decomposition).
// rec_saved / gmasks: as the adjoint of a reconstruction, the mask gradient
// of every level's synthesis from the reconstruction's saved inputs and the
// gradient arriving at its output (the level's input here).
void decompose_q(const WavePlan* w, const float2* x, const float* const* masks, float2* coeffs,
                 void* ws, hipStream_t s, int basis, float2* keep = nullptr,
                 const float2* rec_saved = nullptr, float* const* gmasks = nullptr) {
  QBufs b = carve_q(w, ws);
  const long long B = w->batch, m = w->m, q = w->q;
  const int L = w->levels;
  const bool batched = w->chan_dec != nullptr;
  const std::vector<long long> soff = saved_offsets(w);
  float2* cur = keep ? keep : b.F0;
  top_forward(w, x, cur, b.FW, m, m, s, basis);
  for (int l = 0; l < L; ++l) {
    const WaveLevel& V = w->lv[l];
    const long long n = V.ml / q;
    const bool small = batched && l >= w->small_from;
    float2* next = (batched && l + 1 == L) ? b.ST + w->stage_d1
                   : (keep && l + 1 < L) ? keep + soff[l + 1]
                   : (cur == b.F0 ? b.F1 : b.F0);
    float2* dw = small ? b.ST + w->stage_lvl[l] : b.D;
    if (gmasks && gmasks[l] && rec_saved)
      check(launch_unsplit_q_mask_grad(V.sq, B, rec_saved + soff[l], n, rec_saved + soff[l] + B * n,
                                       (q - 1) * n, masks[l], cur, V.ml, gmasks[l], s));
    {
      TraceScope ts("split_q_kernel", split_q_bytes(B, V.ml), s);
      check(launch_split_q(V.sq, B, cur, V.ml, masks[l], next, n, dw, (q - 1) * n, s));
    }
    if (!small) {
      const long long off = coeff_offset_q(w, l);
      for (long long i = 0; i < B; ++i)
        exec_lattice(V.fftW, true, false, false, b.D + i * (q - 1) * n, coeffs + i * m + off, b.FW,
                     n, n, s);
    }
    cur = next;
  }
  if (batched) {
    exec_batch(w->chan_dec, true, BATCH_PERSISTENT, b.ST, coeffs, b.FW, s);
  } else {
    const WaveLevel& VL = w->lv[L - 1];
    exec_lattice(VL.fftN, true, false, false, cur, coeffs + coeff_offset_q(w, L), b.FW, VL.ml / q,
                 m, s);
  }
}

// The synthesis walk.  dec_saved / gmasks: as the adjoint of a
// decomposition, the mask gradient of every level's split from the
// decomposition's saved inputs and the gradients arriving at its outputs
// (the level's inputs here).
void reconstruct_q(const WavePlan* w, const float2* coeffs, const float* const* masks, float2* x,
                   void* ws, hipStream_t s, int basis, const float2* dec_saved = nullptr,
                   float* const* gmasks = nullptr) {
  QBufs b = carve_q(w, ws);
  const std::vector<long long> soff = saved_offsets(w);
  const long long B = w->batch, m = w->m, q = w->q;
  const int L = w->levels;
  const bool batched = w->chan_rec != nullptr;
  const WaveLevel& VL = w->lv[L - 1];
  float2* cur;
  if (batched) {
    exec_batch(w->chan_rec, false, BATCH_PERSISTENT, coeffs, b.ST, b.FW, s);
    cur = b.ST + w->stage_d1;
  } else {
    cur = q_target(b, L);
    exec_lattice(VL.fftN, false, false, false, coeffs + coeff_offset_q(w, L), cur, b.FW, m,
                 VL.ml / q, s);
  }
  for (int l = L - 1; l >= 0; --l) {
    const WaveLevel& V = w->lv[l];
    const long long n = V.ml / q;
    const bool small = batched && l >= w->small_from;
    float2* dw = small ? b.ST + w->stage_lvl[l] : b.D;
    if (!small) {
      const long long off = coeff_offset_q(w, l);
      for (long long i = 0; i < B; ++i)
        exec_lattice(V.fftW, false, false, false, coeffs + i * m + off, b.D + i * (q - 1) * n, b.FW,
                     n, n, s);
    }
    if (gmasks && gmasks[l] && dec_saved)
      check(launch_split_q_mask_grad(V.sq, B, dec_saved + soff[l], V.ml, masks[l], cur, n, dw,
                                     (q - 1) * n, gmasks[l], s));
    float2* next = q_target(b, l);
    TraceScope ts("unsplit_q_kernel", split_q_bytes(B, V.ml), s);
    check(launch_unsplit_q(V.sq, B, cur, n, dw, (q - 1) * n, masks[l], next, V.ml, s));
    cur = next;
  }
  top_inverse(w, b.F0, x, b.FW, m, m, s, basis);
}

// The synthesis with every level's inputs kept in `saved` (channel 0
// [B][m_l/q], then channels 1 .. q-1 [B][q-1][m_l/q], at offset
// sum_{j<l} B m_j), for the mask gradients of the reconstruction: one level
// at a time, no batched channel launch.
void reconstruct_q_keep(const WavePlan* w, const float2* coeffs, const float* const* masks,
                        float2* x, float2* saved, void* ws, hipStream_t s) {
  QBufs b = carve_q(w, ws);
  const long long B = w->batch, m = w->m, q = w->q;
  const int L = w->levels;
  const std::vector<long long> soff = saved_offsets(w);
  const WaveLevel& VL = w->lv[L - 1];
  float2* cur = saved + soff[L - 1];
  exec_lattice(VL.fftN, false, false, false, coeffs + coeff_offset_q(w, L), cur, b.FW, m,
               VL.ml / q, s);
  for (int l = L - 1; l >= 0; --l) {
    const WaveLevel& V = w->lv[l];
    const long long n = V.ml / q;
    float2* dw = saved + soff[l] + B * n;
    const long long off = coeff_offset_q(w, l);
    for (long long i = 0; i < B; ++i)
      exec_lattice(V.fftW, false, false, false, coeffs + i * m + off, dw + i * (q - 1) * n, b.FW, n,
                   n, s);
    float2* next = l == 0 ? b.F0 : saved + soff[l - 1];
    TraceScope ts("unsplit_q_kernel", split_q_bytes(B, V.ml), s);
    check(launch_unsplit_q(V.sq, B, cur, n, dw, (q - 1) * n, masks[l], next, V.ml, s));
    cur = next;
  }
  top_inverse(w, b.F0, x, b.FW, m, m, s, +1);
}
}  // namespace

void wave_decompose(const WavePlan* w, const float2* x, const float* const* masks, float2* coeffs,
                    float2* saved, void* ws, hipStream_t s) {
  if (w->q != 2) {
    decompose_q(w, x, masks, coeffs, ws, s, -1, saved);
    return;
  }
  if (!saved) {
    decompose_runs(w, x, masks, coeffs, ws, s);
    return;
  }
  // With `saved` (differentiation): one launch per level, the Fourier input
  // of level l kept in saved at offset sum_{j<l} B m_j (batch stride m_l).
  Bufs b = carve(w, ws);
  const long long B = w->batch, m = w->m;
  const int L = w->levels;
  const bool batched = w->chan_dec != nullptr;
  float2* cur = saved;
  top_forward(w, x, cur, b.FW, m, w->lv[0].ml, s, -1);
  long long soff = 0;
  bool forked = false;
  for (int l = 0; l < L; ++l) {
    const WaveLevel& V = w->lv[l];
    const long long half = V.ml / 2;
    float2* next = l + 1 < L ? saved + soff + B * V.ml : (batched ? b.ST + w->stage_d1 : b.F0);
    float2* d2 = d2_slot(w, b, l);
    {
      TraceScope ts("split_kernel", split_bytes(B, V.ml), s);
      check(launch_split(V.sd, B, cur, V.ml, masks[l], next, d2, half, s));
    }
    if (l < w->small_from) {
      // the large channel's FFT overlaps the next splits
      fork(w, w->ev[l], s);
      forked = true;
      exec_lattice(V.fftN, true, false, false, d2, coeffs + coeff_offset(w, l), b.FW2, half, m,
                   side_stream(w, s));
    } else if (!batched) {
      exec_lattice(V.fftN, true, false, false, d2, coeffs + coeff_offset(w, l), b.FW, half, m, s);
    }
    soff += B * V.ml;
    cur = next;
  }
  if (batched) {
    // every small channel and the final low-pass channel in one launch pair
    exec_batch(w->chan_dec, true, BATCH_PERSISTENT, b.ST, coeffs, b.FW, s);
  } else {
    const WaveLevel& VL = w->lv[L - 1];
    exec_lattice(VL.fftN, true, false, false, cur, coeffs + coeff_offset(w, L), b.FW, VL.ml / 2, m,
                 s);
  }
  if (forked) join(w, s);
}

void wave_reconstruct(const WavePlan* w, const float2* coeffs, const float* const* masks,
                      float2* x, float2* saved, void* ws, hipStream_t s) {
  if (w->q != 2) {
    if (saved)
      reconstruct_q_keep(w, coeffs, masks, x, saved, ws, s);
    else
      reconstruct_q(w, coeffs, masks, x, ws, s, +1);
    return;
  }
  if (!saved) {
    reconstruct_runs(w, coeffs, masks, x, ws, s);
    return;
  }
  // With `saved` (differentiation): one stream, one launch per level; the
  // (d1hat, d2hat) of level l are kept in saved at offset sum_{j<l} B m_j.
  Bufs b = carve(w, ws);
  const long long B = w->batch, m = w->m;
  const int L = w->levels;
  std::vector<long long> soff(L, 0);
  {
    long long o = 0;
    for (int l = 0; l < L; ++l) {
      soff[l] = o;
      o += B * w->lv[l].ml;
    }
  }
  const WaveLevel& VL = w->lv[L - 1];
  float2* cur = saved + soff[L - 1];
  exec_lattice(VL.fftN, false, false, false, coeffs + coeff_offset(w, L), cur, b.FW, m, VL.ml / 2,
               s);
  for (int l = L - 1; l >= 0; --l) {
    const WaveLevel& V = w->lv[l];
    const long long half = V.ml / 2;
    float2* d2 = saved + soff[l] + B * half;
    exec_lattice(V.fftN, false, false, false, coeffs + coeff_offset(w, l), d2, b.FW, m, half, s);
    float2* next = l == 0 ? b.F0 : saved + soff[l - 1];
    {
      TraceScope ts("unsplit_kernel", split_bytes(B, V.ml), s);
      check(launch_unsplit(V.sd, B, cur, d2, half, masks[l], next, V.ml, s));
    }
    cur = next;
  }
  top_inverse(w, cur, x, b.FW, w->lv[0].ml, m, s, +1);
}

void wave_decompose_backward(const WavePlan* w, const float2* gc, const float2* saved,
                             const float* const* masks, float2* gx, float* const* gmasks, void* ws,
                             hipStream_t s) {
  if (w->q != 2) {
    // the q-channel split's matrix is real, so the unsplit with the same
    // masks is its adjoint and the synthesis is the adjoint of the analysis
    reconstruct_q(w, gc, masks, gx, ws, s, -1, saved, gmasks);
    return;
  }
  Bufs b = carve(w, ws);
  const long long B = w->batch, m = w->m;
  const int L = w->levels;
  std::vector<long long> soff(L, 0);
  {
    long long o = 0;
    for (int l = 0; l < L; ++l) {
      soff[l] = o;
      o += B * w->lv[l].ml;
    }
  }
  // adjoint of the last inverse FFT is the forward FFT
  const WaveLevel& VL = w->lv[L - 1];
  // ping-pong parity chosen so that level 0 reads F1 and writes F0
  float2* g1 = ((L - 1) % 2 == 0) ? b.F1 : b.F0;
  exec_lattice(VL.fftN, false, false, false, gc + coeff_offset(w, L), g1, b.FW, m, VL.ml / 2, s);
  for (int l = L - 1; l >= 0; --l) {
    const WaveLevel& V = w->lv[l];
    const long long half = V.ml / 2;
    exec_lattice(V.fftN, false, false, false, gc + coeff_offset(w, l), b.D2, b.FW, m, half, s);
    if (gmasks && gmasks[l] && saved)
      check(launch_split_mask_grad(V.sd, B, saved + soff[l], V.ml, g1, b.D2, half, gmasks[l], s));
    float2* next = (l == 0) ? b.F0 : ((g1 == b.F0) ? b.F1 : b.F0);
    // adjoint of the split is the unsplit with the same masks
    check(launch_unsplit(V.sd, B, g1, b.D2, half, masks[l], next, V.ml, s));
    g1 = next;
  }
  // adjoint of the top-level forward transform (with LWT_SAMPLES its real
  // diagonal factor is its own adjoint)
  top_inverse(w, g1, gx, b.FW, w->lv[0].ml, m, s, -1);
}

void wave_reconstruct_backward(const WavePlan* w, const float2* gx, const float2* saved,
                               const float* const* masks, float2* gc, float* const* gmasks,
                               void* ws, hipStream_t s) {
  if (w->q != 2) {
    decompose_q(w, gx, masks, gc, ws, s, +1, nullptr, saved, gmasks);
    return;
  }
  Bufs b = carve(w, ws);
  const long long B = w->batch, m = w->m;
  const int L = w->levels;
  std::vector<long long> soff(L, 0);
  {
    long long o = 0;
    for (int l = 0; l < L; ++l) {
      soff[l] = o;
      o += B * w->lv[l].ml;
    }
  }
  // adjoint of the final inverse FFT is the forward FFT
  float2* g = b.F0;
  top_forward(w, gx, g, b.FW, m, w->lv[0].ml, s, +1);
  for (int l = 0; l < L; ++l) {
    const WaveLevel& V = w->lv[l];
    const long long half = V.ml / 2;
    if (gmasks && gmasks[l] && saved)
      check(launch_unsplit_mask_grad(V.sd, B, saved + soff[l], saved + soff[l] + B * half, half, g,
                                     V.ml, gmasks[l], s));
    float2* next = (g == b.F0) ? b.F1 : b.F0;
    // adjoint of the unsplit is the split with the same masks
    check(launch_split(V.sd, B, g, V.ml, masks[l], next, b.D2, half, s));
    exec_lattice(V.fftN, true, false, false, b.D2, gc + coeff_offset(w, l), b.FW, half, m, s);
    g = next;
  }
  const WaveLevel& VL = w->lv[L - 1];
  exec_lattice(VL.fftN, true, false, false, g, gc + coeff_offset(w, L), b.FW, VL.ml / 2, m, s);
}

}  // namespace lfft
