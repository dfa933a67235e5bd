// extern "C" boundary of liblfft.so (declarations and contracts in
// include/lfft.h).  Converts every internal error into a status code.
#include "lfft.h"

#include <cmath>
#include <new>

#include "batch.hpp"
#include "handles.hpp"
#include "planlog.hpp"
#include "tune_cache.hpp"
#include "plan.hpp"
#include "wave.hpp"

namespace {

template <class F>
int guarded(F&& f) {
  try {
    f();
    return LFFT_OK;
  } catch (const lfft::StatusError& e) {
    return e.code;
  } catch (const lfft::IntOverflow&) {
    return LFFT_E_OVERFLOW;
  } catch (const lfft::SingularMatrix&) {
    return LFFT_E_SINGULAR;
  } catch (const lfft::NotIntegral&) {
    return LFFT_E_NOT_INTEGRAL;
  } catch (const std::bad_alloc&) {
    return LFFT_E_NOMEM;
  } catch (...) {
    return LFFT_E_STATE;
  }
}

void put(const lfft::Mat& A, int64_t* out) {
  if (!out) return;
  for (int i = 0; i < A.d; ++i)
    for (int j = 0; j < A.d; ++j) out[i * A.d + j] = A.a[i][j];
}

bool device_ready(const lfft::LatticePlan* p) { return p->dtab != nullptr; }

int run_lattice(lfft_plan_t plan, bool inverse, const void* in, void* out, void* ws,
                uint32_t layout, hipStream_t stream) {
  if (!plan || !plan->p || !in || !out || in == out) return LFFT_E_ARG;
  if (layout & ~(LFFT_IN_GRID | LFFT_OUT_GRID)) return LFFT_E_ARG;
  const lfft::LatticePlan* p = plan->p;
  if (!device_ready(p)) return LFFT_E_STATE;
  if (p->ws_elems && !ws) return LFFT_E_ARG;
  return guarded([&] {
    lfft::exec_lattice(p, inverse, (layout & LFFT_IN_GRID) != 0, (layout & LFFT_OUT_GRID) != 0, in,
                       out, ws, p->m, p->m, stream);
  });
}

}  // namespace

extern "C" {

int lfft_plan_create(lfft_plan_t* plan, int d, const int64_t* M, int64_t batch, uint32_t flags) {
  if (!plan) return LFFT_E_ARG;
  *plan = nullptr;
  if (flags & ~(LFFT_HOST_ONLY | LFFT_SPLIT_BF16)) return LFFT_E_ARG;
  if (d > lfft::kMaxD) return LFFT_E_UNSUPPORTED;
  lfft::LatticePlan* p = nullptr;
  int st = guarded([&] { p = lfft::build_lattice_plan(d, M, batch, flags); });
  if (st != LFFT_OK) return st;
  if (!(flags & LFFT_HOST_ONLY)) {
    st = guarded([&] { lfft::upload_plan(p); });
    if (st != LFFT_OK) {
      lfft::free_plan(p);
      return st;
    }
  }
  *plan = new (std::nothrow) lfft_plan_s{p};
  if (!*plan) {
    lfft::free_plan(p);
    return LFFT_E_NOMEM;
  }
  lfft::log_lattice_plan(p, "plan");
  return LFFT_OK;
}

int lfft_plan_destroy(lfft_plan_t plan) {
  if (!plan) return LFFT_OK;
  lfft::free_plan(plan->p);
  delete plan;
  return LFFT_OK;
}

int lfft_plan_query(lfft_plan_t plan, int64_t* m, int* d_M, int64_t* eps, int64_t* Q, int64_t* R,
                    int64_t* H_M, int64_t* H_MT) {
  if (!plan || !plan->p) return LFFT_E_ARG;
  const lfft::LatticePlan* p = plan->p;
  if (m) *m = p->m;
  if (d_M) *d_M = (int)p->eps.size();
  if (eps)
    for (int i = 0; i < p->d; ++i) eps[i] = p->Sf.eps[i];
  put(p->Sf.Q, Q);
  put(p->Sf.R, R);
  put(p->HM, H_M);
  put(p->HMT, H_MT);
  return LFFT_OK;
}

int lfft_plan_query_inverse_basis(lfft_plan_t plan, int64_t* Qt, int64_t* Rt) {
  if (!plan || !plan->p) return LFFT_E_ARG;
  put(plan->p->Si.Q, Qt);
  put(plan->p->Si.R, Rt);
  return LFFT_OK;
}

int lfft_plan_info(lfft_plan_t plan, int* passes, int* aligned_forward, int* aligned_inverse) {
  if (!plan || !plan->p) return LFFT_E_ARG;
  if (passes) *passes = (int)plan->p->ranges.size();
  if (aligned_forward) *aligned_forward = plan->p->Sf_aligned ? 1 : 0;
  if (aligned_inverse) *aligned_inverse = plan->p->Si_aligned ? 1 : 0;
  return LFFT_OK;
}

int lfft_index_map(lfft_plan_t plan, int which, int64_t* natural_to_grid) {
  if (!plan || !plan->p || !natural_to_grid || which < 0 || which > 3) return LFFT_E_ARG;
  return guarded([&] { lfft::natural_to_grid(plan->p, which, natural_to_grid); });
}

int lfft_points(lfft_plan_t plan, int which, int64_t* keys, int64_t* sym_num) {
  if (!plan || !plan->p || which < 0 || which > 1) return LFFT_E_ARG;
  return guarded([&] { lfft::points(plan->p, which, keys, sym_num); });
}

size_t lfft_workspace_size(lfft_plan_t plan) {
  if (!plan || !plan->p) return 0;
  return plan->p->ws_elems * 8;
}

int lfft_forward(lfft_plan_t plan, const void* in, void* out, void* workspace, uint32_t layout,
                 hipStream_t stream) {
  return run_lattice(plan, false, in, out, workspace, layout, stream);
}

int lfft_inverse(lfft_plan_t plan, const void* in, void* out, void* workspace, uint32_t layout,
                 hipStream_t stream) {
  return run_lattice(plan, true, in, out, workspace, layout, stream);
}

size_t lfft_basis_workspace_size(lfft_plan_t plan) {
  if (!plan || !plan->p) return 0;
  return (plan->p->ws_elems + (size_t)(plan->p->batch * plan->p->m)) * 8;
}

int lfft_basis_change(lfft_plan_t plan, int direction, int fourier, const void* in, void* out,
                      void* workspace, hipStream_t stream) {
  if (!plan || !plan->p || !in || !out || in == out || !workspace) return LFFT_E_ARG;
  if (direction != LFFT_SAMPLES_TO_COEFFS && direction != LFFT_COEFFS_TO_SAMPLES) return LFFT_E_ARG;
  lfft::LatticePlan* p = plan->p;
  if (!device_ready(p)) return LFFT_E_STATE;
  return guarded([&] {
    lfft::build_boundary(p);
    const long long bm = p->batch * p->m;
    float2* fw = static_cast<float2*>(workspace);
    float2* T = fw + p->ws_elems;
    const float rsm = (float)(1.0 / std::sqrt((double)p->m));
    const float sm = (float)std::sqrt((double)p->m);
    if (direction == LFFT_SAMPLES_TO_COEFFS) {
      // ahat = F(M) s / (sqrt(m) 2^{r/2}); a = F(M)^{-1} ahat
      float2* dst = fourier ? static_cast<float2*>(out) : T;
      lfft::exec_lattice(p, false, false, false, in, dst, fw, p->m, p->m, stream, rsm);
      lfft::scale_boundary(p, -1, dst, p->batch, p->m, stream);
      if (!fourier) lfft::exec_lattice(p, true, false, false, T, out, fw, p->m, p->m, stream);
    } else {
      // s = F(M)^{-1} (sqrt(m) 2^{r/2} ahat), ahat = F(M) a
      if (fourier) {
        if (hipMemcpyAsync(T, in, (size_t)bm * 8, hipMemcpyDeviceToDevice, stream) != hipSuccess)
          throw lfft::StatusError{LFFT_E_HIP};
      } else {
        lfft::exec_lattice(p, false, false, false, in, T, fw, p->m, p->m, stream);
      }
      lfft::scale_boundary(p, +1, T, p->batch, p->m, stream);
      lfft::exec_lattice(p, true, false, false, T, out, fw, p->m, p->m, stream, sm);
    }
  });
}

int lwt_plan_create(lwt_plan_t* plan, int d, const int64_t* M, const int64_t* J, int levels,
                    int64_t batch, uint32_t flags) {
  if (!plan) return LFFT_E_ARG;
  *plan = nullptr;
  if (flags & ~(LFFT_HOST_ONLY | LWT_SINGLE_STREAM | LWT_SAMPLES)) return LFFT_E_ARG;
  if (d > lfft::kMaxD) return LFFT_E_UNSUPPORTED;
  lfft::WavePlan* w = nullptr;
  int st = guarded([&] { w = lfft::build_wave_plan(d, M, J, levels, batch, flags); });
  if (st != LFFT_OK) return st;
  if (!(flags & LFFT_HOST_ONLY)) {
    st = guarded([&] { lfft::upload_wave_plan(w); });
    if (st != LFFT_OK) {
      lfft::free_wave_plan(w);
      return st;
    }
  }
  *plan = new (std::nothrow) lwt_plan_s{w};
  if (!*plan) {
    lfft::free_wave_plan(w);
    return LFFT_E_NOMEM;
  }
  lfft::log_wave_plan(w);
  return LFFT_OK;
}

int lwt_plan_destroy(lwt_plan_t plan) {
  if (!plan) return LFFT_OK;
  lfft::free_wave_plan(plan->w);
  delete plan;
  return LFFT_OK;
}

int lwt_level_info(lwt_plan_t plan, int level, int64_t* N, int64_t* m_level, int64_t* eps_N) {
  if (!plan || !plan->w || level < 0 || level >= plan->w->levels) return LFFT_E_ARG;
  const lfft::WaveLevel& L = plan->w->lv[level];
  put(L.Nl, N);
  if (m_level) *m_level = L.ml;
  if (eps_N)
    for (int i = 0; i < plan->w->d; ++i) eps_N[i] = L.fftN->Sf.eps[i];
  return LFFT_OK;
}

int lwt_level_scaling(lwt_plan_t plan, int level, int* d_M, int* d_N, int64_t* key,
                      int64_t* grid) {
  if (!plan || !plan->w || level < 0 || level >= plan->w->levels) return LFFT_E_ARG;
  int dm = 0, dn = 0;
  lfft::i64 k[lfft::kMaxD] = {}, g[lfft::kMaxD] = {};
  const int st = guarded([&] { lfft::level_scaling(plan->w, level, dm, dn, k, g); });
  if (st != LFFT_OK) return st;
  if (d_M) *d_M = dm;
  if (d_N) *d_N = dn;
  for (int i = 0; i < plan->w->d; ++i) {
    if (key) key[i] = k[i];
    if (grid) grid[i] = g[i];
  }
  return LFFT_OK;
}

int lwt_fiber_map(lwt_plan_t plan, int level, int path, int64_t k0, int64_t count,
                  int64_t* lifts, int64_t* phase) {
  if (!plan || !plan->w) return LFFT_E_ARG;
  return guarded([&] { lfft::fiber_map(plan->w, level, path, k0, count, lifts, phase); });
}

int lwt_coeff_layout(lwt_plan_t plan, int* q, int* nblocks, int64_t* offset, int64_t* length,
                     int* level, int* channel) {
  if (!plan || !plan->w) return LFFT_E_ARG;
  const lfft::WavePlan* w = plan->w;
  if (q) *q = w->q;
  if (nblocks) *nblocks = w->levels * (w->q - 1) + 1;
  int64_t off = 0;
  int b = 0;
  auto put_block = [&](int l, int j, int64_t n) {
    if (offset) offset[b] = off;
    if (length) length[b] = n;
    if (level) level[b] = l;
    if (channel) channel[b] = j;
    off += n;
    ++b;
  };
  for (int l = 0; l < w->levels; ++l)
    for (int j = 1; j < w->q; ++j) put_block(l, j, w->lv[l].ml / w->q);
  put_block(w->levels - 1, 0, w->lv[w->levels - 1].ml / w->q);
  return LFFT_OK;
}

int lwt_dirichlet_mask(lwt_plan_t plan, int level, float* mask) {
  if (!plan || !plan->w || !mask || level < 0 || level >= plan->w->levels) return LFFT_E_ARG;
  return guarded([&] { lfft::dirichlet_mask(plan->w, level, mask); });
}

size_t lwt_workspace_size(lwt_plan_t plan) {
  if (!plan || !plan->w) return 0;
  return plan->w->ws_elems * 8;
}

size_t lwt_saved_elems(lwt_plan_t plan) {
  if (!plan || !plan->w) return 0;
  return lfft::wave_saved_elems(plan->w);
}

#define LWT_CHECK(plan, ws)                                  \
  if (!plan || !plan->w) return LFFT_E_ARG;                  \
  if (!plan->w->uploaded) return LFFT_E_STATE;                \
  if (!ws) return LFFT_E_ARG;

int lwt_decompose(lwt_plan_t plan, const void* samples, const float* const* masks, void* coeffs,
                  void* saved, void* workspace, hipStream_t stream) {
  LWT_CHECK(plan, workspace);
  if (!samples || !coeffs || !masks || samples == coeffs) return LFFT_E_ARG;
  for (int l = 0; l < plan->w->levels; ++l)
    if (!masks[l]) return LFFT_E_ARG;
  return guarded([&] {
    lfft::wave_decompose(plan->w, static_cast<const float2*>(samples), masks,
                         static_cast<float2*>(coeffs), static_cast<float2*>(saved), workspace,
                         stream);
  });
}

int lwt_reconstruct(lwt_plan_t plan, const void* coeffs, const float* const* masks, void* samples,
                    void* saved, void* workspace, hipStream_t stream) {
  LWT_CHECK(plan, workspace);
  if (!samples || !coeffs || !masks || samples == coeffs) return LFFT_E_ARG;
  for (int l = 0; l < plan->w->levels; ++l)
    if (!masks[l]) return LFFT_E_ARG;
  return guarded([&] {
    lfft::wave_reconstruct(plan->w, static_cast<const float2*>(coeffs), masks,
                           static_cast<float2*>(samples), static_cast<float2*>(saved), workspace,
                           stream);
  });
}

int lwt_decompose_backward(lwt_plan_t plan, const void* grad_coeffs, const void* saved,
                           const float* const* masks, void* grad_samples, float* const* grad_masks,
                           void* workspace, hipStream_t stream) {
  LWT_CHECK(plan, workspace);
  if (!grad_coeffs || !grad_samples || !masks || grad_coeffs == grad_samples) return LFFT_E_ARG;
  if (grad_masks && !saved) return LFFT_E_ARG;
  return guarded([&] {
    lfft::wave_decompose_backward(plan->w, static_cast<const float2*>(grad_coeffs),
                                  static_cast<const float2*>(saved), masks,
                                  static_cast<float2*>(grad_samples), grad_masks, workspace, stream);
  });
}

int lwt_reconstruct_backward(lwt_plan_t plan, const void* grad_samples, const void* saved,
                             const float* const* masks, void* grad_coeffs,
                             float* const* grad_masks, void* workspace, hipStream_t stream) {
  LWT_CHECK(plan, workspace);
  if (!grad_coeffs || !grad_samples || !masks || grad_coeffs == grad_samples) return LFFT_E_ARG;
  if (grad_masks && !saved) return LFFT_E_ARG;
  return guarded([&] {
    lfft::wave_reconstruct_backward(plan->w, static_cast<const float2*>(grad_samples),
                                    static_cast<const float2*>(saved), masks,
                                    static_cast<float2*>(grad_coeffs), grad_masks, workspace,
                                    stream);
  });
}

int lfft_batch_create(lfft_batch_t* plan, int count, int d, const int64_t* Ms, uint32_t flags) {
  if (!plan) return LFFT_E_ARG;
  *plan = nullptr;
  if (flags & ~LFFT_HOST_ONLY) return LFFT_E_ARG;
  if (d > lfft::kMaxD) return LFFT_E_UNSUPPORTED;
  lfft::BatchPlan* b = nullptr;
  int st = guarded([&] { b = lfft::build_batch_plan(count, d, Ms, flags); });
  if (st != LFFT_OK) return st;
  *plan = new (std::nothrow) lfft_batch_s{b};
  if (!*plan) {
    lfft::free_batch_plan(b);
    return LFFT_E_NOMEM;
  }
  lfft::log_batch_plan(b, "batch");
  return LFFT_OK;
}

int lfft_batch_destroy(lfft_batch_t plan) {
  if (!plan) return LFFT_OK;
  lfft::free_batch_plan(plan->b);
  delete plan;
  return LFFT_OK;
}

int lfft_batch_offsets(lfft_batch_t plan, int64_t* offsets) {
  if (!plan || !offsets) return LFFT_E_ARG;
  for (size_t i = 0; i < plan->b->off.size(); ++i) offsets[i] = plan->b->off[i];
  return LFFT_OK;
}

size_t lfft_batch_workspace_size(lfft_batch_t plan) {
  if (!plan) return 0;
  return (plan->b->ws_elems + plan->b->extra_ws) * 8;
}

int lfft_batch_configure(lfft_batch_t plan, int tile_lg, int order) {
  if (!plan) return LFFT_E_ARG;
  return guarded([&] {
    lfft::configure_batch(plan->b, tile_lg, order);
    lfft::log_batch_plan(plan->b, "batch configured:");
  });
}

int lfft_batch_config(lfft_batch_t plan, int* tile_lg, int* order, int* eligible) {
  if (!plan) return LFFT_E_ARG;
  if (tile_lg) *tile_lg = plan->b->tile_lg;
  if (order) *order = plan->b->order;
  if (eligible) *eligible = plan->b->eligible;
  return LFFT_OK;
}

int lfft_batch_schedule(lfft_batch_t plan, int i, int* passes, int64_t* pencil, int64_t* tiles,
                        int* post) {
  if (!plan || i < 0 || i >= plan->b->count || !passes) return LFFT_E_ARG;
  const lfft::LatticePlan* p = plan->b->tiled[i];
  *passes = p ? (int)p->fwd.passes.size() : 0;
  if (!p) return LFFT_OK;
  for (int k = 0; k < *passes && k < 2; ++k) {
    const lfft::PassDesc& pd = p->fwd.passes[k];
    if (pencil) pencil[k] = pd.L;
    if (tiles) tiles[k] = ((int64_t)pd.O * pd.S + pd.W - 1) / pd.W;
    if (post) post[k] = pd.post;
  }
  return LFFT_OK;
}

int lfft_batch_tune(lfft_batch_t plan, const void* in, void* out, void* workspace, int reps,
                    float* best_ms, hipStream_t stream) {
  if (!plan || !in || !out || in == out || !workspace || reps < 1) return LFFT_E_ARG;
  if (!plan->b->dheads) return LFFT_E_STATE;
  return guarded([&] {
    lfft::tune_batch(plan->b, in, out, workspace, reps, stream, best_ms);
    lfft::log_batch_plan(plan->b, "batch tuned:");
  });
}

int lfft_batch_tune_save(const char* path) {
  if (!path || !*path) return LFFT_E_ARG;
  return guarded([&] { lfft::tune_cache_save(path); });
}

int lfft_batch_tune_load(const char* path, const char* arch, int* loaded) {
  if (!path || !*path) return LFFT_E_ARG;
  return guarded([&] {
    const std::string a = arch ? std::string(arch) : lfft::device_arch();
    const int n = lfft::tune_cache_load(path, a);
    if (loaded) *loaded = n;
  });
}

int lfft_batch_tune_clear(int* count) {
  if (count) *count = lfft::tune_cache_size();
  lfft::tune_cache_clear();
  return LFFT_OK;
}

int lfft_batch_execute(lfft_batch_t plan, int inverse, int mode, const void* in, void* out,
                       void* workspace, hipStream_t stream) {
  if (!plan || !in || !out || in == out || !workspace) return LFFT_E_ARG;
  if (mode < LFFT_BATCH_LOOP || mode > LFFT_BATCH_GRAPH) return LFFT_E_ARG;
  if (!plan->b->dheads) return LFFT_E_STATE;
  return guarded([&] { lfft::exec_batch(plan->b, inverse != 0, mode, in, out, workspace, stream); });
}

const char* lfft_strerror(int status) {
  switch (status) {
    case LFFT_OK: return "ok";
    case LFFT_E_ARG: return "invalid argument";
    case LFFT_E_SINGULAR: return "singular matrix (det M = 0)";
    case LFFT_E_NOT_INTEGRAL: return "J^{-1} M is not an integer matrix";
    case LFFT_E_OVERFLOW: return "exact integer arithmetic would overflow int64";
    case LFFT_E_UNSUPPORTED: return "unsupported size or dilation";
    case LFFT_E_HIP: return "HIP runtime error";
    case LFFT_E_NOMEM: return "device allocation failed";
    case LFFT_E_STATE: return "invalid plan state";
    case LFFT_E_IO: return "file not readable or writable, or not a tuning cache";
    default: return "unknown status";
  }
}

}  // extern "C"
