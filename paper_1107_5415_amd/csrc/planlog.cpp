// Plan log: with the environment variable LFFT_LOG set to anything but "0",
// every plan the C ABI creates prints its schedule to stderr, one line per
// plan and per pass: the grid (elementary divisors), the pass count, and for
// each pass of the natural-order forward and inverse transforms the kernel
// that runs it with its pencil shape.  Nothing is printed otherwise.
#include "planlog.hpp"

#include <cstdio>
#include <cstdlib>
#include <cstring>
#include <string>

#include "batch.hpp"
#include "kernels.hpp"

namespace lfft {

namespace {

std::string eps_str(const std::vector<i64>& eps) {
  std::string s;
  for (size_t i = 0; i < eps.size(); ++i) s += (i ? "x" : "") + std::to_string(eps[i]);
  return s.empty() ? "1" : s;
}

void log_engine(const LatticePlan* p, const Engine& E, const char* what) {
  const int np = (int)E.passes.size();
  for (int i = 0; i < np; ++i) {
    PassDesc pd = E.passes[i];
    if (i == 0) pd.in = E.in_nat;
    if (i == np - 1) pd.out = E.out_nat;
    if (pd.kind == 4) {
      std::fprintf(stderr, "lfft:   %-8s pass %d/%d chirp-z axis of %d points (convolution %d) x %lld\n",
                   what, i + 1, np, pd.L, pd.bN, (long long)(p->batch * pd.O * pd.S));
      continue;
    }
    // the streaming kernel runs its own compile-time radix sequence; the
    // other kernels run the descriptor's stages
    char stages[32] = "";
    if (pd.kind != 2) std::snprintf(stages, sizeof stages, ", %d stages", pd.nst);
    std::fprintf(stderr, "lfft:   %-8s pass %d/%d %s pencil %d x %d per tile%s, O=%d S=%d%s%s%s%s%s\n",
                 what, i + 1, np, pass_kernel_name(pd), pd.L, pd.W, stages, pd.O, pd.S,
                 pd.post ? ", four-step twiddle" : "", pd.in.mode == MAP_NATURAL ? ", natural in" : "",
                 pd.out.mode == MAP_NATURAL ? ", natural out" : "",
                 pd.stream_in ? " (non-temporal loads)" : "",
                 pd.stream_out ? " (non-temporal stores)" : "");
  }
}

}  // namespace

bool plan_log_on() {
  static const bool on = [] {
    const char* v = std::getenv("LFFT_LOG");
    return v && *v && std::strcmp(v, "0") != 0;
  }();
  return on;
}

void log_lattice_plan(const LatticePlan* p, const char* label) {
  if (!p || !plan_log_on()) return;
  std::fprintf(stderr, "lfft: %s d=%d m=%lld batch=%lld eps=%s passes=%d basis%s%s%s\n", label,
               p->d, (long long)p->m, (long long)p->batch, eps_str(p->eps).c_str(),
               (int)p->fwd.passes.size(), p->Sf_aligned ? " forward-aligned" : "",
               p->Si_aligned ? " inverse-aligned" : "",
               (p->flags & kPlanSplitBf16) ? " split-bf16" : "");
  log_engine(p, p->has_fwd_rev ? p->fwd_rev : p->fwd, "forward");
  log_engine(p, p->has_inv_rev ? p->inv_rev : p->inv_nat, "inverse");
}

void log_wave_plan(const WavePlan* w) {
  if (!w || !plan_log_on()) return;
  std::fprintf(stderr,
               "lfft: pyramid d=%d m=%lld batch=%lld q=%d levels=%d channels batched from level "
               "%d%s%s\n",
               w->d, (long long)w->m, (long long)w->batch, w->q, w->levels, w->small_from,
               w->single_stream ? ", one stream" : "", w->samples ? ", point values" : "");
  log_lattice_plan(w->fftM, "top FFT");
  for (int l = 0; l < w->levels; ++l) {
    const WaveLevel& L = w->lv[l];
    std::fprintf(stderr, "lfft:   level %d m=%lld channel eps=%s%s\n", l, (long long)L.ml,
                 eps_str(L.fftN->eps).c_str(),
                 l >= w->small_from ? " (batched)" : (w->q == 2 ? " (second stream)" : ""));
  }
}

void log_batch_plan(const BatchPlan* b, const char* label) {
  if (!b || !plan_log_on()) return;
  std::fprintf(stderr,
               "lfft: %s lattices=%d d=%d points=%lld in the persistent launch %d, tile 2^%d, "
               "order %d\n",
               label, b->count, b->d, (long long)b->total, b->eligible, b->tile_lg, b->order);
}

}  // namespace lfft
