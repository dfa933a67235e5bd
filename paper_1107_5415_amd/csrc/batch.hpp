// Host side of the batched lattice FFT: many signals on patterns of
// different M, executed by per-lattice launches, by the two-phase persistent
// launch, or by a captured graph of it; plus the autotuner that picks the
// tile size and the pass/radix order.
#pragma once
#include <hip/hip_runtime.h>

#include <cstdint>
#include <map>
#include <tuple>
#include <vector>

#include "plan.hpp"

namespace lfft {

enum BatchMode : int { BATCH_LOOP = 0, BATCH_PERSISTENT = 1, BATCH_GRAPH = 2 };

struct BatchDir {
  void* dpass = nullptr;      // BatchPass[npass]
  void* ditems = nullptr;     // int2[nitems] followed by qbeg[17]
  int npass = 0, nitems = 0;
  int phase_items[2] = {0, 0};
  const int* qbeg = nullptr;  // device: queue x of phase p is [qbeg[8p + x], qbeg[8p + x + 1])
};

struct BatchPlan {
  int count = 0, d = 0;
  std::vector<i64> Ms;                  // count * d * d, row-major per lattice
  std::vector<i64> m, off;              // off: count + 1 prefix offsets
  // element offsets of every lattice's signal in the input, output and
  // workspace buffers (the public plan uses off[i] for all three)
  std::vector<i64> in_off, out_off, ws_off;
  i64 total = 0;
  uint32_t flags = 0;
  int tile_lg = 12, order = 0;
  bool configured = false;
  std::vector<LatticePlan*> tiled;      // fixed-tile plans (nullptr: not eligible)
  std::vector<LatticePlan*> single;     // default plans, built on first per-lattice use
  int eligible = 0;
  BatchDir dir[2];                      // forward, inverse
  int* dheads = nullptr;                // 16 queue heads (8 per phase), kHeadStride apart
  int grid = 0;
  hipStream_t cap = nullptr;            // private stream for graph capture
  std::map<std::tuple<int, const void*, void*, void*>, hipGraphExec_t> graphs;
  size_t ws_elems = 0;
  // lattices through their own plan whose workspace exceeds their slot (a
  // chirp-z axis) share one region of extra_ws elements after ws_elems
  size_t extra_ws = 0;
};

BatchPlan* build_batch_plan(int count, int d, const i64* Ms, uint32_t flags);
// Same with explicit per-lattice offsets (in, out and workspace elements; the
// workspace slot of lattice i holds m_i elements); ws_elems = workspace size.
BatchPlan* build_batch_plan_at(int count, int d, const i64* Ms, const i64* in_off,
                               const i64* out_off, const i64* ws_off, size_t ws_elems,
                               uint32_t flags, int tile_lg, int order);
void free_batch_plan(BatchPlan* b);
// (Re)build the fixed-tile schedules and device queues for one configuration.
void configure_batch(BatchPlan* b, int tile_lg, int order);
void exec_batch(BatchPlan* b, bool inverse, int mode, const void* in, void* out, void* ws,
                hipStream_t s);
// Times every candidate configuration on the caller's buffers (persistent
// mode) and keeps the fastest; results are cached per set of matrices.
void tune_batch(BatchPlan* b, const void* in, void* out, void* ws, int reps, hipStream_t s,
                float* best_ms);

}  // namespace lfft
