// Batched lattice FFT host logic (see batch.hpp).
#include "batch.hpp"

#include <algorithm>
#include <cstring>
#include <mutex>
#include <numeric>

#include "kernels.hpp"
#include "ktrace.hpp"
#include "tune_cache.hpp"

namespace lfft {

namespace {

i64 pass_tiles(const PassDesc& pd) {
  const i64 npen = pd.batch * (i64)pd.O * pd.S;
  return (npen + pd.W - 1) / pd.W;
}

int variant_of(const PassDesc& pd, bool first, bool last) {
  const bool cols = pd.S > 1;
  if (first && last) return BATCH_ROWS_NN;
  if (first) return cols ? BATCH_COLS_NI : BATCH_ROWS_NI;
  return cols ? BATCH_COLS_IN : BATCH_ROWS_IN;
}

void free_dir(BatchDir& D) {
  if (D.dpass) (void)hipFree(D.dpass);
  if (D.ditems) (void)hipFree(D.ditems);
  D = BatchDir{};
}

void drop_graphs(BatchPlan* b) {
  for (auto& kv : b->graphs) (void)hipGraphExecDestroy(kv.second);
  b->graphs.clear();
}

void drop_tiled(BatchPlan* b) {
  for (auto* p : b->tiled) free_plan(p);
  b->tiled.clear();
  for (auto& D : b->dir) free_dir(D);
  drop_graphs(b);
  b->configured = false;
}

template <class T>
void* upload(const std::vector<T>& v) {
  void* d = nullptr;
  const size_t n = std::max<size_t>(1, v.size() * sizeof(T));
  if (hipMalloc(&d, n) != hipSuccess) throw StatusError{E_NOMEM};
  if (!v.empty() && hipMemcpy(d, v.data(), v.size() * sizeof(T), hipMemcpyHostToDevice) != hipSuccess) {
    (void)hipFree(d);
    throw StatusError{E_HIP};
  }
  return d;
}

// Fill the eight XCD queues of both phases of one direction: phase 0 holds
// the first pass of every lattice, phase 1 the second pass of the lattices
// that need two.  Lattices go to queues by longest-processing-time
// assignment, largest first inside a queue.
void build_dir(BatchPlan* b, bool inverse, BatchDir& D) {
  std::vector<BatchPass> passes;
  struct Inst {
    int first;      // index of its first BatchPass
    int np;
    i64 work;
  };
  std::vector<Inst> insts;
  for (int i = 0; i < b->count; ++i) {
    LatticePlan* p = b->tiled[i];
    if (!p) continue;
    const Engine& E = inverse ? (p->has_inv_rev ? p->inv_rev : p->inv_nat) : p->fwd;
    const int np = (int)E.passes.size();
    if (np < 1 || np > 2) throw StatusError{E_STATE};
    Inst in{(int)passes.size(), np, b->m[i]};
    for (int k = 0; k < np; ++k) {
      BatchPass bp{};
      bp.pd = E.passes[k];
      bp.pd.batch = 1;
      bp.pd.in.bstride = b->m[i];
      bp.pd.out.bstride = b->m[i];
      const bool first = k == 0, last = k == np - 1;
      if (first) {
        bp.pd.in = E.in_nat;
        bp.pd.in.bstride = b->m[i];
      }
      if (last) {
        bp.pd.out = E.out_nat;
        bp.pd.out.bstride = b->m[i];
      }
      if (bp.pd.kind != 1 || bp.pd.P != 16 || bp.pd.split ||
          (i64)bp.pd.W * bp.pd.L != (i64(1) << b->tile_lg))
        throw StatusError{E_STATE};
      bp.in_off = first ? b->in_off[i] : b->ws_off[i];
      bp.out_off = last ? b->out_off[i] : b->ws_off[i];
      bp.in_buf = first ? 0 : 2;
      bp.out_buf = last ? 1 : 2;
      bp.variant = variant_of(bp.pd, first, last);
      passes.push_back(bp);
    }
    insts.push_back(in);
  }
  std::vector<int> order(insts.size());
  std::iota(order.begin(), order.end(), 0);
  std::stable_sort(order.begin(), order.end(),
                   [&](int x, int y) { return insts[x].work > insts[y].work; });
  std::vector<std::vector<int>> q(8);
  std::vector<i64> load(8, 0);
  for (int k : order) {
    int best = (int)(std::min_element(load.begin(), load.end()) - load.begin());
    q[best].push_back(k);
    load[best] += insts[k].work;
  }
  std::vector<int2> items;
  std::vector<int> qbeg(17, 0);
  for (int ph = 0; ph < 2; ++ph) {
    for (int x = 0; x < 8; ++x) {
      qbeg[8 * ph + x] = (int)items.size();
      for (int k : q[x]) {
        const Inst& I = insts[k];
        if (ph >= I.np) continue;
        const int pi = I.first + ph;
        const i64 nt = pass_tiles(passes[pi].pd);
        for (i64 t = 0; t < nt; ++t) items.push_back(make_int2(pi, (int)t));
      }
    }
    D.phase_items[ph] = (int)items.size() - qbeg[8 * ph];
  }
  qbeg[16] = (int)items.size();
  if (items.size() > (size_t)0x7fffffff) throw StatusError{E_UNSUPPORTED};
  D.npass = (int)passes.size();
  D.nitems = (int)items.size();
  D.dpass = upload(passes);
  std::vector<uint8_t> blob(items.size() * sizeof(int2) + 17 * sizeof(int));
  std::memcpy(blob.data(), items.data(), items.size() * sizeof(int2));
  std::memcpy(blob.data() + items.size() * sizeof(int2), qbeg.data(), 17 * sizeof(int));
  D.ditems = upload(blob);
  D.qbeg = reinterpret_cast<const int*>(static_cast<uint8_t*>(D.ditems) + items.size() * sizeof(int2));
}

// workspace of lattice i through its own plan: its slot, or the shared
// region after the slots when its plan needs more (a chirp-z axis)
float2* single_ws(const BatchPlan* b, const LatticePlan* p, int i, void* ws) {
  float2* w = static_cast<float2*>(ws);
  return p->ws_elems > (size_t)b->m[i] ? w + b->ws_elems : w + b->ws_off[i];
}

LatticePlan* single_plan(BatchPlan* b, int i) {
  if (!b->single[i]) {
    LatticePlan* p = build_lattice_plan(b->d, &b->Ms[(size_t)i * b->d * b->d], 1, 0);
    try {
      upload_plan(p);
    } catch (...) {
      free_plan(p);
      throw;
    }
    b->single[i] = p;
  }
  return b->single[i];
}

void enqueue_persistent(BatchPlan* b, bool inverse, const void* in, void* out, void* ws,
                        hipStream_t s, bool trace) {
  const BatchDir& D = b->dir[inverse ? 1 : 0];
  if (D.nitems > 0) {
    hipError_t e = launch_batch_clear(b->dheads, 16, s);
    if (e != hipSuccess) throw StatusError{E_HIP};
    for (int ph = 0; ph < 2; ++ph) {
      if (D.phase_items[ph] == 0) continue;
      // method bytes: 16 B per point of every lattice with a pass in this
      // phase, over its number of passes; pass bytes: 16 B per point
      double bytes = 0, pass_bytes = 0;
      for (int i = 0; i < b->count; ++i) {
        const LatticePlan* p = b->tiled[i];
        const int np = p ? (int)p->fwd.passes.size() : 0;
        if (np > ph) {
          bytes += 16.0 * (double)b->m[i] / np;
          pass_bytes += 16.0 * (double)b->m[i];
        }
      }
      TraceScope ts(trace && trace_on() ? batch_kernel_name(b->tile_lg) : nullptr, bytes,
                    pass_bytes, s);
      // never more workgroups than items: idle ones would only contend for
      // the queue heads
      const int grid = std::min(b->grid, std::max(8, D.phase_items[ph]));
      e = launch_batch(b->tile_lg, static_cast<const BatchPass*>(D.dpass),
                       static_cast<const int2*>(D.ditems), D.qbeg + 8 * ph,
                       b->dheads + 8 * kHeadStride * ph, static_cast<const float2*>(in),
                       static_cast<float2*>(out), static_cast<float2*>(ws), grid, s);
      if (e != hipSuccess) throw StatusError{E_HIP};
    }
  }
  // lattices the fixed-tile schedule does not cover: one plan each
  for (int i = 0; i < b->count; ++i) {
    if (b->tiled[i]) continue;
    LatticePlan* p = single_plan(b, i);
    exec_lattice(p, inverse, false, false, static_cast<const float2*>(in) + b->in_off[i],
                 static_cast<float2*>(out) + b->out_off[i], single_ws(b, p, i, ws), p->m, p->m, s);
  }
}

}  // namespace

BatchPlan* build_batch_plan(int count, int d, const i64* Ms, uint32_t flags) {
  return build_batch_plan_at(count, d, Ms, nullptr, nullptr, nullptr, 0, flags, 12, 0);
}

BatchPlan* build_batch_plan_at(int count, int d, const i64* Ms, const i64* in_off,
                               const i64* out_off, const i64* ws_off, size_t ws_elems,
                               uint32_t flags, int tile_lg, int order) {
  if (count < 1 || d < 1 || d > kMaxD || !Ms) throw StatusError{E_ARG};
  auto* b = new BatchPlan();
  try {
    b->count = count;
    b->d = d;
    b->flags = flags;
    b->Ms.assign(Ms, Ms + (size_t)count * d * d);
    b->off.push_back(0);
    for (int i = 0; i < count; ++i) {
      Mat A = Mat::from(d, &b->Ms[(size_t)i * d * d]);
      i64 D = det(A);
      if (D == 0) throw StatusError{E_SINGULAR};
      const i64 mi = D < 0 ? -D : D;
      if (mi >= (i64(1) << 31)) throw StatusError{E_UNSUPPORTED};
      b->m.push_back(mi);
      b->off.push_back(cadd(b->off.back(), mi));
    }
    b->total = b->off.back();
    if (b->total >= (i64(1) << 40)) throw StatusError{E_UNSUPPORTED};
    b->single.assign(count, nullptr);
    if (in_off && out_off && ws_off) {
      b->in_off.assign(in_off, in_off + count);
      b->out_off.assign(out_off, out_off + count);
      b->ws_off.assign(ws_off, ws_off + count);
      b->ws_elems = ws_elems;
    } else {
      b->in_off.assign(b->off.begin(), b->off.end() - 1);
      b->out_off = b->in_off;
      b->ws_off = b->in_off;
      b->ws_elems = (size_t)b->total;
    }
    // lattices whose own plan needs more workspace than their slot (a
    // chirp-z axis; every elementary divisor a power of two never does)
    for (int i = 0; i < count; ++i) {
      const Smith S = smith(Mat::from(d, &b->Ms[(size_t)i * d * d]));
      bool pow2 = true;
      for (int j = 0; j < d; ++j) pow2 = pow2 && (S.eps[j] & (S.eps[j] - 1)) == 0;
      if (pow2) continue;
      LatticePlan* hp = build_lattice_plan(d, &b->Ms[(size_t)i * d * d], 1, kPlanHostOnly);
      if (hp->ws_elems > (size_t)b->m[i]) b->extra_ws = std::max(b->extra_ws, hp->ws_elems);
      free_plan(hp);
    }
    if (b->extra_ws && in_off) throw StatusError{E_UNSUPPORTED};
    if (!(flags & kPlanHostOnly)) {
      const size_t n = 16 * kHeadStride * sizeof(int);
      if (hipMalloc(&b->dheads, n) != hipSuccess) throw StatusError{E_NOMEM};
      if (hipMemset(b->dheads, 0, n) != hipSuccess) throw StatusError{E_HIP};
      if (hipStreamCreateWithFlags(&b->cap, hipStreamNonBlocking) != hipSuccess)
        throw StatusError{E_HIP};
    }
    configure_batch(b, tile_lg, order);
  } catch (...) {
    free_batch_plan(b);
    throw;
  }
  return b;
}

void free_batch_plan(BatchPlan* b) {
  if (!b) return;
  drop_tiled(b);
  for (auto* p : b->single) free_plan(p);
  if (b->dheads) (void)hipFree(b->dheads);
  if (b->cap) (void)hipStreamDestroy(b->cap);
  delete b;
}

void configure_batch(BatchPlan* b, int tile_lg, int order) {
  if (tile_lg < 11 || tile_lg > 13 || order < 0 || order > 7) throw StatusError{E_ARG};
  drop_tiled(b);
  b->tile_lg = tile_lg;
  b->order = order;
  b->tiled.assign(b->count, nullptr);
  b->eligible = 0;
  for (int i = 0; i < b->count; ++i) {
    try {
      b->tiled[i] = build_lattice_plan(b->d, &b->Ms[(size_t)i * b->d * b->d], 1, 0, tile_lg, order);
      ++b->eligible;
    } catch (const StatusError& e) {
      if (e.code != E_UNSUPPORTED) throw;
      b->tiled[i] = nullptr;
    }
  }
  if (b->flags & kPlanHostOnly) {  // schedules only, no device tables
    b->configured = true;
    return;
  }
  for (auto* p : b->tiled)
    if (p) upload_plan(p);
  int occ = batch_occupancy(tile_lg);
  if (occ < 1) throw StatusError{E_HIP};
  int dev = 0, cus = 0;
  if (hipGetDevice(&dev) != hipSuccess ||
      hipDeviceGetAttribute(&cus, hipDeviceAttributeMultiprocessorCount, dev) != hipSuccess)
    throw StatusError{E_HIP};
  b->grid = cus * occ;
  build_dir(b, false, b->dir[0]);
  build_dir(b, true, b->dir[1]);
  b->configured = true;
}

void exec_batch(BatchPlan* b, bool inverse, int mode, const void* in, void* out, void* ws,
                hipStream_t s) {
  if (!b->configured || !b->dheads) throw StatusError{E_STATE};
  if (mode == BATCH_LOOP) {
    for (int i = 0; i < b->count; ++i) {
      LatticePlan* p = single_plan(b, i);
      exec_lattice(p, inverse, false, false, static_cast<const float2*>(in) + b->in_off[i],
                   static_cast<float2*>(out) + b->out_off[i], single_ws(b, p, i, ws), p->m, p->m,
                   s);
    }
    return;
  }
  if (mode == BATCH_PERSISTENT) {
    enqueue_persistent(b, inverse, in, out, ws, s, true);
    return;
  }
  if (mode != BATCH_GRAPH) throw StatusError{E_ARG};
  // ineligible lattices are built before capture (no allocation while capturing)
  for (int i = 0; i < b->count; ++i)
    if (!b->tiled[i]) single_plan(b, i);
  auto key = std::make_tuple(inverse ? 1 : 0, in, out, ws);
  auto it = b->graphs.find(key);
  if (it == b->graphs.end()) {
    if (hipStreamBeginCapture(b->cap, hipStreamCaptureModeThreadLocal) != hipSuccess)
      throw StatusError{E_HIP};
    try {
      enqueue_persistent(b, inverse, in, out, ws, b->cap, false);
    } catch (...) {
      hipGraph_t g = nullptr;
      (void)hipStreamEndCapture(b->cap, &g);
      if (g) (void)hipGraphDestroy(g);
      throw;
    }
    hipGraph_t g = nullptr;
    if (hipStreamEndCapture(b->cap, &g) != hipSuccess || !g) throw StatusError{E_HIP};
    hipGraphExec_t ex = nullptr;
    hipError_t e = hipGraphInstantiate(&ex, g, nullptr, nullptr, 0);
    (void)hipGraphDestroy(g);
    if (e != hipSuccess) throw StatusError{E_HIP};
    it = b->graphs.emplace(key, ex).first;
  }
  double bytes = 16.0 * (double)b->total;
  TraceScope ts(trace_on() ? "fft_batch_graph" : nullptr, bytes, s);
  if (hipGraphLaunch(it->second, s) != hipSuccess) throw StatusError{E_HIP};
}

void tune_batch(BatchPlan* b, const void* in, void* out, void* ws, int reps, hipStream_t s,
                float* best_ms) {
  if (!b->dheads || reps < 1) throw StatusError{E_ARG};
  TuneKey key;
  key.arch = device_arch();
  key.d = b->d;
  key.flags = b->flags;
  key.Ms = b->Ms;
  TuneVal known;
  if (tune_cache_find(key, &known)) {
    if (known.tile_lg != b->tile_lg || known.order != b->order || !b->configured)
      configure_batch(b, known.tile_lg, known.order);
    if (best_ms) *best_ms = -1.0f;
    return;
  }
  hipEvent_t e0, e1;
  if (hipEventCreate(&e0) != hipSuccess || hipEventCreate(&e1) != hipSuccess)
    throw StatusError{E_HIP};
  float best = -1.0f;
  std::pair<int, int> arg{12, 0};
  try {
    for (int tl : {11, 12, 13}) {
      for (int ord : {0, 1, 2, 3}) {
        configure_batch(b, tl, ord);
        enqueue_persistent(b, false, in, out, ws, s, false);
        float tmin = -1.0f;
        for (int r = 0; r < reps; ++r) {
          (void)hipEventRecord(e0, s);
          enqueue_persistent(b, false, in, out, ws, s, false);
          (void)hipEventRecord(e1, s);
          if (hipEventSynchronize(e1) != hipSuccess) throw StatusError{E_HIP};
          float ms = 0;
          (void)hipEventElapsedTime(&ms, e0, e1);
          if (tmin < 0 || ms < tmin) tmin = ms;
        }
        if (best < 0 || tmin < best) {
          best = tmin;
          arg = {tl, ord};
        }
      }
    }
  } catch (...) {
    (void)hipEventDestroy(e0);
    (void)hipEventDestroy(e1);
    throw;
  }
  (void)hipEventDestroy(e0);
  (void)hipEventDestroy(e1);
  configure_batch(b, arg.first, arg.second);
  tune_cache_put(key, TuneVal{arg.first, arg.second, best});
  if (best_ms) *best_ms = best;
}

}  // namespace lfft
