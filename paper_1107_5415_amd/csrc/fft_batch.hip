// Batched persistent launch: the lattice FFTs of many signals on patterns of
// different M.  Every pass of every lattice is cut into tiles of T elements,
// each processed by T / 16 threads with the register-resident pass body of
// fast_tile.hpp.  The tiles of all first passes (and of lattices done in one
// pass) form phase 0, the tiles of all second passes phase 1; each phase is
// one persistent launch over eight work queues, one per XCD, that the host
// fills largest lattice first so that a lattice's tiles stay on one XCD.
// The kernel boundary between the phases orders the two passes of every
// lattice, so the tiles need no counters, fences or waits.
//
// A workgroup takes items from the queue of its own XCD (dispatch index
// mod 8) and, once that is empty, from the others; it exits when all eight
// are empty.
#include <hip/hip_runtime.h>

#include <atomic>

#include "fast_tile.hpp"
#include "kernels.hpp"

namespace lfft {
namespace {
using namespace dev;

// blockDim.x = T / 16 threads (128, 256 or 512) for tiles of T elements.
// qbeg[0..8]: queue boundaries of this phase; heads[32 q]: head of queue q
// (one 128-byte line per head, so claims on different queues do not
// serialise on one line).
__global__ void __launch_bounds__(512) fft_batch_kernel(const BatchPass* __restrict__ passes,
                                                        const int2* __restrict__ items,
                                                        const int* __restrict__ qbeg, int* heads,
                                                        const float2* in, float2* out,
                                                        float2* ws) {
  extern __shared__ float2 lds_raw[];
  __shared__ int s_item;
  const int tid = threadIdx.x;
  const int q0 = blockIdx.x & 7;
  int tried = 0;  // queues found empty (thread 0)
  for (;;) {
    if (tid == 0) {
      int it = -1;
      while (tried < 8) {
        const int q = (q0 + tried) & 7;
        const int k = atomicAdd(&heads[kHeadStride * q], 1);
        if (qbeg[q] + k < qbeg[q + 1]) {
          it = qbeg[q] + k;
          break;
        }
        ++tried;
      }
      s_item = it;
    }
    __syncthreads();
    const int it = __builtin_amdgcn_readfirstlane(s_item);
    if (it < 0) break;
    const int2 I = items[it];
    const int pi = __builtin_amdgcn_readfirstlane(I.x);
    const long long tile = __builtin_amdgcn_readfirstlane(I.y);
    const BatchPass& bp = passes[pi];
    const float2* src = (bp.in_buf == 0 ? in : bp.in_buf == 1 ? out : ws) + bp.in_off;
    float2* dst = (bp.out_buf == 1 ? out : ws) + bp.out_off;
    switch (bp.variant) {
      case BATCH_ROWS_NN:
        fastk::fast_tile<16, false, false, MAP_NATURAL, MAP_NATURAL>(bp.pd, tile, tid, src, dst, lds_raw);
        break;
      case BATCH_ROWS_NI:
        fastk::fast_tile<16, false, false, MAP_NATURAL, MAP_IDENTITY>(bp.pd, tile, tid, src, dst, lds_raw);
        break;
      case BATCH_COLS_NI:
        fastk::fast_tile<16, true, false, MAP_NATURAL, MAP_IDENTITY>(bp.pd, tile, tid, src, dst, lds_raw);
        break;
      case BATCH_ROWS_IN:
        fastk::fast_tile<16, false, false, MAP_IDENTITY, MAP_NATURAL>(bp.pd, tile, tid, src, dst, lds_raw);
        break;
      default:
        fastk::fast_tile<16, true, false, MAP_IDENTITY, MAP_NATURAL>(bp.pd, tile, tid, src, dst, lds_raw);
        break;
    }
    __syncthreads();
  }
}

// Zero the queue heads (a kernel rather than a memset so that the launch can
// be captured into a graph).
__global__ void __launch_bounds__(64) batch_clear_kernel(int* heads, int n) {
  const int i = threadIdx.x;
  if (i < n) heads[kHeadStride * i] = 0;
}

std::atomic<bool> g_attr{false};

hipError_t set_attr() {
  if (g_attr.load(std::memory_order_acquire)) return hipSuccess;
  // the dynamic size requested exactly: the kernel also has static LDS
  hipError_t e = hipFuncSetAttribute((const void*)fft_batch_kernel,
                                     hipFuncAttributeMaxDynamicSharedMemorySize,
                                     (int)batch_lds_bytes(1 << 13));
  if (e == hipSuccess) g_attr.store(true, std::memory_order_release);
  return e;
}

}  // namespace

size_t batch_lds_bytes(int tile) { return (size_t)(tile + tile / 16 + 1) * sizeof(float2); }

int batch_occupancy(int tile_lg) {
  if (tile_lg < 11 || tile_lg > 13 || set_attr() != hipSuccess) return 0;
  int nb = 0;
  if (hipOccupancyMaxActiveBlocksPerMultiprocessor(&nb, fft_batch_kernel, 1 << (tile_lg - 4),
                                                   batch_lds_bytes(1 << tile_lg)) != hipSuccess)
    return 0;
  return nb;
}

const char* batch_kernel_name(int) { return "fft_batch_kernel"; }

hipError_t launch_batch_clear(int* heads, int n, hipStream_t s) {
  if (n < 1 || n > 64) return hipErrorInvalidValue;
  hipLaunchKernelGGL(batch_clear_kernel, dim3(1), dim3(64), 0, s, heads, n);
  return hipGetLastError();
}

hipError_t launch_batch(int tile_lg, const BatchPass* passes, const int2* items, const int* qbeg,
                        int* heads, const float2* in, float2* out, float2* ws, int grid,
                        hipStream_t s) {
  if (tile_lg < 11 || tile_lg > 13) return hipErrorInvalidValue;
  hipError_t e = set_attr();
  if (e != hipSuccess) return e;
  hipLaunchKernelGGL(fft_batch_kernel, dim3(grid), dim3(1 << (tile_lg - 4)),
                     batch_lds_bytes(1 << tile_lg), s, passes, items, qbeg, heads, in, out, ws);
  return hipGetLastError();
}

}  // namespace lfft
