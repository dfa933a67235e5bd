// Batched persistent launch: the lattice FFTs of many signals on patterns of
// different M in one kernel.  Every pass of every lattice is cut into tiles
// of T elements, each processed by T / 16 threads with the register-resident
// pass body of fast_tile.hpp;
// the tiles form eight work queues, one per XCD, that the host fills so that
// each lattice stays on one XCD and its second pass follows its first pass
// by at least one wave of workgroups.
//
// A workgroup takes items from the queue of its own XCD (dispatch index
// mod 8) and then from the others.  The second pass of a lattice waits until
// a counter shows that every tile of its first pass is done; the items are
// claimed in queue order, so every item waited for has already been claimed
// by a running workgroup that never waits for a later item, and the wait
// always ends.  The wait is still bounded: past the spin limit it records
// an error flag and goes on, so a wrong schedule gives a reported error, not
// a hang.
#include <hip/hip_runtime.h>

#include "fast_tile.hpp"
#include "kernels.hpp"

namespace lfft {
namespace {
using namespace dev;

// blockDim.x = T / 16 threads (128, 256 or 512) for tiles of T elements.
__global__ void __launch_bounds__(512) fft_batch_kernel(const BatchPass* __restrict__ passes,
                                                       const int2* __restrict__ items,
                                                       const int* __restrict__ qbeg, int* ctl,
                                                       int* counters, const float2* in,
                                                       float2* out, float2* ws, int spin_limit) {
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
        const int k = atomicAdd(&ctl[q], 1);
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
    if (bp.need > 0) {
      if (tid == 0) {
        int n = 0;
        while (__hip_atomic_load(&counters[bp.inst], __ATOMIC_RELAXED,
                                 __HIP_MEMORY_SCOPE_AGENT) < bp.need) {
          if (++n > spin_limit) {
            atomicOr(&ctl[8], 1);
            break;
          }
          __builtin_amdgcn_s_sleep(2);
        }
      }
      __syncthreads();
      __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "agent");
    }
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
    if (bp.signal) {
      __builtin_amdgcn_fence(__ATOMIC_RELEASE, "agent");
      __syncthreads();
      if (tid == 0)
        __hip_atomic_fetch_add(&counters[bp.inst], 1, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
    }
    __syncthreads();
  }
}

// Zero the queue heads and the per-lattice counters (a kernel rather than a
// memset so that the launch can be captured into a graph).
__global__ void __launch_bounds__(256) batch_clear_kernel(int* ctl, int* counters, int n) {
  const int i = blockIdx.x * blockDim.x + threadIdx.x;
  if (i < 8) ctl[i] = 0;
  for (int k = i; k < n; k += gridDim.x * blockDim.x) counters[k] = 0;
}

bool g_attr = false;

hipError_t set_attr() {
  if (g_attr) return hipSuccess;
  // the dynamic size requested exactly: the kernel also has static LDS
  hipError_t e = hipFuncSetAttribute((const void*)fft_batch_kernel,
                                     hipFuncAttributeMaxDynamicSharedMemorySize,
                                     (int)batch_lds_bytes(1 << 13));
  if (e == hipSuccess) g_attr = true;
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

hipError_t launch_batch_clear(int* ctl, int* counters, int n, hipStream_t s) {
  int blocks = (n + 255) / 256;
  if (blocks < 1) blocks = 1;
  if (blocks > 1024) blocks = 1024;
  hipLaunchKernelGGL(batch_clear_kernel, dim3(blocks), dim3(256), 0, s, ctl, counters, n);
  return hipGetLastError();
}

hipError_t launch_batch(int tile_lg, const BatchPass* passes, const int2* items, const int* qbeg,
                        int* ctl, int* counters, const float2* in, float2* out, float2* ws,
                        int spin_limit, int grid, hipStream_t s) {
  if (tile_lg < 11 || tile_lg > 13) return hipErrorInvalidValue;
  hipError_t e = set_attr();
  if (e != hipSuccess) return e;
  hipLaunchKernelGGL(fft_batch_kernel, dim3(grid), dim3(1 << (tile_lg - 4)),
                     batch_lds_bytes(1 << tile_lg), s, passes, items, qbeg, ctl, counters, in, out,
                     ws, spin_limit);
  return hipGetLastError();
}

}  // namespace lfft
