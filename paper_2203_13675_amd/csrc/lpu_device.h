// Device helpers: deterministic FP64 block reductions; global-memory views.
#pragma once

#include <hip/hip_runtime.h>

#include "lpu_internal.h"

namespace lpu {

// Global-memory view of a pointer read from a descriptor in memory (the
// compiler cannot tell its address space and would emit flat loads, which
// also count against the LDS wait counter, so every wait for an LDS read in
// the same wave would wait for them too).
template <typename T>
__device__ __forceinline__ const __attribute__((address_space(1))) T* as_global(const T* p) {
  return (const __attribute__((address_space(1))) T*)(p);
}
template <typename T>
__device__ __forceinline__ __attribute__((address_space(1))) T* as_global(T* p) {
  return (__attribute__((address_space(1))) T*)(p);
}

// Sum NV values over the block; the result is valid in thread 0.  The shape of
// the tree is fixed, so the result does not depend on scheduling.
// smem: NV * (blockDim.x / 64) doubles.
template <int NV>
__device__ __forceinline__ void block_sum(double (&v)[NV], double* smem) {
#pragma unroll
  for (int k = 0; k < NV; ++k)
#pragma unroll
    for (int off = 32; off > 0; off >>= 1) v[k] += __shfl_down(v[k], off, 64);
  const int lane = threadIdx.x & 63, wid = threadIdx.x >> 6, nw = blockDim.x >> 6;
  __syncthreads();
  if (lane == 0)
#pragma unroll
    for (int k = 0; k < NV; ++k) smem[k * nw + wid] = v[k];
  __syncthreads();
  if (threadIdx.x == 0)
#pragma unroll
    for (int k = 0; k < NV; ++k) {
      double s = 0.0;
      for (int w = 0; w < nw; ++w) s += smem[k * nw + w];
      v[k] = s;
    }
}

}  // namespace lpu
