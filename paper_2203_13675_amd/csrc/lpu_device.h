// Device helpers: deterministic FP64 block reductions.
#pragma once

#include <hip/hip_runtime.h>

#include "lpu_internal.h"

namespace lpu {

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
