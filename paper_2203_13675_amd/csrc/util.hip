// Small elementwise utility: a pointwise product.
#include "lpu_internal.h"

namespace lpu {

template <typename T>
__global__ void k_scale_by(size_t n, const T* __restrict__ a, const T* __restrict__ b,
                           T* __restrict__ out) {
  for (size_t p = blockIdx.x * (size_t)blockDim.x + threadIdx.x; p < n;
       p += (size_t)gridDim.x * blockDim.x)
    out[p] = a[p] * b[p];
}

template <typename T>
void launch_scale_by(hipStream_t st, size_t n, const T* a, const T* b, T* out) {
  const int grid = (int)std::min<size_t>((n + 255) / 256, 8192);
  hipLaunchKernelGGL(k_scale_by<T>, dim3(std::max(grid, 1)), dim3(256), 0, st, n, a, b, out);
}
template void launch_scale_by<float>(hipStream_t, size_t, const float*, const float*, float*);
template void launch_scale_by<double>(hipStream_t, size_t, const double*, const double*, double*);

}  // namespace lpu
