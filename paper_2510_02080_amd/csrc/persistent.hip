#include "align_kernels.h"
#include "align_launch.h"

namespace s3a {

__global__ void k_fill_zero(uint32_t* p, int64_t n) {
  for (int64_t i = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; i < n; i += (int64_t)gridDim.x * blockDim.x) p[i] = 0u;
}

hipError_t launch_fill_zero(uint32_t* p, int64_t n, hipStream_t st) {
  if (n <= 0) return hipSuccess;
  const int grid = (int)std::min<int64_t>((n + 255) / 256, 1024);
  hipLaunchKernelGGL(k_fill_zero, dim3(grid), dim3(256), 0, st, p, n);
  return hipGetLastError();
}

hipError_t launch_persistent(int, const LaunchCfg&, const Shape&, const CallDesc*, const Work&, int, hipStream_t) {
  return hipErrorNotSupported;
}

}  // namespace s3a
