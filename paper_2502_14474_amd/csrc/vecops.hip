// Small vector kernels of the host driver.
#include "device.h"

namespace mdp {

namespace {

__global__ __launch_bounds__(kBlock) void k_negate(double* __restrict__ x, int64_t n) {
  for (int64_t i = static_cast<int64_t>(blockIdx.x) * kBlock + threadIdx.x; i < n;
       i += static_cast<int64_t>(gridDim.x) * kBlock)
    x[i] = -x[i];
}

}  // namespace

hipError_t launch_negate(hipStream_t st, double* x, int64_t n) {
  if (n <= 0) return hipSuccess;
  const int64_t g = std::min<int64_t>(8192, (n + kBlock - 1) / kBlock);
  k_negate<<<static_cast<unsigned>(g), kBlock, 0, st>>>(x, n);
  return hipGetLastError();
}

}  // namespace mdp
