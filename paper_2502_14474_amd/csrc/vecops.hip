// Small vector kernels of the host driver.
#include "device.h"

namespace mdp {

namespace {

__global__ __launch_bounds__(kBlock) void k_negate(double* __restrict__ x, int64_t n) {
  for (int64_t i = static_cast<int64_t>(blockIdx.x) * kBlock + threadIdx.x; i < n;
       i += static_cast<int64_t>(gridDim.x) * kBlock)
    x[i] = -x[i];
}

// one thread per stored row: copy its entries and cost from the natural row
__global__ __launch_bounds__(kBlock) void k_permute_rows(int64_t S, int A, const int32_t* __restrict__ rp_old,
                                                         const int32_t* __restrict__ col_old,
                                                         const double* __restrict__ val_old,
                                                         const double* __restrict__ cost_old,
                                                         const int32_t* __restrict__ rp_new,
                                                         int32_t* __restrict__ col_new,
                                                         double* __restrict__ val_new,
                                                         double* __restrict__ cost_new) {
  const int64_t rows = S * A;
  for (int64_t r = static_cast<int64_t>(blockIdx.x) * kBlock + threadIdx.x; r < rows;
       r += static_cast<int64_t>(gridDim.x) * kBlock) {
    const int64_t s = state_of_row(r, A, S);
    const int T = sweep_tile_states(A);
    const int64_t t0 = (s / T) * T;
    const int64_t n = (S - t0) < T ? (S - t0) : T;
    const int a = static_cast<int>((r - t0 * A) / n);
    const int64_t ro = s * A + a;
    const int src = rp_old[ro], len = rp_old[ro + 1] - src, dst = rp_new[r];
    for (int e = 0; e < len; ++e) {
      col_new[dst + e] = col_old[src + e];
      val_new[dst + e] = val_old[src + e];
    }
    cost_new[r] = cost_old[ro];
  }
}

}  // namespace

hipError_t launch_permute_rows(hipStream_t st, int64_t S, int A, const int32_t* rp_old,
                               const int32_t* col_old, const double* val_old,
                               const double* cost_old, const int32_t* rp_new, int32_t* col_new,
                               double* val_new, double* cost_new) {
  const int64_t rows = S * A;
  const int64_t g = std::min<int64_t>(65536, (rows + kBlock - 1) / kBlock);
  k_permute_rows<<<static_cast<unsigned>(g), kBlock, 0, st>>>(S, A, rp_old, col_old, val_old, cost_old,
                                                              rp_new, col_new, val_new, cost_new);
  return hipGetLastError();
}

hipError_t launch_negate(hipStream_t st, double* x, int64_t n) {
  if (n <= 0) return hipSuccess;
  const int64_t g = std::min<int64_t>(8192, (n + kBlock - 1) / kBlock);
  k_negate<<<static_cast<unsigned>(g), kBlock, 0, st>>>(x, n);
  return hipGetLastError();
}

}  // namespace mdp
