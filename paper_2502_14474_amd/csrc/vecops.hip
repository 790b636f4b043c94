// Small vector kernels of the host driver.
#include "device.h"

namespace mdp {

namespace {

__global__ __launch_bounds__(kBlock) void k_negate(double* __restrict__ x, int64_t n) {
  for (int64_t i = static_cast<int64_t>(blockIdx.x) * kBlock + threadIdx.x; i < n;
       i += static_cast<int64_t>(gridDim.x) * kBlock)
    x[i] = -x[i];
}

// One workgroup per sweep tile.  A tile covers the same rows, and the same
// range of entries, in the natural and the stored order, so its stored row
// offsets are the tile's first natural offset plus a scan of the stored row
// lengths over the tile's n*A <= 4*kBlock rows.  Groups of 8 lanes then copy
// one row's entries each.
__global__ __launch_bounds__(kBlock) void k_permute_rows(int64_t S, int A, const int32_t* __restrict__ rp_old,
                                                         const int32_t* __restrict__ col_old,
                                                         const double* __restrict__ val_old,
                                                         const double* __restrict__ cost_old,
                                                         int32_t* __restrict__ rp_new,
                                                         int32_t* __restrict__ col_new,
                                                         double* __restrict__ val_new,
                                                         double* __restrict__ cost_new) {
  constexpr int kMaxRows = 4 * kBlock;
  constexpr int G = 8;  // lanes per copied row
  __shared__ int off[kMaxRows + 1];
  __shared__ int src[kMaxRows];
  const int T = sweep_tile_states(A);
  const int64_t tiles = (S + T - 1) / T;
  for (int64_t tile = blockIdx.x; tile < tiles; tile += gridDim.x) {
    const int64_t t0 = tile * T;
    const int n = static_cast<int>((S - t0) < T ? (S - t0) : T);
    const int R = n * A;
    const int64_t r0 = t0 * A;
    const int base = rp_old[r0];
    for (int i = threadIdx.x; i < R; i += kBlock) {
      const int a = i / n;
      const int64_t ro = (t0 + (i - a * n)) * A + a;
      const int b = rp_old[ro];
      src[i] = b;
      off[i] = rp_old[ro + 1] - b;
      cost_new[r0 + i] = cost_old[ro];
    }
    __syncthreads();
    block_exclusive_scan(off, R);
    for (int i = threadIdx.x; i < R; i += kBlock) rp_new[r0 + i] = base + off[i];
    if (tile == tiles - 1 && threadIdx.x == 0) rp_new[r0 + R] = base + off[R];
    const int l = threadIdx.x % G;
    for (int i = threadIdx.x / G; i < R; i += kBlock / G) {
      const int d = base + off[i], b = src[i], len = off[i + 1] - off[i];
      for (int e = l; e < len; e += G) {
        col_new[d + e] = col_old[b + e];
        val_new[d + e] = val_old[b + e];
      }
    }
    __syncthreads();
  }
}

}  // namespace

hipError_t launch_permute_rows(hipStream_t st, int64_t S, int A, const int32_t* rp_old,
                               const int32_t* col_old, const double* val_old,
                               const double* cost_old, int32_t* rp_new, int32_t* col_new,
                               double* val_new, double* cost_new) {
  if (static_cast<int64_t>(sweep_tile_states(A)) * A > 4 * kBlock) return hipErrorInvalidValue;
  const int T = sweep_tile_states(A);
  const int64_t g = std::min<int64_t>(65536, (S + T - 1) / T);
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
