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

// Entry checks in natural row order, one thread per row (grid-stride, so a
// thread's rows increase and its first failure is its lowest).  The row sum
// adds the entries in order, as the host check does.
__global__ __launch_bounds__(kBlock) void k_validate(int64_t S, int64_t rows, const int32_t* __restrict__ rp,
                                                     const int32_t* __restrict__ col,
                                                     const double* __restrict__ val,
                                                     const double* __restrict__ cost,
                                                     int64_t* __restrict__ out) {
  constexpr int64_t kNone = INT64_MAX;
  __shared__ int64_t s_cost[kBlock], s_row[kBlock];
  __shared__ int s_why[kBlock];
  int64_t bad_cost = kNone, bad_row = kNone;
  int why = 0;
  for (int64_t r = static_cast<int64_t>(blockIdx.x) * kBlock + threadIdx.x; r < rows;
       r += static_cast<int64_t>(gridDim.x) * kBlock) {
    if (bad_cost == kNone && !isfinite(cost[r])) bad_cost = r;
    if (bad_row != kNone) continue;
    const int b = rp[r], e_end = rp[r + 1];
    double sum = 0.0;
    int w = 0;
    for (int e = b; e < e_end; ++e) {
      const int c = col[e];
      const double x = val[e];
      if (c < 0 || c >= S) { w = 1; break; }
      if (!(x >= 0.0) || !isfinite(x)) { w = 2; break; }
      sum += x;
    }
    if (w == 0 && fabs(sum - 1.0) > 1e-12 * fmax(1.0, static_cast<double>(e_end - b))) w = 3;
    if (w != 0) {
      bad_row = r;
      why = w;
    }
  }
  s_cost[threadIdx.x] = bad_cost;
  s_row[threadIdx.x] = bad_row;
  s_why[threadIdx.x] = why;
  __syncthreads();
  for (int h = kBlock / 2; h > 0; h >>= 1) {
    if (threadIdx.x < h) {
      const int o = threadIdx.x + h;
      if (s_cost[o] < s_cost[threadIdx.x]) s_cost[threadIdx.x] = s_cost[o];
      if (s_row[o] < s_row[threadIdx.x]) {
        s_row[threadIdx.x] = s_row[o];
        s_why[threadIdx.x] = s_why[o];
      }
    }
    __syncthreads();
  }
  if (threadIdx.x == 0) {
    out[3 * blockIdx.x + 0] = s_cost[0] == kNone ? -1 : s_cost[0];
    out[3 * blockIdx.x + 1] = s_row[0] == kNone ? -1 : s_row[0];
    out[3 * blockIdx.x + 2] = s_why[0];
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

int validate_blocks(int64_t rows) {
  return static_cast<int>(std::max<int64_t>(1, std::min<int64_t>(1024, (rows + kBlock - 1) / kBlock)));
}

hipError_t launch_validate(hipStream_t st, int64_t S, int64_t rows, const int32_t* rp, const int32_t* col,
                           const double* val, const double* cost, int64_t* out, int blocks) {
  if (blocks != validate_blocks(rows)) return hipErrorInvalidValue;
  k_validate<<<blocks, kBlock, 0, st>>>(S, rows, rp, col, val, cost, out);
  return hipGetLastError();
}

hipError_t launch_negate(hipStream_t st, double* x, int64_t n) {
  if (n <= 0) return hipSuccess;
  const int64_t g = std::min<int64_t>(8192, (n + kBlock - 1) / kBlock);
  k_negate<<<static_cast<unsigned>(g), kBlock, 0, st>>>(x, n);
  return hipGetLastError();
}

}  // namespace mdp
