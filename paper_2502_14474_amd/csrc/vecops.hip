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

// Entry checks in natural row order, 8 lanes per row (grid-stride over rows,
// so each group's rows increase and its first failure is its lowest).  A
// row's failure is its lowest failing entry.  The row sum is the library's
// fixed order: lane l adds entries l, l+8, ... in order, then the eight
// partials combine as ((p0+p4)+(p2+p6)) + ((p1+p5)+(p3+p7)), which the xor
// butterfly below computes on every lane (addition commutes exactly); the
// host check forms the same sum.
__global__ __launch_bounds__(kBlock) void k_validate(int64_t S, int64_t rows, const int32_t* __restrict__ rp,
                                                     const int32_t* __restrict__ col,
                                                     const double* __restrict__ val,
                                                     const double* __restrict__ cost,
                                                     int64_t* __restrict__ out) {
  constexpr int G = 8;
  constexpr int64_t kNone = INT64_MAX;
  __shared__ int64_t s_cost[kBlock], s_row[kBlock];
  __shared__ int s_why[kBlock];
  const int lane = threadIdx.x % G;
  int64_t bad_cost = kNone, bad_row = kNone;
  int why = 0;
  const int64_t gstride = static_cast<int64_t>(gridDim.x) * (kBlock / G);
  for (int64_t r = (static_cast<int64_t>(blockIdx.x) * kBlock + threadIdx.x) / G; r < rows; r += gstride) {
    if (lane == 0 && bad_cost == kNone && !isfinite(cost[r])) bad_cost = r;
    if (bad_row != kNone) continue;  // uniform within the group
    const int b = rp[r], e_end = rp[r + 1];
    int first = INT_MAX, w = 0;
    double part = 0.0;
    for (int j = b + lane; j < e_end; j += G) {
      const int c = col[j];
      const double x = val[j];
      if (first != INT_MAX) continue;
      if (c < 0 || c >= S) {
        first = j;
        w = 1;
      } else if (!(x >= 0.0) || !isfinite(x)) {
        first = j;
        w = 2;
      } else {
        part += x;
      }
    }
#pragma unroll
    for (int off = G / 2; off > 0; off >>= 1) {
      const int of = __shfl_xor(first, off, G);
      const int ow = __shfl_xor(w, off, G);
      if (of < first) {
        first = of;
        w = ow;
      }
      part = part + __shfl_xor(part, off, G);
    }
    if (first == INT_MAX && fabs(part - 1.0) > 1e-12 * fmax(1.0, static_cast<double>(e_end - b))) w = 3;
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

__global__ __launch_bounds__(kBlock) void k_narrow_offsets(const int64_t* __restrict__ src,
                                                           int32_t* __restrict__ dst, int64_t n) {
  for (int64_t i = static_cast<int64_t>(blockIdx.x) * kBlock + threadIdx.x; i < n;
       i += static_cast<int64_t>(gridDim.x) * kBlock)
    dst[i] = static_cast<int32_t>(src[i]);
}

}  // namespace

hipError_t launch_narrow_offsets(hipStream_t st, const int64_t* src, int32_t* dst, int64_t n) {
  if (n <= 0) return hipSuccess;
  const int64_t g = std::min<int64_t>(8192, (n + kBlock - 1) / kBlock);
  k_narrow_offsets<<<static_cast<unsigned>(g), kBlock, 0, st>>>(src, dst, n);
  return hipGetLastError();
}

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
  constexpr int64_t kRowsPerBlock = kBlock / 8;
  return static_cast<int>(std::max<int64_t>(1, std::min<int64_t>(2048, (rows + kRowsPerBlock - 1) / kRowsPerBlock)));
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
