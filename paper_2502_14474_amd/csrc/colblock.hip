// Column-blocked float64 Bellman sweep.
//
// When the gathered vector v is much larger than one XCD's L2 (4 MB) and most
// columns of a row lie far from its own state, every gather of a plain CSR
// sweep pulls a line from the Infinity Cache.  Cutting the columns into
// slices of at most 4 MB of v (one XCD's L2) and making one pass per slice
// keeps most of each pass's gathers inside L2; the price is a float64 partial sum per row carried from
// pass to pass (read and written once per pass).
//
// Storage (built once at mdp_create): the entries of slice b form one
// segment; inside it, the sweep tiles follow each other and inside a tile the
// rows, each row keeping its entries in CSR order.  off[b][t] is the first
// entry of tile t in slice b (off[b][ntiles] the end of the slice) and
// rel[b][r] the first entry of row r relative to its tile's start (16 bits).
// Rows holding more than 255 entries of one slice, rows whose slices are not
// in increasing order and tiles holding more than 65535 entries of one slice
// are not supported: the copy is then not built.
//
// The slice parts of a row are short (a row's k entries spread over all
// slices), so a pass streams each tile's segment as a flat array, every lane
// taking every kBlock-th entry, and only then assigns the products to rows
// (through LDS).  A row's sum is the sum of its slice parts in slice order,
// each part an fma chain in CSR order, so the result is deterministic and
// identical rows give identical sums.
#include <cstdlib>

#include "device.h"

namespace mdp {

namespace {

// cnt[b][r] for every row; *far += entries outside the row's own slice;
// *bad = 1 when a row is not supported.
__global__ __launch_bounds__(kBlock) void k_cb_count(int64_t S, int64_t rows, int A, const int* __restrict__ rp,
                                                     const int* __restrict__ col, int slice,
                                                     uint8_t* __restrict__ cnt,
                                                     unsigned long long* __restrict__ far,
                                                     int* __restrict__ bad) {
  const int64_t r = static_cast<int64_t>(blockIdx.x) * kBlock + threadIdx.x;
  unsigned long long f = 0;
  int b_bad = 0;
  if (r < rows) {
    const int own = static_cast<int>(state_of_row(r, A, S) / slice);
    int cur = -1, run = 0;
    for (int e = rp[r]; e < rp[r + 1]; ++e) {
      const int b = col[e] / slice;
      if (b != cur) {
        if (cur >= 0) cnt[static_cast<int64_t>(cur) * rows + r] = static_cast<uint8_t>(run);
        if (b < cur) b_bad = 1;
        cur = b;
        run = 0;
      }
      run = run < 255 ? run + 1 : (b_bad = 1, run);
      f += b != own ? 1ull : 0ull;
    }
    if (cur >= 0) cnt[static_cast<int64_t>(cur) * rows + r] = static_cast<uint8_t>(run);
  }
  f = wave_sum(f);
  b_bad = wave_sum(b_bad);
  if ((threadIdx.x & (kWave - 1)) == 0) {
    if (f) atomicAdd(far, f);
    if (b_bad) atomicOr(bad, 1);
  }
}

// tsum[b][t] = entries of tile t in slice b.
__global__ __launch_bounds__(kBlock) void k_cb_tile_sums(int64_t rows, int tile_rows, int ntiles,
                                                         const uint8_t* __restrict__ cnt,
                                                         int* __restrict__ tsum) {
  const int t = blockIdx.x, b = blockIdx.y;
  const int64_t r0 = static_cast<int64_t>(t) * tile_rows;
  const int nr = static_cast<int>(min<int64_t>(tile_rows, rows - r0));
  double s = 0.0, mx = 0.0;  // exact: at most 255 * 1024 per tile
  for (int i = threadIdx.x; i < nr; i += kBlock) s += cnt[static_cast<int64_t>(b) * rows + r0 + i];
  block_max_sum(mx, s);
  if (threadIdx.x == 0) tsum[static_cast<int64_t>(b) * ntiles + t] = static_cast<int>(s);
}

// Copy the entries of each row to their blocked positions and record each
// row's start inside its tile.  One workgroup per tile; each thread owns up to
// 4 rows and walks them slice by slice.
__global__ __launch_bounds__(kBlock) void k_cb_scatter(int64_t rows, int tile_rows, int ntiles,
                                                       int nblk, int slice,
                                                       const int* __restrict__ rp,
                                                       const int* __restrict__ col,
                                                       const double* __restrict__ val,
                                                       const uint8_t* __restrict__ cnt,
                                                       const int* __restrict__ off,
                                                       int* __restrict__ cb_col,
                                                       double* __restrict__ cb_val,
                                                       uint16_t* __restrict__ rel) {
  __shared__ int pos[4 * kBlock + 1];
  const int t = blockIdx.x;
  const int64_t r0 = static_cast<int64_t>(t) * tile_rows;
  const int nr = static_cast<int>(min<int64_t>(tile_rows, rows - r0));
  int cur[4], end[4];
#pragma unroll
  for (int j = 0; j < 4; ++j) {
    const int i = threadIdx.x + j * kBlock;
    cur[j] = i < nr ? rp[r0 + i] : 0;
    end[j] = i < nr ? rp[r0 + i + 1] : 0;
  }
  for (int b = 0; b < nblk; ++b) {
    for (int i = threadIdx.x; i < nr; i += kBlock) pos[i] = cnt[static_cast<int64_t>(b) * rows + r0 + i];
    __syncthreads();
    block_exclusive_scan(pos, nr);
    const int base = off[static_cast<int64_t>(b) * (ntiles + 1) + t];
#pragma unroll
    for (int j = 0; j < 4; ++j) {
      const int i = threadIdx.x + j * kBlock;
      if (i >= nr) continue;
      rel[static_cast<int64_t>(b) * rows + r0 + i] = static_cast<uint16_t>(pos[i]);
      int d = base + pos[i];
      while (cur[j] < end[j] && col[cur[j]] / slice == b) {
        cb_col[d] = col[cur[j]];
        cb_val[d] = val[cur[j]];
        ++d;
        ++cur[j];
      }
    }
    __syncthreads();
  }
}

// One pass of the blocked sweep over slice b for one tile of states.  The
// tile's entries in slice b are one contiguous segment; it is streamed in
// chunks of kCbChunk entries.  Every thread loads entries i, i + kBlock, ...
// of a chunk (coalesced column and value streams), gathers their v values
// from the L2-resident slice, and leaves each (value, v) pair in LDS; the next
// chunk's loads are issued before the pairs are stored, so they stay in
// flight.  Then thread i carries rows i, i + kBlock, ... of the tile (at most
// 4) through the chunk: a row's slice part is the fma chain over its entries
// in CSR order, started from 0, and continues across chunks.  Passes before
// the last add the part into acc; the last forms Q = g + gamma (acc + part)
// in LDS and finishes the tile like the plain sweep.
// Nontemporal accesses for the running sums, the slice parts and the row starts: each is touched once per pass, and
// kept out of the way they leave the L2 to the slice of the gathered vector
// (on the 4M-state workload: sweep 11.7 -> 11.2 ms, product 809 -> 790 us).
#ifndef MDP_NT_PARTS
#define MDP_NT_PARTS 1
#endif
#ifndef MDP_CB_CHUNK
#define MDP_CB_CHUNK 1024
#endif
constexpr int kCbChunk = MDP_CB_CHUNK;

constexpr int kCbRpt = 4;  // rows per thread: tiles hold at most 4 * kBlock rows

// The slice-b parts of the rows of one tile: part[k] for row threadIdx.x + k *
// kBlock (0 for rows past the tile), each the fma chain over the row's entries
// in slice b in CSR order, started from 0.
__device__ __forceinline__ void cb_tile_parts(int64_t S, int A, int tile_states, int ntiles, int b, int tile,
                                              const uint16_t* __restrict__ rel, const int* __restrict__ off,
                                              const int* __restrict__ cb_col, const double* __restrict__ cb_val,
                                              const double* __restrict__ v, double* lp, double* lx,
                                              double (&sum)[kCbRpt]) {
  constexpr int EPT = kCbChunk / kBlock;
  const int64_t rows = S * A;
  const int64_t s0 = static_cast<int64_t>(tile) * tile_states;
  const int ns = static_cast<int>(min<int64_t>(tile_states, S - s0));
  const int nrows = ns * A;
  const int64_t row0 = s0 * A;
  const int64_t ob = static_cast<int64_t>(b) * (ntiles + 1) + tile;
  const int base = off[ob];
  const int n = off[ob + 1] - base;
  const uint16_t* __restrict__ rl = rel + static_cast<int64_t>(b) * rows + row0;
  const int* __restrict__ cc = cb_col + base;
  const double* __restrict__ cv = cb_val + base;
  const Gather<double> gx(v, S);
  int st[kCbRpt], en[kCbRpt];
#pragma unroll
  for (int k = 0; k < kCbRpt; ++k) {
    const int i = threadIdx.x + k * kBlock;
    const bool valid = i < nrows;
#if MDP_NT_PARTS
    const int a = __builtin_nontemporal_load(rl + (valid ? i : 0));
    const int z = __builtin_nontemporal_load(rl + (i + 1 < nrows ? i + 1 : 0));
#else
    const int a = rl[valid ? i : 0];
    const int z = rl[i + 1 < nrows ? i + 1 : 0];
#endif
    st[k] = valid ? a : 0;
    en[k] = valid ? (i + 1 < nrows ? z : n) : 0;
    sum[k] = 0.0;
  }
  int c[EPT];
  double p[EPT];
  // unconditional loads: lanes past the segment read its first entry (an
  // empty segment is never fetched)
  auto fetch = [&](int c0) {
#pragma unroll
    for (int e = 0; e < EPT; ++e) {
      const int idx = c0 + threadIdx.x + e * kBlock;
      const bool ok = idx < n;
      const int craw = ld_col(cc + (ok ? idx : 0));
      const double praw = ld_val(cv + (ok ? idx : 0));
      c[e] = ok ? craw : -1;
      p[e] = ok ? praw : 0.0;
    }
  };
  if (n > 0) fetch(0);
  for (int c0 = 0; c0 < n; c0 += kCbChunk) {
    double x[EPT], pc[EPT];
#pragma unroll
    for (int e = 0; e < EPT; ++e) {
      x[e] = gx(c[e]);  // 0 past the segment (c = -1)
      pc[e] = p[e];
    }
    fetch(c0 + kCbChunk < n ? c0 + kCbChunk : c0);
#pragma unroll
    for (int e = 0; e < EPT; ++e) {
      lp[threadIdx.x + e * kBlock] = pc[e];
      lx[threadIdx.x + e * kBlock] = x[e];
    }
    __syncthreads();
    const int c1 = c0 + kCbChunk;
#pragma unroll
    for (int k = 0; k < kCbRpt; ++k) {
      const int lo = st[k] > c0 ? st[k] : c0;
      const int hi = en[k] < c1 ? en[k] : c1;
      double sk = sum[k];
      for (int j = lo; j < hi; ++j) sk = fma(lp[j - c0], lx[j - c0], sk);
      sum[k] = sk;
    }
    __syncthreads();
  }
}

template <bool FIRST, bool LAST, typename RT>
__global__ __launch_bounds__(kBlock) void k_bellman_cb(
    int64_t S, int A, int tile_states, int ntiles, int b, const uint16_t* __restrict__ rel,
    const int* __restrict__ off, const int* __restrict__ cb_col, const double* __restrict__ cb_val,
    const double* __restrict__ cost, const double* __restrict__ v, double gamma,
    double* __restrict__ acc, double* __restrict__ Tv, int* __restrict__ pi, RT* __restrict__ r0,
    double4* __restrict__ partials) {
  extern __shared__ double q[];  // LAST: one value per row of the tile
  __shared__ double lp[kCbChunk], lx[kCbChunk];
  const int tile = xcd_tile(blockIdx.x, gridDim.x);
  const int64_t s0 = static_cast<int64_t>(tile) * tile_states;
  const int ns = static_cast<int>(min<int64_t>(tile_states, S - s0));
  const int nrows = ns * A;
  const int64_t row0 = s0 * A;
  double prev[kCbRpt];
#pragma unroll
  for (int k = 0; k < kCbRpt; ++k) {
    const int i = threadIdx.x + k * kBlock;
#if MDP_NT_PARTS
    prev[k] = FIRST ? 0.0 : __builtin_nontemporal_load(acc + row0 + (i < nrows ? i : 0));
#else
    prev[k] = FIRST ? 0.0 : acc[row0 + (i < nrows ? i : 0)];
#endif
  }
  double sum[kCbRpt];
  cb_tile_parts(S, A, tile_states, ntiles, b, tile, rel, off, cb_col, cb_val, v, lp, lx, sum);
#pragma unroll
  for (int k = 0; k < kCbRpt; ++k) {
    const int i = threadIdx.x + k * kBlock;
    if (i >= nrows) continue;
    const double total = FIRST ? sum[k] : prev[k] + sum[k];
    if (LAST) {
      q[(i % ns) * A + i / ns] = fma(gamma, total, cost[row0 + i]);  // stored row -> (state, action)
    } else {
#if MDP_NT_PARTS
      __builtin_nontemporal_store(total, acc + row0 + i);
#else
      acc[row0 + i] = total;
#endif
    }
  }
  if (LAST) {
    __syncthreads();
    sweep_finish<double, double, RT>(s0, ns, A, q, v, Tv, pi, r0, partials, tile);
  }
}

// The float64 sweep streamed tile by tile over the CSR rows themselves, for
// MDPs with short rows: a tile's rows are contiguous in the stored order, so
// its entries form one segment, streamed in chunks through LDS as a slice
// segment is above, and each row's sum is the fma chain over its entries in
// CSR order (the one-slice blocked sweep, without a copy).  With a few
// entries per row this leaves no lane of a row group idle.
template <typename RT>
__global__ __launch_bounds__(kBlock) void k_bellman_flat(int64_t S, int A, int tile_states,
                                                         const int* __restrict__ row_ptr, const int* __restrict__ col,
                                                         const double* __restrict__ val,
                                                         const double* __restrict__ cost,
                                                         const double* __restrict__ v, double gamma,
                                                         double* __restrict__ Tv, int* __restrict__ pi,
                                                         RT* __restrict__ r0, double4* __restrict__ partials) {
  extern __shared__ double q[];  // one value per row of the tile
  __shared__ double lp[kCbChunk], lx[kCbChunk];
  constexpr int EPT = kCbChunk / kBlock;
  const int tile = xcd_tile(blockIdx.x, gridDim.x);
  const int64_t s0 = static_cast<int64_t>(tile) * tile_states;
  const int ns = static_cast<int>(min<int64_t>(tile_states, S - s0));
  const int nrows = ns * A;
  const int64_t row0 = s0 * A;
  const int base = row_ptr[row0];
  const int n = row_ptr[row0 + nrows] - base;
  const int* __restrict__ cc = col + base;
  const double* __restrict__ cv = val + base;
  const Gather<double> gx(v, S);
  int st[kCbRpt], en[kCbRpt];
  double sum[kCbRpt];
#pragma unroll
  for (int k = 0; k < kCbRpt; ++k) {
    const int i = threadIdx.x + k * kBlock;
    const bool valid = i < nrows;
    st[k] = valid ? row_ptr[row0 + i] - base : 0;
    en[k] = valid ? row_ptr[row0 + i + 1] - base : 0;
    sum[k] = 0.0;
  }
  int c[EPT];
  double p[EPT];
  auto fetch = [&](int c0) {
#pragma unroll
    for (int e = 0; e < EPT; ++e) {
      const int idx = c0 + threadIdx.x + e * kBlock;
      const bool ok = idx < n;
      const int craw = ld_col(cc + (ok ? idx : 0));
      const double praw = ld_val(cv + (ok ? idx : 0));
      c[e] = ok ? craw : -1;
      p[e] = ok ? praw : 0.0;
    }
  };
  if (n > 0) fetch(0);
  for (int c0 = 0; c0 < n; c0 += kCbChunk) {
    double x[EPT], pc[EPT];
#pragma unroll
    for (int e = 0; e < EPT; ++e) {
      x[e] = gx(c[e]);  // 0 past the segment (c = -1)
      pc[e] = p[e];
    }
    fetch(c0 + kCbChunk < n ? c0 + kCbChunk : c0);
#pragma unroll
    for (int e = 0; e < EPT; ++e) {
      lp[threadIdx.x + e * kBlock] = pc[e];
      lx[threadIdx.x + e * kBlock] = x[e];
    }
    __syncthreads();
    const int c1 = c0 + kCbChunk;
#pragma unroll
    for (int k = 0; k < kCbRpt; ++k) {
      const int lo = st[k] > c0 ? st[k] : c0;
      const int hi = en[k] < c1 ? en[k] : c1;
      double sk = sum[k];
      for (int j = lo; j < hi; ++j) sk = fma(lp[j - c0], lx[j - c0], sk);
      sum[k] = sk;
    }
    __syncthreads();
  }
#pragma unroll
  for (int k = 0; k < kCbRpt; ++k) {
    const int i = threadIdx.x + k * kBlock;
    if (i < nrows) q[(i % ns) * A + i / ns] = fma(gamma, sum[k], cost[row0 + i]);  // stored row -> (state, action)
  }
  __syncthreads();
  sweep_finish<double, double, RT>(s0, ns, A, q, v, Tv, pi, r0, partials, tile);
}

// All slices of a pass in one launch: workgroup w takes slice pass * 8 + w % 8
// of tile w / 8, so XCD w % 8 (the dispatcher's choice for workgroup w) keeps
// only its own slice of v in its L2.  The rows' slice parts go to
// acc[b * rows + row]; k_bellman_cb_sum then adds them.
__global__ __launch_bounds__(kBlock) void k_bellman_cb_xcd(
    int64_t S, int A, int tile_states, int ntiles, int nblk, int pass, const uint16_t* __restrict__ rel,
    const int* __restrict__ off, const int* __restrict__ cb_col, const double* __restrict__ cb_val,
    const double* __restrict__ v, double* __restrict__ acc) {
  __shared__ double lp[kCbChunk], lx[kCbChunk];
  const int b = pass * kNumXcd + static_cast<int>(blockIdx.x % kNumXcd);
  const int tile = static_cast<int>(blockIdx.x / kNumXcd);
  if (b >= nblk || tile >= ntiles) return;  // the same for the whole workgroup
  const int64_t rows = S * A;
  const int64_t s0 = static_cast<int64_t>(tile) * tile_states;
  const int nrows = static_cast<int>(min<int64_t>(tile_states, S - s0)) * A;
  double sum[kCbRpt];
  cb_tile_parts(S, A, tile_states, ntiles, b, tile, rel, off, cb_col, cb_val, v, lp, lx, sum);
  double* __restrict__ out = acc + static_cast<int64_t>(b) * rows + s0 * A;
#pragma unroll
  for (int k = 0; k < kCbRpt; ++k) {
    const int i = threadIdx.x + k * kBlock;
#if MDP_NT_PARTS
    if (i < nrows) __builtin_nontemporal_store(sum[k], out + i);
#else
    if (i < nrows) out[i] = sum[k];
#endif
  }
}

// A row's sum is its slice parts added in slice order (as the sequential
// passes carry it), then Q = g + gamma * sum, and the tile is finished like
// the plain sweep.
template <typename RT>
__global__ __launch_bounds__(kBlock) void k_bellman_cb_sum(
    int64_t S, int A, int tile_states, int nblk, const double* __restrict__ acc, const double* __restrict__ cost,
    const double* __restrict__ v, double gamma, double* __restrict__ Tv, int* __restrict__ pi,
    RT* __restrict__ r0, double4* __restrict__ partials) {
  extern __shared__ double q[];
  const int tile = xcd_tile(blockIdx.x, gridDim.x);
  const int64_t rows = S * A;
  const int64_t s0 = static_cast<int64_t>(tile) * tile_states;
  const int ns = static_cast<int>(min<int64_t>(tile_states, S - s0));
  const int nrows = ns * A;
  const int64_t row0 = s0 * A;
  for (int i = threadIdx.x; i < nrows; i += kBlock) {
#if MDP_NT_PARTS
    double total = __builtin_nontemporal_load(acc + row0 + i);
    for (int b = 1; b < nblk; ++b) total = total + __builtin_nontemporal_load(acc + static_cast<int64_t>(b) * rows + row0 + i);
#else
    double total = acc[row0 + i];
    for (int b = 1; b < nblk; ++b) total = total + acc[static_cast<int64_t>(b) * rows + row0 + i];
#endif
    q[(i % ns) * A + i / ns] = fma(gamma, total, cost[row0 + i]);
  }
  __syncthreads();
  sweep_finish<double, double, RT>(s0, ns, A, q, v, Tv, pi, r0, partials, tile);
}

template <typename RT>
hipError_t cb_passes(mdp_handle* h, const double* v, double* Tv, int32_t* pi, RT* r0,
                     double4* part, int nb) {
  const int ts = sweep_tile_states(h->A);
  const int nblk = h->cb_blocks;
  const size_t lds_last = static_cast<size_t>(ts) * h->A * sizeof(double);
  if (h->cb_xcd) {
    const int64_t grid = static_cast<int64_t>(kNumXcd) * nb;
    for (int p = 0; p * kNumXcd < nblk; ++p)
      k_bellman_cb_xcd<<<static_cast<unsigned>(grid), kBlock, 0, h->stream>>>(
          h->S, h->A, ts, nb, nblk, p, h->cb_rel, h->cb_off, h->cb_col, h->cb_val, v, h->cb_acc);
    k_bellman_cb_sum<RT><<<nb, kBlock, lds_last, h->stream>>>(h->S, h->A, ts, nblk, h->cb_acc, h->cost, v,
                                                             h->gamma, Tv, pi, r0, part);
    return hipGetLastError();
  }
#define MDP_CB_ARGS(B)                                                                     \
  h->S, h->A, ts, nb, (B), h->cb_rel, h->cb_off, h->cb_col, h->cb_val, h->cost, v, h->gamma, \
      h->cb_acc, Tv, pi, r0, part
  if (nblk == 1) {
    k_bellman_cb<true, true, RT><<<nb, kBlock, lds_last, h->stream>>>(MDP_CB_ARGS(0));
    return hipGetLastError();
  }
  k_bellman_cb<true, false, RT><<<nb, kBlock, 0, h->stream>>>(MDP_CB_ARGS(0));
  for (int b = 1; b + 1 < nblk; ++b)
    k_bellman_cb<false, false, RT><<<nb, kBlock, 0, h->stream>>>(MDP_CB_ARGS(b));
  k_bellman_cb<false, true, RT><<<nb, kBlock, lds_last, h->stream>>>(MDP_CB_ARGS(nblk - 1));
#undef MDP_CB_ARGS
  return hipGetLastError();
}

}  // namespace

hipError_t launch_bellman_flat(mdp_handle* h, const double* v, double* Tv, int32_t* pi, void* r0, bool r0_f32,
                               double4* part, int nb) {
  const int ts = sweep_tile_states(h->A);
  const size_t lds = static_cast<size_t>(ts) * h->A * sizeof(double);
  if (r0_f32)
    k_bellman_flat<float><<<nb, kBlock, lds, h->stream>>>(h->S, h->A, ts, h->row_ptr, h->col, h->val, h->cost, v,
                                                          h->gamma, Tv, pi, static_cast<float*>(r0), part);
  else
    k_bellman_flat<double><<<nb, kBlock, lds, h->stream>>>(h->S, h->A, ts, h->row_ptr, h->col, h->val, h->cost, v,
                                                           h->gamma, Tv, pi, static_cast<double*>(r0), part);
  return hipGetLastError();
}

hipError_t launch_bellman_cb(mdp_handle* h, const double* v, double* Tv, int32_t* pi, void* r0,
                             bool r0_f32, double4* part, int nb) {
  if (r0_f32) return cb_passes<float>(h, v, Tv, pi, static_cast<float*>(r0), part, nb);
  return cb_passes<double>(h, v, Tv, pi, static_cast<double*>(r0), part, nb);
}

hipError_t build_colblocks(mdp_handle* h, int blocks, bool require, bool* built, double* far_frac) {
  *built = false;
  *far_frac = 0.0;
  const int64_t rows = h->rows;
  const int slice = static_cast<int>((h->S + blocks - 1) / blocks);
  const int ts = sweep_tile_states(h->A);
  const int tile_rows = ts * h->A;
  const int ntiles = static_cast<int>((h->S + ts - 1) / ts);
  uint8_t* cnt = nullptr;
  void* scratch = nullptr;  // far counter + bad flag
  int* tsum = nullptr;
  int* off = nullptr;
  uint16_t* rel = nullptr;
  int* cb_col = nullptr;
  double* cb_val = nullptr;
  double* acc = nullptr;
  auto done = [&](hipError_t r) {
    (void)hipStreamSynchronize(h->stream);
    if (scratch) handle_free(h, scratch);
    if (tsum) handle_free(h, tsum);
    if (cnt) handle_free(h, cnt);
    if (!*built) {
      if (off) handle_free(h, off);
      if (rel) handle_free(h, rel);
      if (cb_col) handle_free(h, cb_col);
      if (cb_val) handle_free(h, cb_val);
      if (acc) handle_free(h, acc);
    }
    return r;
  };
  hipError_t e = hipSuccess;
#define CB_CHK(call)                              \
  do {                                            \
    if ((e = (call)) != hipSuccess) return done(e); \
  } while (0)
  const size_t cnt_bytes = static_cast<size_t>(blocks) * rows;
  CB_CHK(handle_alloc(h, reinterpret_cast<void**>(&cnt), cnt_bytes));
  CB_CHK(handle_alloc(h, &scratch, 16));
  CB_CHK(hipMemsetAsync(cnt, 0, cnt_bytes, h->stream));
  CB_CHK(hipMemsetAsync(scratch, 0, 16, h->stream));
  auto* far = static_cast<unsigned long long*>(scratch);
  int* bad = reinterpret_cast<int*>(static_cast<char*>(scratch) + 8);
  k_cb_count<<<static_cast<unsigned>((rows + kBlock - 1) / kBlock), kBlock, 0, h->stream>>>(
      h->S, rows, h->A, h->row_ptr, h->col, slice, cnt, far, bad);
  CB_CHK(hipGetLastError());
  unsigned long long far_h = 0;
  int bad_h = 0;
  CB_CHK(copy_out(&far_h, far, 8, h->stream));
  CB_CHK(copy_out(&bad_h, bad, 4, h->stream));
  CB_CHK(hipStreamSynchronize(h->stream));
  *far_frac = static_cast<double>(far_h) / static_cast<double>(h->nnz);
  if (bad_h || (!require && *far_frac < 0.5)) return done(hipSuccess);

  const size_t nt = static_cast<size_t>(blocks) * ntiles;
  CB_CHK(handle_alloc(h, reinterpret_cast<void**>(&tsum), nt * sizeof(int)));
  k_cb_tile_sums<<<dim3(ntiles, blocks), kBlock, 0, h->stream>>>(rows, tile_rows, ntiles, cnt, tsum);
  CB_CHK(hipGetLastError());
  std::vector<int> ts_h(nt), off_h(static_cast<size_t>(blocks) * (ntiles + 1));
  CB_CHK(copy_out(ts_h.data(), tsum, nt * sizeof(int), h->stream));
  CB_CHK(hipStreamSynchronize(h->stream));
  int64_t run = 0;
  for (int b = 0; b < blocks; ++b) {
    for (int t = 0; t < ntiles; ++t) {
      const int n = ts_h[static_cast<size_t>(b) * ntiles + t];
      if (n > 65535) return done(hipSuccess);  // 16-bit row starts would overflow
      off_h[static_cast<size_t>(b) * (ntiles + 1) + t] = static_cast<int>(run);
      run += n;
    }
    off_h[static_cast<size_t>(b) * (ntiles + 1) + ntiles] = static_cast<int>(run);
  }
  if (run != h->nnz) return done(hipErrorInvalidValue);
  CB_CHK(handle_alloc(h, reinterpret_cast<void**>(&off), off_h.size() * sizeof(int)));
  CB_CHK(copy_in(off, off_h.data(), off_h.size() * sizeof(int), h->stream));
  CB_CHK(handle_alloc(h, reinterpret_cast<void**>(&rel), cnt_bytes * sizeof(uint16_t)));
  CB_CHK(handle_alloc(h, reinterpret_cast<void**>(&cb_col), h->nnz * sizeof(int)));
  CB_CHK(handle_alloc(h, reinterpret_cast<void**>(&cb_val), h->nnz * sizeof(double)));
  // the parts of all slices side by side (one launch for all slices), or
  // one running sum per row carried from pass to pass
  // (MDP_CB_PARTS_MAX_BYTES in the environment replaces the limit)
  int64_t parts_max = kCbXcdMaxBytes;
  if (const char* env = std::getenv("MDP_CB_PARTS_MAX_BYTES")) parts_max = std::atoll(env);
  const bool xcd = static_cast<int64_t>(blocks) * rows * static_cast<int64_t>(sizeof(double)) <= parts_max;
  const int64_t acc_rows = xcd ? static_cast<int64_t>(blocks) * rows : rows;
  CB_CHK(handle_alloc(h, reinterpret_cast<void**>(&acc), acc_rows * sizeof(double)));
  k_cb_scatter<<<ntiles, kBlock, 0, h->stream>>>(rows, tile_rows, ntiles, blocks, slice, h->row_ptr,
                                                 h->col, h->val, cnt, off, cb_col, cb_val, rel);
  CB_CHK(hipGetLastError());
  CB_CHK(hipStreamSynchronize(h->stream));
#undef CB_CHK
  h->cb_blocks = blocks;
  h->cb_slice = slice;
  h->cb_rel = rel;
  h->cb_off = off;
  h->cb_col = cb_col;
  h->cb_val = cb_val;
  h->cb_acc = acc;
  h->cb_xcd = xcd;
  h->device_bytes += static_cast<int64_t>(cnt_bytes * sizeof(uint16_t) + off_h.size() * sizeof(int) +
                                          h->nnz * 12 + acc_rows * 8);
  *built = true;
  return done(hipSuccess);
}

}  // namespace mdp
