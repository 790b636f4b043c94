// HIP kernels of the inexact-policy-iteration hot path (gfx950).
//
// The path is a memory-bound sparse contraction (about 2 flops per 12 bytes
// of CSR data), so none of it uses MFMA.  What matters is streaming the CSR
// value and column arrays once, coalesced, with enough loads in flight, while
// the gathered vector stays in L2 / Infinity Cache:
//   * L lanes of a 64-wide wavefront share one CSR row; lane l takes the row's
//     entries l, l+L, l+2L, ... and the L partial sums meet in an xor
//     butterfly.  The summation order of a row is therefore a fixed function of
//     positions inside the row, so identical rows give bitwise identical
//     results and the Bellman sweep and the policy products agree bit for bit.
//   * every group keeps U rows in flight (their first entries are loaded
//     before any gather is consumed);
//   * the value and column streams use non-temporal loads so that they do not
//     evict the gathered vector;
//   * workgroups are remapped so that each of the 8 XCDs (one L2 each) works
//     on a contiguous range of states, keeping banded gathers XCD-local;
//   * every reduction is a fixed-order two-stage reduction (per-workgroup
//     partials, then one small kernel), so results are deterministic.
#pragma once

#include "internal.h"

#include <cmath>
#include <type_traits>

namespace mdp {

// ----------------------------------------------------------------------------
// helpers
// ----------------------------------------------------------------------------

__device__ __forceinline__ int xcd_tile(int bid, int nb) {
  // Workgroups are dispatched round-robin over the XCDs; give XCD x the
  // contiguous tile range [x*base + min(x, rem), ...).
  const int q = bid / kNumXcd, x = bid - q * kNumXcd;
  const int base = nb / kNumXcd, rem = nb - base * kNumXcd;
  return x * base + (x < rem ? x : rem) + q;
}

__device__ __forceinline__ double ld_val(const double* p) { return __builtin_nontemporal_load(p); }
__device__ __forceinline__ float ld_val(const float* p) { return __builtin_nontemporal_load(p); }
__device__ __forceinline__ float ld_val(const __half* p) {
  const unsigned short b = __builtin_nontemporal_load(reinterpret_cast<const unsigned short*>(p));
  return __half2float(__ushort_as_half(b));
}
__device__ __forceinline__ int ld_col(const int* p) { return __builtin_nontemporal_load(p); }

__device__ __forceinline__ double max_nan(double a, double b) {
  if (a != a) return a;
  if (b != b) return b;
  return a > b ? a : b;
}

// Gathers from the vector x go through a raw buffer resource: an index of -1
// (empty lane) falls outside the buffer and reads as 0 without a branch, so
// every gather stays unconditional and the prefetched loads keep flowing.
// The third resource word is the raw-buffer setting for CDNA3/CDNA4.
constexpr int kRawBufferWord3 = 0x00020000;

template <typename T>
struct Gather {
  __amdgpu_buffer_rsrc_t r;
  __device__ __forceinline__ Gather(const T* x, int64_t n)
      : r(__builtin_amdgcn_make_buffer_rsrc(
            const_cast<T*>(x), static_cast<short>(0),
            static_cast<int>(static_cast<uint32_t>(n * static_cast<int64_t>(sizeof(T)))), kRawBufferWord3)) {}
  __device__ __forceinline__ T operator()(int c) const;
};
// The byte offset is formed in unsigned 32-bit arithmetic: the hardware reads
// it as unsigned, c = -1 becomes 0xFFFFFFF8 (0xFFFFFFFC), beyond any buffer,
// and the library admits no vector of 2^29 float64 entries or more
// (check_size_limits), so every real offset fits.
template <>
__device__ __forceinline__ double Gather<double>::operator()(int c) const {
  return __builtin_bit_cast(
      double, __builtin_amdgcn_raw_buffer_load_b64(r, static_cast<int>(static_cast<uint32_t>(c) * 8u), 0, 0));
}
template <>
__device__ __forceinline__ float Gather<float>::operator()(int c) const {
  return __builtin_bit_cast(
      float, __builtin_amdgcn_raw_buffer_load_b32(r, static_cast<int>(static_cast<uint32_t>(c) * 4u), 0, 0));
}

// Lane exchange inside a row of 16 lanes through the DPP crossbar (no LDS):
// lane i reads lane i' of the same row as selected by the DPP control word.
template <int CTRL, typename T>
__device__ __forceinline__ T dpp_read(T v) {
  static_assert(sizeof(T) == 4 || sizeof(T) == 8, "4- or 8-byte values");
  if constexpr (sizeof(T) == 4) {
    return __builtin_bit_cast(T, __builtin_amdgcn_mov_dpp(__builtin_bit_cast(int, v), CTRL, 0xF, 0xF, false));
  } else {
    const long long b = __builtin_bit_cast(long long, v);
    const int lo = __builtin_amdgcn_mov_dpp(static_cast<int>(b), CTRL, 0xF, 0xF, false);
    const int hi = __builtin_amdgcn_mov_dpp(static_cast<int>(b >> 32), CTRL, 0xF, 0xF, false);
    return __builtin_bit_cast(T, (static_cast<long long>(hi) << 32) | static_cast<unsigned int>(lo));
  }
}

// Butterfly combine over aligned groups of L lanes (L a power of two, <= 64).
// Stage k pairs lane i with lane i xor k.  Stages k = 32 and 16 cross 16-lane
// rows and use the LDS permute.  Inside a row, k = 8 is a DPP row rotation by
// 8 (exactly i xor 8); k = 4 is a rotation by 4 when the k = 8 stage ran
// before it (every lane then holds the value of its class mod 8, so lane
// i+4 mod 16 carries the same value as i xor 4), and otherwise (L = 8, where
// the rotation would leave the group) the LDS permute; k = 2 and 1 are quad
// permutations.  The result is bitwise that of the plain xor butterfly, and
// every lane ends with it.
template <int L, typename T, typename Op>
__device__ __forceinline__ T group_combine(T v, Op op) {
  if constexpr (L >= 64) v = op(v, __shfl_xor(v, 32, kWave));
  if constexpr (L >= 32) v = op(v, __shfl_xor(v, 16, kWave));
  if constexpr (L >= 16) v = op(v, dpp_read<0x128>(v));  // row_ror:8
  if constexpr (L >= 16) v = op(v, dpp_read<0x124>(v));  // row_ror:4
  if constexpr (L == 8) v = op(v, __shfl_xor(v, 4, kWave));
  if constexpr (L >= 4) v = op(v, dpp_read<0x4E>(v));    // quad_perm [2,3,0,1]
  if constexpr (L >= 2) v = op(v, dpp_read<0xB1>(v));    // quad_perm [1,0,3,2]
  return v;
}

template <int L, typename T>
__device__ __forceinline__ T group_sum(T v) {
  return group_combine<L>(v, [](T a, T b) { return a + b; });
}

template <typename T>
__device__ __forceinline__ T wave_sum(T v) {
  return group_sum<kWave>(v);
}

__device__ __forceinline__ double wave_max_nan(double v) {
  return group_combine<kWave>(v, [](double a, double b) { return max_nan(a, b); });
}

// s + p[t] + p[t + kBlock] + p[t + 2 kBlock] + ... for t = threadIdx.x, in that
// order, with the loads of KB terms issued before their additions.
template <int KB = 8>
__device__ __forceinline__ double strided_sum(const double* __restrict__ p, int n, double s) {
  for (int b0 = threadIdx.x; b0 < n; b0 += KB * kBlock) {
    double v[KB];
#pragma unroll
    for (int k = 0; k < KB; ++k) {
      const int b = b0 + k * kBlock;
      v[k] = p[b < n ? b : b0];
    }
#pragma unroll
    for (int k = 0; k < KB; ++k) s = b0 + k * kBlock < n ? s + v[k] : s;
  }
  return s;
}

// (max, sum) over the workgroup; the result is valid in thread 0.
__device__ __forceinline__ void block_max_sum(double& mx, double& sm) {
  __shared__ double s_mx[kBlock / kWave], s_sm[kBlock / kWave];
  mx = wave_max_nan(mx);
  sm = wave_sum(sm);
  const int w = threadIdx.x / kWave;
  if ((threadIdx.x & (kWave - 1)) == 0) {
    s_mx[w] = mx;
    s_sm[w] = sm;
  }
  __syncthreads();
  if (threadIdx.x == 0) {
    mx = s_mx[0];
    sm = s_sm[0];
#pragma unroll
    for (int i = 1; i < kBlock / kWave; ++i) {
      mx = max_nan(mx, s_mx[i]);
      sm += s_sm[i];
    }
  }
  __syncthreads();
}

// Row products of one workgroup, software pipelined.  `n` rows are handed out
// to lane groups of L lanes: row idx = it*G*U + g + u*G (consecutive groups
// take consecutive rows, so the CSR streams are read in order).  Lane l of a
// group takes the row's entries l, l+L, l+2L, ... and the L partial sums meet
// in an xor butterfly, so a row's summation order depends only on positions
// inside the row.  The first entry of every row of iteration it+1 (column,
// value, and the row's cost) is loaded before the gathers of iteration it are
// consumed, which keeps streaming loads in flight behind the dependent gathers.
//
//   range(idx, st, en, ri, si): entry range [st, en), global row index ri and
//     the state si whose own value x[si] the sink needs (NEEDOWN).
//   sink(idx, pv, gcost, xown): called by every lane of the group with
//     pv = P[ri,:] x (float16 copy: plus the row-sum correction),
//     gcost = cost[ri] (NEEDCOST) and xown = x[si] (NEEDOWN), all prefetched
//     with the row so that the sink issues no load of its own.
template <int L, int U, typename VT, typename XT, typename AT, bool CORR, bool NEEDCOST,
          bool NEEDOWN, typename RangeF, typename SinkF>
__device__ __forceinline__ void pipelined_rows(int n, RangeF range, const int* __restrict__ col,
                                               const VT* __restrict__ val,
                                               const XT* __restrict__ x, int64_t nx,
                                               const double* __restrict__ cost,
                                               const double* __restrict__ corr, SinkF sink) {
  constexpr int G = kBlock / L;
  // The float32 copy is packed per row (columns, then values, in one run of
  // words), so that a selected row of 16 entries is one 128-byte line: `col`
  // and `val` then point at the same array, and entry e of the row [st, en)
  // has its column at word st + e and its value at word en + e.
  constexpr bool PACKED = std::is_same<VT, float>::value;
  const Gather<XT> gx(x, nx);
  constexpr int STEP = G * U;
  const int g = threadIdx.x / L, lane = threadIdx.x % L;
  const int n_it = (n + STEP - 1) / STEP;
  int st[U], en[U], ri[U], c[U], si[U];
  AT p[U];
  double gc[U];
  XT xo[U];
  // Loads are unconditional (out-of-range lanes read entry 0, which always
  // exists) and masked afterwards with selects: a load under a branch makes
  // the compiler wait for every outstanding load before the branch joins,
  // which would drain the prefetched iteration.
  auto fetch = [&](int it) {
#pragma unroll
    for (int u = 0; u < U; ++u) {
      const int idx = it * STEP + g + u * G;
      const bool valid = idx < n;
      int a, b, r, o;
      range(valid ? idx : 0, a, b, r, o);
      st[u] = valid ? a : 0;
      en[u] = valid ? b : 0;
      ri[u] = valid ? r : 0;
      si[u] = valid ? o : -1;
      const int e = st[u] + lane;
      const bool ok = e < en[u];
      const int es = ok ? e : 0;
      int craw;
      AT praw;
      if constexpr (PACKED) {
        // word indices reach 2*nnz: formed in 64 bits.  Idle lanes read word 0,
        // one address for all of them, as the unpacked arrays' idle lanes read
        // entry 0 (an address inside each row would cost a line per row).
        craw = ld_col(col + (ok ? static_cast<int64_t>(st[u]) + e : int64_t{0}));
        praw = static_cast<AT>(ld_val(val + (ok ? static_cast<int64_t>(en[u]) + e : int64_t{0})));
      } else {
        craw = ld_col(col + es);
        praw = static_cast<AT>(ld_val(val + es));
      }
      c[u] = ok ? craw : -1;
      p[u] = ok ? praw : AT(0);
      if (NEEDCOST) gc[u] = cost[ri[u]];
      if (NEEDOWN) xo[u] = gx(si[u]);
    }
  };
  if (n_it > 0) fetch(0);
  for (int it = 0; it < n_it; ++it) {
    int cst[U], cen[U], cri[U], cc[U];
    AT cp[U];
    double cgc[U];
    XT cxo[U];
#pragma unroll
    for (int u = 0; u < U; ++u) {
      cst[u] = st[u];
      cen[u] = en[u];
      cri[u] = ri[u];
      cc[u] = c[u];
      cp[u] = p[u];
      cgc[u] = gc[u];
      cxo[u] = xo[u];
    }
    // Gathers of this iteration first, then the prefetch of the next one:
    // loads complete in issue order, so waiting for the gathers then leaves
    // the prefetch in flight.  The prefetch is unconditional (past the end
    // the rows are empty): a branch would make the compiler drain the loads.
    AT acc[U], xs[U];
    AT xr[U];
#pragma unroll
    for (int u = 0; u < U; ++u) xr[u] = static_cast<AT>(gx(cc[u]));  // 0 when cc = -1
    fetch(it + 1);
#pragma unroll
    for (int u = 0; u < U; ++u) {
      acc[u] = fma(cp[u], xr[u], AT(0));  // cp = 0 on empty lanes
      xs[u] = xr[u];
    }
#pragma unroll
    for (int u = 0; u < U; ++u) {
      for (int e = cst[u] + lane + L; e < cen[u]; e += L) {
        const int64_t co = PACKED ? static_cast<int64_t>(cst[u]) + e : e;
        const int64_t vo = PACKED ? static_cast<int64_t>(cen[u]) + e : e;
        const AT xv = static_cast<AT>(gx(ld_col(col + co)));
        acc[u] = fma(static_cast<AT>(ld_val(val + vo)), xv, acc[u]);
        if (CORR) xs[u] += xv;
      }
    }
#pragma unroll
    for (int u = 0; u < U; ++u) {
      acc[u] = group_sum<L>(acc[u]);
      if (CORR) {
        xs[u] = group_sum<L>(xs[u]);
        const int len = cen[u] - cst[u];
        if (len > 0) acc[u] += static_cast<AT>(corr[cri[u]]) * (xs[u] / static_cast<AT>(len));
      }
      const int idx = it * STEP + g + u * G;
      if (idx < n) sink(idx, acc[u], cgc[u], cxo[u]);
    }
  }
}

template <typename T> struct Acc { using type = float; };
template <> struct Acc<double> { using type = double; };

// Row offsets of the CSR matrix.  When every row holds the same number of
// entries (kfix > 0) row r spans [r*kfix, (r+1)*kfix) and no offset is read,
// which spares the scattered row_ptr reads of the policy products.
struct RowIndex {
  const int* row_ptr;
  int kfix;
};

// Second phase of a sweep tile: q holds Q(s, a) of the tile's ns states
// (row-major, A per state).  One thread per state takes the minimum over
// a = 0..A-1 with a strict '<' (lowest action wins ties), writes Tv, pi and
// r0 = Tv - v, and accumulates max|Tv - v|, sum (Tv - v)^2 and max|Tv| into
// the tile's partials.
template <typename AT, typename XT, typename RT>
__device__ __forceinline__ void sweep_finish(int64_t s0, int ns, int A, const AT* q,
                                             const XT* __restrict__ v, double* __restrict__ Tv,
                                             int* __restrict__ pi, RT* __restrict__ r0,
                                             double4* __restrict__ partials, int tile) {
  double dmax = 0.0, dsum = 0.0, tmax = 0.0;
  for (int t = threadIdx.x; t < ns; t += kBlock) {
    const int64_t s = s0 + t;
    const AT* qs = q + t * A;
    AT best = qs[0];
    int arg = 0;
    bool nan = best != best;
    for (int a = 1; a < A; ++a) {
      const AT qa = qs[a];
      nan |= qa != qa;
      if (qa < best) {
        best = qa;
        arg = a;
      }
    }
    const double tv = nan ? NAN : static_cast<double>(best);
    if (Tv) Tv[s] = tv;
    if (pi) pi[s] = arg;
    const double d = tv - static_cast<double>(v[s]);
    if (r0) r0[s] = static_cast<RT>(d);
    dmax = max_nan(dmax, fabs(d));
    dsum = fma(d, d, dsum);
    tmax = max_nan(tmax, fabs(tv));
  }
  block_max_sum(dmax, dsum);
  double tm2 = 0.0;
  block_max_sum(tmax, tm2);
  if (threadIdx.x == 0) partials[tile] = make_double4(dmax, dsum, tmax, 0.0);
}

// Exclusive prefix sum of c[0..n) in LDS (n <= 4 * kBlock), in place;
// c[n] receives the total.  Every thread of the workgroup must call it.
__device__ __forceinline__ void block_exclusive_scan(int* c, int n) {
  __shared__ int wsum[kBlock];
  constexpr int P = 4;
  const int t = threadIdx.x;
  int loc[P], run = 0;
#pragma unroll
  for (int k = 0; k < P; ++k) {
    const int i = t * P + k;
    loc[k] = run;
    run += i < n ? c[i] : 0;
  }
  wsum[t] = run;
  __syncthreads();
  for (int off = 1; off < kBlock; off <<= 1) {
    const int add = t >= off ? wsum[t - off] : 0;
    __syncthreads();
    wsum[t] += add;
    __syncthreads();
  }
  const int before = t > 0 ? wsum[t - 1] : 0;
#pragma unroll
  for (int k = 0; k < P; ++k) {
    const int i = t * P + k;
    if (i < n) c[i] = before + loc[k];
  }
  if (t == kBlock - 1) c[n] = wsum[kBlock - 1];
  __syncthreads();
}

// ----------------------------------------------------------------------------
// K1: fused Bellman sweep
// ----------------------------------------------------------------------------
// Workgroup = tile of `tile_states` states (all A rows of each).  The tile's
// row offsets are staged in LDS with one coalesced pass.  Phase 1: lane groups
// compute Q(s,a) = g(s,a) + gamma * (P v)(s,a) into LDS.  Phase 2: one thread
// per state takes the minimum over a = 0..A-1 with a strict '<' (lowest action
// wins ties), writes Tv, pi and r0 = Tv - v, and accumulates max|Tv - v|,
// sum (Tv - v)^2 and max|Tv| into this workgroup's partials.
template <int L, int U, typename VT, typename XT, bool CORR, typename RT>
__device__ __forceinline__ void bellman_tile(
    int64_t S, int A, int tile_states, RowIndex rix,
    const int* __restrict__ col, const VT* __restrict__ val, const double* __restrict__ corr,
    const double* __restrict__ cost, const XT* __restrict__ v, double gamma,
    double* __restrict__ Tv, int* __restrict__ pi, RT* __restrict__ r0,
    double4* __restrict__ partials, int tile, double* lds_d) {
  using AT = typename Acc<XT>::type;
  const int tile_rows = tile_states * A;
  AT* q = reinterpret_cast<AT*>(lds_d);
  int* rp = reinterpret_cast<int*>(lds_d + tile_rows);  // tile_rows + 1 entries
  const int64_t s0 = static_cast<int64_t>(tile) * tile_states;
  const int ns = static_cast<int>(min<int64_t>(tile_states, S - s0));
  const int nrows = ns * A;
  const int64_t row0 = s0 * A;
  const AT gam = static_cast<AT>(gamma);
  // stage the tile's row offsets: loads first (unconditional), then LDS
  const int* __restrict__ row_ptr = rix.row_ptr;
  const int kfix = rix.kfix;
  if (kfix == 0) {
    for (int base = 0; base <= nrows; base += 5 * kBlock) {
      int buf[5];
#pragma unroll
      for (int k = 0; k < 5; ++k) {
        const int i = base + threadIdx.x + k * kBlock;
        buf[k] = row_ptr[row0 + (i <= nrows ? i : 0)];
      }
#pragma unroll
      for (int k = 0; k < 5; ++k) {
        const int i = base + threadIdx.x + k * kBlock;
        if (i <= nrows) rp[i] = buf[k];
      }
    }
    __syncthreads();
  }

  pipelined_rows<L, U, VT, XT, AT, CORR, true, false>(
      nrows,
      [&](int idx, int& st, int& en, int& ri, int& si) {
        ri = static_cast<int>(row0 + idx);
        if (kfix > 0) {
          st = ri * kfix;
          en = st + kfix;
        } else {
          st = rp[idx];
          en = rp[idx + 1];
        }
        si = -1;
      },
      col, val, v, S, cost, corr,
      [&](int idx, AT pv, double gc, XT) {
        // stored row idx of the tile is action idx / ns of state idx % ns
        if ((threadIdx.x % L) == 0) q[(idx % ns) * A + idx / ns] = fma(gam, pv, static_cast<AT>(gc));
      });
  __syncthreads();
  sweep_finish<AT, XT, RT>(s0, ns, A, q, v, Tv, pi, r0, partials, tile);
}

// Stage the selected rows of kApplyTile states: thread t loads pi(s0+t) and
// the two row offsets of the stored row of (s, pi(s)) (all independent loads).
__device__ __forceinline__ void stage_policy_rows(int64_t S, int64_t s0, int ns, int A, RowIndex rix,
                                                  const int* __restrict__ pi, int* st_l,
                                                  int* en_l, int* rw_l) {
  constexpr int KP = (kApplyTile + kBlock - 1) / kBlock;
  int pv[KP], a[KP], b[KP];
#pragma unroll
  for (int k = 0; k < KP; ++k) {
    const int t = threadIdx.x + k * kBlock;
    pv[k] = pi[s0 + (t < ns ? t : 0)];
  }
#pragma unroll
  for (int k = 0; k < KP; ++k) {
    const int t = threadIdx.x + k * kBlock;
    const int r = static_cast<int>(row_of(s0 + (t < ns ? t : 0), pv[k], A, S));
    pv[k] = r;
    if (rix.kfix > 0) {
      a[k] = r * rix.kfix;
      b[k] = a[k] + rix.kfix;
    } else {
      a[k] = rix.row_ptr[r];
      b[k] = rix.row_ptr[r + 1];
    }
  }
#pragma unroll
  for (int k = 0; k < KP; ++k) {
    const int t = threadIdx.x + k * kBlock;
    if (t < ns) {
      rw_l[t] = pv[k];
      st_l[t] = a[k];
      en_l[t] = b[k];
    }
  }
  __syncthreads();
}

// ----------------------------------------------------------------------------
// K2/K3/K10: products with P_pi, gathering the stored rows of (s, pi(s))
// ----------------------------------------------------------------------------
// MODE kApplyOp : y = x - gamma P_pi x
// MODE kApplyT  : y = g_pi + gamma P_pi x, partials (max|y - x|, sum (y-x)^2)
// MODE kApplyRes: y = g_pi - (x - gamma P_pi x), partials (max|y|, sum y^2)
// Each workgroup owns kApplyTile consecutive states.
template <int L, int U, int MODE, typename VT, typename XT, typename YT, bool CORR>
__device__ __forceinline__ void apply_tile(
    int64_t S, int A, RowIndex rix, const int* __restrict__ col,
    const VT* __restrict__ val, const double* __restrict__ corr,
    const double* __restrict__ cost, const int* __restrict__ pi, const XT* __restrict__ x,
    double gamma, YT* __restrict__ y, double4* __restrict__ partials, int tile) {
  using AT = typename Acc<XT>::type;
  __shared__ int st_l[kApplyTile], en_l[kApplyTile], rw_l[kApplyTile];
  const int64_t s0 = static_cast<int64_t>(tile) * kApplyTile;
  const int ns = static_cast<int>(min<int64_t>(kApplyTile, S - s0));
  const AT gam = static_cast<AT>(gamma);
  stage_policy_rows(S, s0, ns, A, rix, pi, st_l, en_l, rw_l);
  double dmax = 0.0, dsum = 0.0;

  pipelined_rows<L, U, VT, XT, AT, CORR, MODE != kApplyOp, true>(
      ns,
      [&](int idx, int& st, int& en, int& ri, int& si) {
        st = st_l[idx];
        en = en_l[idx];
        ri = rw_l[idx];
        si = static_cast<int>(s0 + idx);
      },
      col, val, x, S, cost, corr,
      [&](int ss, AT pv, double gc, XT xown) {
        if ((threadIdx.x % L) != 0) return;
        const int64_t s = s0 + ss;
        const AT xs_own = static_cast<AT>(xown);
        if (MODE == kApplyOp) {
          y[s] = static_cast<YT>(xs_own - gam * pv);
        } else if (MODE == kApplyT) {
          const AT yv = fma(gam, pv, static_cast<AT>(gc));
          y[s] = static_cast<YT>(yv);
          const double d = static_cast<double>(yv) - static_cast<double>(xs_own);
          dmax = max_nan(dmax, fabs(d));
          dsum = fma(d, d, dsum);
        } else {
          const double r = gc - (static_cast<double>(xs_own) -
                                 static_cast<double>(gam) * static_cast<double>(pv));
          y[s] = static_cast<YT>(r);
          dmax = max_nan(dmax, fabs(r));
          dsum = fma(r, r, dsum);
        }
      });
  if (MODE != kApplyOp) {
    block_max_sum(dmax, dsum);
    if (threadIdx.x == 0) partials[tile] = make_double4(dmax, dsum, 0.0, 0.0);
  }
}

// ----------------------------------------------------------------------------
// GMRES kernels (K4-K7) on (I - gamma P_pi)
// ----------------------------------------------------------------------------
// Basis vectors are stored unnormalised: column i of the orthonormal basis is
// ctl->scale[i] * U_i.  That lets the normalisation of a new vector ride on the
// next pass instead of costing a pass of its own.

// One Horner step of the polynomial preconditioner M^-1 = sum_{i<d} (gamma P_pi)^i
// (a truncated Neumann series of (I - gamma P_pi)^-1):  y = b + gamma P_pi x.
// d - 1 steps from x = b give M^-1 b.  The tile's b values are staged in LDS
// with its selected rows, so the sink issues no load of its own.
template <int L, int U, typename VT, typename XT, bool CORR>
__device__ __forceinline__ void horner_tile(int64_t S, int A, RowIndex rix, const int* __restrict__ col,
                                            const VT* __restrict__ val, const double* __restrict__ corr,
                                            const int* __restrict__ pi, const XT* __restrict__ x,
                                            const XT* __restrict__ b, double gamma, XT* __restrict__ y,
                                            int tile) {
  using AT = typename Acc<XT>::type;
  __shared__ int st_l[kApplyTile], en_l[kApplyTile], rw_l[kApplyTile];
  __shared__ XT b_l[kApplyTile];
  const int64_t s0 = static_cast<int64_t>(tile) * kApplyTile;
  const int ns = static_cast<int>(min<int64_t>(kApplyTile, S - s0));
  const AT gam = static_cast<AT>(gamma);
  for (int t = threadIdx.x; t < ns; t += kBlock) b_l[t] = b[s0 + t];
  stage_policy_rows(S, s0, ns, A, rix, pi, st_l, en_l, rw_l);  // its barrier publishes b_l
  pipelined_rows<L, U, VT, XT, AT, CORR, false, false>(
      ns,
      [&](int idx, int& st, int& en, int& ri, int& si) {
        st = st_l[idx];
        en = en_l[idx];
        ri = rw_l[idx];
        si = -1;
      },
      col, val, x, S, nullptr, corr,
      [&](int ss, AT pv, double, XT) {
        if ((threadIdx.x % L) == 0) y[s0 + ss] = static_cast<XT>(fma(gam, pv, static_cast<AT>(b_l[ss])));
      });
}

template <typename BT, int TILE = kApplyTile>
__device__ __forceinline__ void cgs_dots_tile(const BT* __restrict__ Ub, int64_t ldu, int j, int64_t s0, int ns,
                                              const double* w_lds, double* __restrict__ partials, int tile,
                                              int nb);

// K2+K4: w = scale_j * (I - gamma P_pi) U_j stored into U_{j+1}, and the
// workgroup's partial dot products sum_s U_i[s] w[s], i = 0..j (classical
// Gram-Schmidt, one pass over the basis).  partials[i * nb + tile].
template <int L, int U, typename VT, typename BT, bool CORR>
__device__ __forceinline__ void arnoldi_apply_tile(
    int64_t S, int A, RowIndex rix, const int* __restrict__ col,
    const VT* __restrict__ val, const double* __restrict__ corr, const int* __restrict__ pi,
    BT* __restrict__ Ub, int64_t ldu, int j, double gamma, const Ctl* __restrict__ ctl,
    double* __restrict__ partials, int tile, int nb, const BT* __restrict__ xin = nullptr) {
  using AT = typename Acc<BT>::type;
  __shared__ double w_lds[kApplyTile];
  __shared__ int st_l[kApplyTile], en_l[kApplyTile], rw_l[kApplyTile];
  const int64_t s0 = static_cast<int64_t>(tile) * kApplyTile;
  const int ns = static_cast<int>(min<int64_t>(kApplyTile, S - s0));
  const AT gam = static_cast<AT>(gamma);
  // the product's input: U_j, or (polynomial preconditioning) M^-1 U_j
  const BT* __restrict__ xj = xin ? xin : Ub + static_cast<int64_t>(j) * ldu;
  BT* __restrict__ w = Ub + static_cast<int64_t>(j + 1) * ldu;
  const double cj = ctl->scale[j];
  stage_policy_rows(S, s0, ns, A, rix, pi, st_l, en_l, rw_l);

  pipelined_rows<L, U, VT, BT, AT, CORR, false, true>(
      ns,
      [&](int idx, int& st, int& en, int& ri, int& si) {
        st = st_l[idx];
        en = en_l[idx];
        ri = rw_l[idx];
        si = static_cast<int>(s0 + idx);
      },
      col, val, xj, S, nullptr, corr,
      [&](int ss, AT pv, double, BT xown) {
        if ((threadIdx.x % L) != 0) return;
        const int64_t s = s0 + ss;
        const AT av = static_cast<AT>(xown) - gam * pv;
        const BT wv = static_cast<BT>(cj * static_cast<double>(av));
        w[s] = wv;
        w_lds[ss] = static_cast<double>(wv);
      });
  __syncthreads();
  cgs_dots_tile<BT>(Ub, ldu, j, s0, ns, w_lds, partials, tile, nb);
}

// The classical Gram-Schmidt dots of an Arnoldi tile: the workgroup's partial
// sum_s U_i[s] w[s] for i = 0..j into partials[i * nb + tile], with the tile's
// w values (already written to U_{j+1}) in w_lds.  Every thread must call it.
template <typename BT, int TILE>
__device__ __forceinline__ void cgs_dots_tile(const BT* __restrict__ Ub, int64_t ldu, int j, int64_t s0, int ns,
                                              const double* w_lds, double* __restrict__ partials, int tile,
                                              int nb) {
  __shared__ double red[kBlock / kWave][8];
  const int wv_id = threadIdx.x / kWave;
  constexpr int KS = TILE / kBlock;
  for (int i0 = 0; i0 <= j; i0 += 8) {
    double a8[8];
#pragma unroll
    for (int c = 0; c < 8; ++c) a8[c] = 0.0;
    BT ub[KS][8];
#pragma unroll
    for (int k = 0; k < KS; ++k) {
      const int t = threadIdx.x + k * kBlock;
      const int64_t s = s0 + (t < ns ? t : 0);
#pragma unroll
      for (int c = 0; c < 8; ++c) {
        const int col_i = i0 + c <= j ? i0 + c : j;
        ub[k][c] = Ub[static_cast<int64_t>(col_i) * ldu + s];
      }
    }
#pragma unroll
    for (int k = 0; k < KS; ++k) {
      const int t = threadIdx.x + k * kBlock;
      const double wt = t < ns ? w_lds[t] : 0.0;
#pragma unroll
      for (int c = 0; c < 8; ++c) {
        const double prod = fma(static_cast<double>(ub[k][c]), wt, a8[c]);
        a8[c] = (t < ns && i0 + c <= j) ? prod : a8[c];
      }
    }
#pragma unroll
    for (int c = 0; c < 8; ++c) a8[c] = wave_sum(a8[c]);
    if ((threadIdx.x & (kWave - 1)) == 0) {
#pragma unroll
      for (int c = 0; c < 8; ++c) red[wv_id][c] = a8[c];
    }
    __syncthreads();
    if (threadIdx.x < 8 && i0 + static_cast<int>(threadIdx.x) <= j) {
      double sum = red[0][threadIdx.x];
#pragma unroll
      for (int k = 1; k < kBlock / kWave; ++k) sum += red[k][threadIdx.x];
      partials[static_cast<int64_t>(i0 + threadIdx.x) * nb + tile] = sum;
    }
    __syncthreads();
  }
}

// Reduce column i (= blockIdx.x) of the dot partials: H[i, j] = scale_i * sum.
__device__ __forceinline__ void reduce_dots_body(const double* __restrict__ partials, int nb,
                                                 int j, Ctl* __restrict__ ctl, int i) {
  double s = strided_sum(partials + static_cast<int64_t>(i) * nb, nb, 0.0);
  double mx = 0.0;
  block_max_sum(mx, s);
  if (threadIdx.x == 0) {
    const double h = ctl->scale[i] * s;
    ctl->H[i + j * (kMaxRestart + 1)] = h;
    ctl->hc[i] = h * ctl->scale[i];
  }
}

// CGS2, second pass: the dots of the once-orthogonalised w = U_{j+1} with
// U_0..U_j, as in the first pass (same tiles, same order).
template <typename BT>
__device__ __forceinline__ void cgs2_dots_tile(int64_t S, const BT* __restrict__ Ub, int64_t ldu, int j,
                                               double* __restrict__ partials, int tile, int nb) {
  __shared__ double w_lds[kApplyTile];
  const int64_t s0 = static_cast<int64_t>(tile) * kApplyTile;
  const int ns = static_cast<int>(min<int64_t>(kApplyTile, S - s0));
  const BT* __restrict__ w = Ub + static_cast<int64_t>(j + 1) * ldu;
  for (int t = threadIdx.x; t < ns; t += kBlock) w_lds[t] = static_cast<double>(w[s0 + t]);
  __syncthreads();
  cgs_dots_tile<BT>(Ub, ldu, j, s0, ns, w_lds, partials, tile, nb);
}

// CGS2, second pass: column i (= blockIdx.x) of the dots; the coefficient h2
// is added to H[i, j], becomes the next update's coefficient, and its square
// is kept for the loss-of-orthogonality measure.
__device__ __forceinline__ void reduce_dots2_body(const double* __restrict__ partials, int nb, int j,
                                                  Ctl* __restrict__ ctl, int i) {
  double s = strided_sum(partials + static_cast<int64_t>(i) * nb, nb, 0.0);
  double mx = 0.0;
  block_max_sum(mx, s);
  if (threadIdx.x == 0) {
    const double h2 = ctl->scale[i] * s;
    ctl->H[i + j * (kMaxRestart + 1)] += h2;
    ctl->hc[i] = h2 * ctl->scale[i];
    ctl->h2sq[i] = h2 * h2;
  }
}

// K5: w <- w - sum_{i<=j} hc_i U_i, with the workgroup's partial ||w||^2.
// kUpdTile states per workgroup, KU per thread; the basis loop is unrolled by
// 4 so that 4*KU independent loads are in flight per thread.
template <typename BT>
__device__ __forceinline__ void arnoldi_update_body(int64_t S, BT* __restrict__ Ub, int64_t ldu,
                                                    int j, const Ctl* __restrict__ ctl,
                                                    double* __restrict__ partials, int blk) {
  __shared__ double hc[kMaxRestart + 4];
  if (threadIdx.x < kMaxRestart + 4) hc[threadIdx.x] = threadIdx.x <= j ? ctl->hc[threadIdx.x] : 0.0;
  __syncthreads();
  constexpr int KU = kUpdTile / kBlock;
  const int64_t s0 = static_cast<int64_t>(blk) * kUpdTile + threadIdx.x;
  BT* __restrict__ w = Ub + static_cast<int64_t>(j + 1) * ldu;
  double acc[KU];
  bool in[KU];
#pragma unroll
  for (int k = 0; k < KU; ++k) {
    const int64_t s = s0 + k * kBlock;
    in[k] = s < S;
    acc[k] = in[k] ? static_cast<double>(w[s]) : 0.0;
  }
  for (int i = 0; i <= j; i += 4) {
    BT u4[4][KU];
#pragma unroll
    for (int q = 0; q < 4; ++q) {
      const BT* __restrict__ ui = Ub + static_cast<int64_t>(i + q <= j ? i + q : j) * ldu;
#pragma unroll
      for (int k = 0; k < KU; ++k) u4[q][k] = ui[in[k] ? s0 + k * kBlock : 0];
    }
#pragma unroll
    for (int q = 0; q < 4; ++q) {
      const double c = -hc[i + q];
#pragma unroll
      for (int k = 0; k < KU; ++k) {
        const double t = fma(c, static_cast<double>(u4[q][k]), acc[k]);
        acc[k] = i + q <= j ? t : acc[k];
      }
    }
  }
  double sq = 0.0;
#pragma unroll
  for (int k = 0; k < KU; ++k) {
    if (in[k]) {
      const BT wv = static_cast<BT>(acc[k]);
      w[s0 + k * kBlock] = wv;
      const double wd = static_cast<double>(wv);
      sq = fma(wd, wd, sq);
    }
  }
  double mx = 0.0;
  block_max_sum(mx, sq);
  if (threadIdx.x == 0) partials[blk] = sq;
}

// K6: ||w|| from the partials, then the Givens update of column j, the
// residual estimate and the stop decision.  One workgroup; the back
// substitution at the end of a cycle runs column by column over the threads.
__device__ __forceinline__ void norm_givens_body(const double* __restrict__ partials, int nb,
                                                 int j, int m, Ctl* __restrict__ ctl, bool gs2 = false) {
  __shared__ int s_done;
  __shared__ double s_t[kMaxRestart];
  __shared__ double s_h[kMaxRestart + 2], s_cs[kMaxRestart], s_sn[kMaxRestart];
  const int ld = kMaxRestart + 1;
  const int n = j + 1;
  // the column and the earlier rotations, staged with one parallel round trip
  if (threadIdx.x <= j) s_h[threadIdx.x] = ctl->H[threadIdx.x + j * ld];
  if (threadIdx.x < j) {
    s_cs[threadIdx.x] = ctl->cs[threadIdx.x];
    s_sn[threadIdx.x] = ctl->sn[threadIdx.x];
  }
  double s = strided_sum(partials, nb, 0.0);
  double mx = 0.0;
  block_max_sum(mx, s);  // its barriers also publish the staged values
  if (threadIdx.x == 0) {
    const double hn = sqrt(s);
    if (gs2) {
      // size of the second Gram-Schmidt correction relative to the final vector
      double q = 0.0;
      for (int i = 0; i <= j; ++i) q += ctl->h2sq[i];
      const double loss = hn > 0.0 ? sqrt(q) / hn : 0.0;
      ctl->orth_loss = max_nan(ctl->orth_loss, loss);
    }
    // size of the column before orthogonalisation, for the breakdown test
    double colnorm2 = hn * hn;
    for (int i = 0; i <= j; ++i) colnorm2 += s_h[i] * s_h[i];
    // apply the earlier rotations; `carry` is entry i of the partly rotated column
    double carry = s_h[0];
    for (int i = 0; i < j; ++i) {
      const double nx = s_h[i + 1];
      const double t = s_cs[i] * carry + s_sn[i] * nx;
      carry = -s_sn[i] * carry + s_cs[i] * nx;
      s_h[i] = t;
    }
    const double a = carry, b = hn;
    const double r = hypot(a, b);
    double c = 1.0, sn = 0.0;
    if (r > 0.0) {
      c = a / r;
      sn = b / r;
    }
    ctl->cs[j] = c;
    ctl->sn[j] = sn;
    s_h[j] = r;
    s_h[j + 1] = 0.0;
    const double gj = ctl->g[j];
    ctl->g[j + 1] = -sn * gj;
    ctl->g[j] = c * gj;
    const double est = fabs(ctl->g[j + 1]);
    ctl->res_est = est;
    ctl->steps += 1;
    const bool brk = !(hn > 1e-14 * sqrt(colnorm2));
    ctl->scale[j + 1] = brk ? 0.0 : 1.0 / hn;
    ctl->j = n;
    int done = 0;
    if (est <= ctl->tol_cycle) done = 1;
    if (est <= ctl->tol) ctl->converged = 1;
    if (brk) {
      ctl->breakdown = 1;
      done = 1;
    }
    if (n >= m) done = 1;
    if (!(est == est)) done = 1;
    s_done = done;
  }
  __syncthreads();
  if (threadIdx.x <= j + 1) ctl->H[threadIdx.x + j * ld] = s_h[threadIdx.x];
  if (!s_done) return;
  __syncthreads();
  // back substitution R y = g, R = H[0:n, 0:n] upper triangular
  if (threadIdx.x < n) s_t[threadIdx.x] = ctl->g[threadIdx.x];
  __syncthreads();
  for (int i = n - 1; i >= 0; --i) {
    // column j is read from LDS, the earlier columns come from earlier launches
    const double* hcol = i == j ? s_h : ctl->H + i * ld;
    const double yi = s_t[i] / hcol[i];
    __syncthreads();
    if (threadIdx.x == 0) ctl->y[i] = yi;
    if (threadIdx.x < i) s_t[threadIdx.x] -= hcol[threadIdx.x] * yi;
    __syncthreads();
  }
  if (threadIdx.x == 0) ctl->done = 1;
}

// K7: x += sum_{i < n} y_i scale_i U_i for the n = ctl->j completed columns.
template <typename BT, typename XT>
__device__ __forceinline__ void gmres_update_x_body(int64_t S, XT* __restrict__ x,
                                                    const BT* __restrict__ Ub, int64_t ldu,
                                                    const Ctl* __restrict__ ctl, int blk) {
  const int n = ctl->j;
  if (n == 0) return;
  __shared__ double coef[kMaxRestart + 4];
  if (threadIdx.x < kMaxRestart + 4)
    coef[threadIdx.x] = threadIdx.x < n ? ctl->y[threadIdx.x] * ctl->scale[threadIdx.x] : 0.0;
  __syncthreads();
  constexpr int KU = kUpdTile / kBlock;
  const int64_t s0 = static_cast<int64_t>(blk) * kUpdTile + threadIdx.x;
  double d[KU];
  bool in[KU];
#pragma unroll
  for (int k = 0; k < KU; ++k) {
    d[k] = 0.0;
    in[k] = s0 + k * kBlock < S;
  }
  for (int i = 0; i < n; i += 4) {
    BT u4[4][KU];
#pragma unroll
    for (int q = 0; q < 4; ++q) {
      const BT* __restrict__ ui = Ub + static_cast<int64_t>(i + q < n ? i + q : n - 1) * ldu;
#pragma unroll
      for (int k = 0; k < KU; ++k) u4[q][k] = ui[in[k] ? s0 + k * kBlock : 0];
    }
#pragma unroll
    for (int q = 0; q < 4; ++q)
#pragma unroll
      for (int k = 0; k < KU; ++k) {
        const double t = fma(coef[i + q], static_cast<double>(u4[q][k]), d[k]);
        d[k] = i + q < n ? t : d[k];
      }
  }
#pragma unroll
  for (int k = 0; k < KU; ++k) {
    const int64_t s = s0 + k * kBlock;
    if (in[k]) x[s] = static_cast<XT>(static_cast<double>(x[s]) + d[k]);
  }
}

// ----------------------------------------------------------------------------
// reductions of (max, sum) partials and the control-block transitions
// ----------------------------------------------------------------------------


__device__ __forceinline__ void reduce_ms_body(const double4* __restrict__ partials, int nb,
                                               int mode, int first_cycle, double alpha,
                                               double floor_rel, Ctl* __restrict__ ctl) {
  double mx = 0.0, sm = 0.0, am = 0.0, unused = 0.0;
  for (int b = threadIdx.x; b < nb; b += kBlock) {
    const double4 p = partials[b];
    mx = max_nan(mx, p.x);
    sm += p.y;
    am = max_nan(am, p.z);
  }
  block_max_sum(mx, sm);
  block_max_sum(am, unused);
  if (threadIdx.x != 0) return;
  ctl->res_max = mx;
  ctl->sumsq = sm;
  ctl->aux_max = am;
  if (mode == kRedGmresStart) {
    const double beta = sqrt(sm);
    ctl->beta = beta;
    if (first_cycle) {
      ctl->beta0 = beta;
      ctl->tol = alpha * beta;
      ctl->steps = 0;
      ctl->converged = 0;
    }
    // a cycle never asks for more relative reduction than its arithmetic can
    // give (floor_rel > 0 for float32 Arnoldi steps); float64 restarts catch up
    const double tol_cycle = fmax(ctl->tol, floor_rel * beta);
    ctl->res_est = beta;
    ctl->g[0] = beta;
    ctl->scale[0] = beta > 0.0 ? 1.0 / beta : 0.0;
    ctl->j = 0;
    ctl->breakdown = 0;
    ctl->done = 0;
    if (!(beta > tol_cycle)) {
      ctl->done = 1;
      if (beta <= ctl->tol) ctl->converged = 1;
    }
    ctl->tol_cycle = tol_cycle;
  } else if (mode == kRedRichardson) {
    if (first_cycle) ctl->tol = alpha * mx;
    ctl->steps += 1;
    ctl->rich_cur ^= 1;
    ctl->res_est = mx;
    if (mx <= ctl->tol || !(mx == mx)) {
      ctl->done = 1;
      ctl->converged = mx <= ctl->tol ? 1 : 0;
    }
  }
}

// ----------------------------------------------------------------------------
// K9: reduced-precision copies of P, and casts
// ----------------------------------------------------------------------------
// IEEE binary64 -> binary16 with round-to-nearest-even, taken directly from
// the binary64 bits (no intermediate float32 rounding).
__device__ __forceinline__ unsigned short f64_to_f16_bits(double x) {
  unsigned long long b = static_cast<unsigned long long>(__double_as_longlong(x));
  const unsigned short sign = static_cast<unsigned short>((b >> 48) & 0x8000u);
  b &= 0x7FFFFFFFFFFFFFFFull;
  const int e = static_cast<int>(b >> 52);
  const unsigned long long frac = b & ((1ull << 52) - 1);
  if (e == 0x7FF) return sign | 0x7C00u | (frac ? 0x200u : 0u);
  if (e == 0) return sign;  // binary64 subnormals are far below the binary16 range
  const int E = e - 1023;
  if (E > 15) return sign | 0x7C00u;
  const unsigned long long mant = frac | (1ull << 52);
  const int shift = E >= -14 ? 42 : 28 - E;
  if (shift >= 54) return sign;
  unsigned long long q = mant >> shift;
  const unsigned long long rem = mant & ((1ull << shift) - 1);
  const unsigned long long half = 1ull << (shift - 1);
  if (rem > half || (rem == half && (q & 1ull))) ++q;
  if (E >= -14) {
    int Eo = E;
    if (q == (1ull << 11)) {
      q >>= 1;
      ++Eo;
    }
    if (Eo + 15 >= 31) return sign | 0x7C00u;
    return sign | static_cast<unsigned short>(((Eo + 15) << 10) | (q & 0x3FFu));
  }
  return sign | static_cast<unsigned short>(q);  // q == 0x400 is the smallest normal
}

}  // namespace mdp

