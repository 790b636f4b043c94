// XCD-partitioned P_pi products for large vectors.
//
// When x spans many times one XCD's 4 MB L2 and a row's columns fall anywhere
// in it, each gather of a plain product pulls a line from the Infinity Cache,
// which serves about 64G gathers/s; gathers that stay inside each XCD's L2 run
// about three times faster.  The dispatcher hands workgroup w to XCD w % 8,
// so the product is cut by columns to match: the columns fall into 8 slices
// (8 P slices in P passes when x is larger than 8 x 4 MB), a copy of P_pi
// holds each slice's entries tile by tile, and workgroup w streams the
// entries of slice (w % 8) of tile w / 8, so each XCD's L2 only ever holds its
// own slice of x.  Every workgroup writes its slice's part of (P_pi x)[s] for
// the tile's states; a second kernel adds the parts in slice order and
// finishes the Arnoldi step exactly as the plain product kernel does (new
// basis vector and the classical Gram-Schmidt dot partials).
//
// Where the columns stay near their rows (no column-blocked copy on the
// handle) the copy has one slice: it is P_pi stored contiguously, tile by
// tile, and the product streams each tile's rows as one segment, which reads
// fewer partly used lines than gathering the selected rows through row_ptr.
//
// The copy is formed once per policy, with no host round trip: a placing
// kernel (entries of each state in each slice, each state's start in its
// tile's segments, the segments placed by atomic adds) and a scatter kernel
// that walks each selected row once, in CSR order, so inside a slice a
// state's entries keep their CSR order.  A state's part in a slice is
// the fma chain over its entries there, started from 0, and the parts are
// added in slice order: results are deterministic.
#include <algorithm>

#include "device.h"

namespace mdp {

namespace {

constexpr int kPPTile = 4 * kBlock;                    // states per tile (4 per thread)
constexpr int kPPMaxBlocks = 16;                       // slices (two passes)
constexpr int64_t kPPSliceBytes = int64_t{4} << 20;   // x bytes per slice: one XCD's L2
// Nontemporal accesses for the slice parts and the state starts: each is touched once per pass, and
// kept out of the way they leave the L2 to the slice of the gathered vector
// (on the 4M-state workload: sweep 11.7 -> 11.2 ms, product 809 -> 790 us).
#ifndef MDP_NT_PARTS
#define MDP_NT_PARTS 1
#endif
#ifndef MDP_PP_CHUNK
#define MDP_PP_CHUNK 1024
#endif
constexpr int kPPChunk = MDP_PP_CHUNK;                 // entries staged per step
static_assert(kPPChunk % kBlock == 0, "chunk of whole rounds");

__device__ __forceinline__ void selected_row(int64_t s, const int* __restrict__ pi, int A, int64_t S, RowIndex rix,
                                             int* a, int* e) {
  const int64_t r = row_of(s, pi[s], A, S);
  if (rix.kfix > 0) {
    *a = static_cast<int>(r * rix.kfix);
    *e = *a + rix.kfix;
  } else {
    *a = rix.row_ptr[r];
    *e = rix.row_ptr[r + 1];
  }
}

// A tile's selected rows are read two at a time per wavefront: each half of
// the wavefront (32 lanes) takes one state and reads its row 32 entries at a
// time (coalesced); ballots over the lanes' slice numbers give the per-slice
// counts, and lane b of a half keeps the count of slice b.  The loop bounds
// are uniform over the wavefront (both halves run as many chunks as the
// longer row), so every ballot sees all 64 lanes.  The next pair's row bounds
// are loaded before the current pair is worked on.
constexpr int kPPWaves = kBlock / kWave;

// A state's part in slice k (read once).
__device__ __forceinline__ double ld_part(const double* __restrict__ part, int64_t S, int k, int64_t s) {
#if MDP_NT_PARTS
  return __builtin_nontemporal_load(part + static_cast<int64_t>(k) * S + s);
#else
  return part[static_cast<int64_t>(k) * S + s];
#endif
}

__device__ __forceinline__ uint32_t half_ballot(bool p, int half) {
  return static_cast<uint32_t>(__ballot(p) >> (32 * half));
}

// Walk the tile's selected rows in pairs: body(i, a, n, cf, vf) for this
// half's state i (a = first entry, n = entries; n = 0 past the tile), with the
// row's first chunk of columns (and, VAL, values) already loaded into cf, vf
// (lane hl: entry hl, when hl < n).  The wavefronts take pairs in turn, so the
// workgroup reads neighbouring rows together (giving each wavefront a
// contiguous quarter of the tile made the scatter 16% slower), a batch of
// pairs at a time, so that the loads of several rows are in flight while one
// row is worked on.
#ifndef MDP_PP_WALK_DIRECT
#define MDP_PP_WALK_DIRECT 8
#endif
#ifndef MDP_PP_WALK_STAGED
#define MDP_PP_WALK_STAGED 4
#endif

// Row bounds computed per batch: the batch's first chunks are loaded
// together and the next batch's bounds before the bodies run.  On the
// 4M-state, 24-column workload (uniform rows, bounds from the policy entry
// alone) batches of four pairs took placing 624 -> 578 us and scattering
// 1127 -> 1041 us per policy against one pair at a time, and batches of
// eight scatter in 972 us (on the maze, whose rows now take the staged walk,
// eight slowed this walk's scatter from 534 to 743 us).
template <bool VAL, typename Body>
__device__ __forceinline__ void walk_pairs_direct(int64_t S, int A, RowIndex rix, const int* __restrict__ pi,
                                                  int64_t s0, int ns, const int* __restrict__ col,
                                                  const double* __restrict__ val, Body body) {
  constexpr int kWalk = MDP_PP_WALK_DIRECT;
  const int half = (threadIdx.x % kWave) / 32, wave = threadIdx.x / kWave, hl = threadIdx.x % 32;
  constexpr int kStep = 2 * kPPWaves;
  const int lo = 2 * wave;  // the wavefront's first pair (uniform over the wavefront)
  int a[kWalk], e[kWalk];
#pragma unroll
  for (int d = 0; d < kWalk; ++d) {
    const int i = lo + half + d * kStep;
    a[d] = e[d] = 0;
    if (i < ns) selected_row(s0 + i, pi, A, S, rix, &a[d], &e[d]);
  }
  for (int ib = lo; ib < ns; ib += kWalk * kStep) {
    int ia[kWalk], na[kWalk], cf[kWalk];
    double vf[kWalk];
#pragma unroll
    for (int d = 0; d < kWalk; ++d) {
      ia[d] = a[d];
      na[d] = e[d] - a[d];
      cf[d] = hl < na[d] ? col[a[d] + hl] : 0;
      vf[d] = VAL && hl < na[d] ? val[a[d] + hl] : 0.0;
    }
#pragma unroll
    for (int d = 0; d < kWalk; ++d) {
      const int i = ib + half + (kWalk + d) * kStep;
      a[d] = e[d] = 0;
      if (i < ns) selected_row(s0 + i, pi, A, S, rix, &a[d], &e[d]);
    }
#pragma unroll
    for (int d = 0; d < kWalk; ++d) body(ib + half + d * kStep, ia[d], na[d], cf[d], vf[d]);
  }
}

// Row bounds staged in LDS first (every policy entry and row offset of the
// tile loaded at once), and the next batch's first chunks loaded before the
// current batch is worked on, so one round trip is in flight behind the
// work instead of the chain policy -> row offsets -> columns per batch.  On
// the maze (rows through row_ptr) placing 419 -> 267 us and scattering
// 534 -> 391 us per policy; on the uniform rows above it was slower (663 and
// 1080 us: the staging costs the placing kernel occupancy, 5 waves per SIMD
// instead of 7).
template <bool VAL, typename Body>
__device__ __forceinline__ void walk_pairs_staged(int64_t S, int A, RowIndex rix, const int* __restrict__ pi,
                                                  int64_t s0, int ns, const int* __restrict__ col,
                                                  const double* __restrict__ val, Body body) {
  constexpr int kWalk = MDP_PP_WALK_STAGED;
  __shared__ int b_lo[kPPTile], b_n[kPPTile];
#pragma unroll
  for (int k = 0; k < kPPTile / kBlock; ++k) {
    const int i = threadIdx.x + k * kBlock;
    int a = 0, e = 0;
    if (i < ns) selected_row(s0 + i, pi, A, S, rix, &a, &e);
    b_lo[i] = a;
    b_n[i] = e - a;
  }
  __syncthreads();
  const int half = (threadIdx.x % kWave) / 32, wave = threadIdx.x / kWave, hl = threadIdx.x % 32;
  constexpr int kStep = 2 * kPPWaves;
  const int lo = 2 * wave;  // the wavefront's first pair (uniform over the wavefront)
  int cf[kWalk];
  double vf[kWalk];
  auto load = [&](int ib, int (&c)[kWalk], double (&v)[kWalk]) {
#pragma unroll
    for (int d = 0; d < kWalk; ++d) {
      const int i = ib + half + d * kStep;
      const int a = i < ns ? b_lo[i] : 0, n = i < ns ? b_n[i] : 0;
      c[d] = hl < n ? col[a + hl] : 0;
      v[d] = VAL && hl < n ? val[a + hl] : 0.0;
    }
  };
  load(lo, cf, vf);
  for (int ib = lo; ib < ns; ib += kWalk * kStep) {
    int cn[kWalk];
    double vn[kWalk];
    load(ib + kWalk * kStep, cn, vn);
#pragma unroll
    for (int d = 0; d < kWalk; ++d) {
      const int i = ib + half + d * kStep;
      body(i, i < ns ? b_lo[i] : 0, i < ns ? b_n[i] : 0, cf[d], vf[d]);
    }
#pragma unroll
    for (int d = 0; d < kWalk; ++d) {
      cf[d] = cn[d];
      vf[d] = vn[d];
    }
  }
}

// STAGED: row bounds from LDS (rows through row_ptr); else computed per
// batch (uniform rows, whose bounds need only the policy entry).
template <bool VAL, bool STAGED, typename Body>
__device__ __forceinline__ void walk_pairs(int64_t S, int A, RowIndex rix, const int* __restrict__ pi, int64_t s0,
                                           int ns, const int* __restrict__ col, const double* __restrict__ val,
                                           Body body) {
  if constexpr (STAGED)
    walk_pairs_staged<VAL>(S, A, rix, pi, s0, ns, col, val, body);
  else
    walk_pairs_direct<VAL>(S, A, rix, pi, s0, ns, col, val, body);
}

// Forming the copy, first kernel (tile t): per-state slice counts, each
// state's start inside the tile's segment of each slice (rel[b * S + s]), and
// one atomic add per slice on *fill that places the segment in the copy
// (seg[b * ntiles + t] = first entry, length).  Where a segment lands depends
// on the order of the atomic adds; what it holds does not, nor does any sum.
// Needs rows of at most 255 entries and at most 65535 entries per segment
// (guaranteed on the host from the longest row of the MDP).
template <bool STAGED>
__global__ __launch_bounds__(kBlock) void k_pp_place(int64_t S, int A, RowIndex rix, const int* __restrict__ col,
                                                     const int* __restrict__ pi, int slice, int nblk, int ntiles,
                                                     uint16_t* __restrict__ rel, int2* __restrict__ seg,
                                                     int* __restrict__ fill, const int* __restrict__ changed) {
  if (*changed == 0) return;  // the copy already holds this policy (the same for every workgroup)
  __shared__ __align__(16) uint8_t c8[kPPMaxBlocks][kPPTile];
  __shared__ int wtot[kPPWaves][kPPMaxBlocks];
  const int t = blockIdx.x;
  const int64_t s0 = static_cast<int64_t>(t) * kPPTile;
  const int ns = static_cast<int>(min<int64_t>(kPPTile, S - s0));
  const int hl = threadIdx.x % 32, half = (threadIdx.x % kWave) / 32;
  walk_pairs<false, STAGED>(S, A, rix, pi, s0, ns, col, nullptr, [&](int i, int a, int n, int cf, double) {
    const int nmax = max(n, __shfl_xor(n, 32));
    int cnt = 0;  // lane hl < nblk: entries of slice hl
    for (int c0 = 0; c0 < nmax; c0 += 32) {
      const int b = c0 + hl < n ? (c0 == 0 ? cf : col[a + c0 + hl]) / slice : -1;
      for (int bb = 0; bb < nblk; ++bb) {
        const uint32_t m = half_ballot(b == bb, half);
        if (hl == bb) cnt += __popc(m);
      }
    }
    if (i < ns && hl < nblk) c8[hl][i] = static_cast<uint8_t>(cnt);
  });
  __syncthreads();
  // The exclusive scans of every slice's counts at once: thread u owns states
  // 4u .. 4u + 3 (one 32-bit word of c8[b]); a wavefront scan of the thread
  // sums, then the sums of the earlier wavefronts.  Two barriers in all
  // (one scan of the 1024 counts per slice took some 18; placing 580 -> 544 us
  // per policy on the 4M-state, 24-column workload, 266 -> 225 us on the maze).
  static_assert(kPPTile == 4 * kBlock, "one word of four counts per thread");
  const int u = threadIdx.x, lane = u % kWave, wv = u / kWave;
  auto counts = [&](int b, int (&c)[4]) {
    uint32_t w;
    __builtin_memcpy(&w, &c8[b][4 * u], sizeof(w));  // one aligned 32-bit LDS read
    int sum = 0;
#pragma unroll
    for (int k = 0; k < 4; ++k) {
      c[k] = 4 * u + k < ns ? static_cast<int>((w >> (8 * k)) & 0xffu) : 0;  // past the tile: unwritten
      sum += c[k];
    }
    return sum;
  };
  auto wave_incl = [&](int x) {
#pragma unroll
    for (int off = 1; off < kWave; off <<= 1) {
      const int y = __shfl_up(x, off, kWave);
      x += lane >= off ? y : 0;
    }
    return x;
  };
  for (int b = 0; b < nblk; ++b) {
    int c[4];
    const int incl = wave_incl(counts(b, c));
    if (lane == kWave - 1) wtot[wv][b] = incl;
  }
  __syncthreads();
  for (int b = 0; b < nblk; ++b) {
    int c[4];
    const int own = counts(b, c);
    int run = wave_incl(own) - own;
    for (int q = 0; q < wv; ++q) run += wtot[q][b];
    uint16_t* __restrict__ rb = rel + static_cast<int64_t>(b) * S + s0;
#pragma unroll
    for (int k = 0; k < 4; ++k) {
      if (4 * u + k < ns) rb[4 * u + k] = static_cast<uint16_t>(run);
      run += c[k];
    }
    if (u == 0) {
      int len = 0;
      for (int q = 0; q < kPPWaves; ++q) len += wtot[q][b];
      seg[static_cast<int64_t>(b) * ntiles + t] = make_int2(atomicAdd(fill, len), len);
    }
  }
}

// Forming the copy, second kernel: the selected rows of tile t scattered into
// the tile's segments.  An entry's place is its segment's start, its state's
// start there (rel), the entries of its state and slice in earlier chunks of
// the row, and those before it in its chunk (from the ballot), so each state
// keeps its CSR order inside every slice.
template <bool STAGED>
__global__ __launch_bounds__(kBlock) void k_pp_scatter(int64_t S, int A, RowIndex rix, const int* __restrict__ col,
                                                       const double* __restrict__ val, const int* __restrict__ pi,
                                                       int slice, int nblk, int ntiles, const int2* __restrict__ seg,
                                                       const uint16_t* __restrict__ rel, int* __restrict__ pcol,
                                                       double* __restrict__ pval, const int* __restrict__ changed) {
  if (*changed == 0) return;  // the copy already holds this policy
  __shared__ int base[kPPMaxBlocks];
  const int t = blockIdx.x;
  const int64_t s0 = static_cast<int64_t>(t) * kPPTile;
  const int ns = static_cast<int>(min<int64_t>(kPPTile, S - s0));
  const int hl = threadIdx.x % 32, half = (threadIdx.x % kWave) / 32;
  if (threadIdx.x < nblk) base[threadIdx.x] = seg[static_cast<int64_t>(threadIdx.x) * ntiles + t].x;
  __syncthreads();
  walk_pairs<true, STAGED>(S, A, rix, pi, s0, ns, col, val, [&](int i, int a, int n, int cf, double vf) {
    const int nmax = max(n, __shfl_xor(n, 32));
    // lane hl < nblk: the state's next place in slice hl
    int next = (i < ns && hl < nblk) ? base[hl] + rel[static_cast<int64_t>(hl) * S + s0 + i] : 0;
    for (int c0 = 0; c0 < nmax; c0 += 32) {
      const bool valid = c0 + hl < n;
      const int q = a + c0 + hl;
      const int c = valid ? (c0 == 0 ? cf : col[q]) : 0;
      const double v = valid ? (c0 == 0 ? vf : val[q]) : 0.0;
      const int b = valid ? c / slice : -1;
      uint32_t same = 0;
      int add = 0;
      for (int bb = 0; bb < nblk; ++bb) {
        const uint32_t m = half_ballot(b == bb, half);
        if (b == bb) same = m;
        if (hl == bb) add = __popc(m);
      }
      const int first = __shfl(next, (threadIdx.x % kWave) - hl + (b < 0 ? 0 : b));
      if (valid) {
        const int d = first + __popc(same & ((1u << hl) - 1u));
        pcol[d] = c;  // plain stores: the L2 gathers the short runs into whole lines
        pval[d] = v;
      }
      next += add;
    }
  });
}

// Has the policy changed since the copy was formed?  snap holds the policy
// of the last formation: every entry is compared and then overwritten, and
// *changed is set when any differs (or always, with force).  The formation
// kernels exit at once when it stays 0, so a policy that the greedy step
// left as it was costs one pass over 2 x 4 S bytes instead of a formation
// (on the 4M-state, 24-column workload the last two of a solve's six).
__global__ __launch_bounds__(kBlock) void k_pp_policy_changed(int64_t S, const int* __restrict__ pi,
                                                              int* __restrict__ snap, int force,
                                                              int* __restrict__ changed) {
  int diff = force;
  for (int64_t s = static_cast<int64_t>(blockIdx.x) * kBlock + threadIdx.x; s < S;
       s += static_cast<int64_t>(gridDim.x) * kBlock) {
    const int p = pi[s];
    diff |= snap[s] != p;
    snap[s] = p;
  }
  if (__syncthreads_or(diff) && threadIdx.x == 0) atomicOr(changed, 1);
}

// The longest row of the MDP (stored offsets), into *out.
__global__ __launch_bounds__(kBlock) void k_longest_row(const int* __restrict__ rp, int64_t rows,
                                                        unsigned* __restrict__ out) {
  int m = 0;
  for (int64_t r = static_cast<int64_t>(blockIdx.x) * kBlock + threadIdx.x; r < rows;
       r += static_cast<int64_t>(gridDim.x) * kBlock)
    m = max(m, rp[r + 1] - rp[r]);
  double mx = static_cast<double>(m), sm = 0.0;
  block_max_sum(mx, sm);
  if (threadIdx.x == 0) atomicMax(out, static_cast<unsigned>(mx));
}

// Slice parts of P_pi x: workgroup w takes slice pass * 8 + w % 8 of tile w / 8
// and writes part[b * S + s] for the tile's states.  The segment is streamed in
// chunks of kPPChunk entries: every thread loads every kBlock-th entry
// (coalesced), gathers x from the XCD's slice and leaves the (value, x) pair in
// LDS, with the next chunk's loads issued first; then each thread carries its
// states (at most 4) through the chunk.  Exits at once when the GMRES cycle is
// done.
// The sums over slice b of tile t (its states s0 + threadIdx.x + k * kBlock,
// k < 4, into sum[k]; 0 past the tile) of the copy's entries times x.
// Every thread must call it; lp and lx are the chunk's LDS staging.
template <typename XT>
__device__ __forceinline__ void pp_tile_sums(int64_t S, int ntiles, int b, int t, int64_t s0, int ns,
                                             const uint16_t* __restrict__ rel, const int2* __restrict__ seg,
                                             const int* __restrict__ pcol, const double* __restrict__ pval,
                                             const XT* __restrict__ x, double* lp, double* lx, double (&sum)[4]) {
  constexpr int EPT = kPPChunk / kBlock;
  const int2 sg = seg[static_cast<int64_t>(b) * ntiles + t];
  const int seg0 = sg.x;
  const int n = sg.y;
  const uint16_t* __restrict__ rl = rel + static_cast<int64_t>(b) * S + s0;
  const int* __restrict__ cc = pcol + seg0;
  const double* __restrict__ cv = pval + seg0;
  const Gather<XT> gx(x, S);
  int st[4], en[4];
#pragma unroll
  for (int k = 0; k < 4; ++k) {
    const int i = threadIdx.x + k * kBlock;
    const bool valid = i < ns;
#if MDP_NT_PARTS
    const int a = __builtin_nontemporal_load(rl + (valid ? i : 0));
    const int z = __builtin_nontemporal_load(rl + (i + 1 < ns ? i + 1 : 0));
#else
    const int a = rl[valid ? i : 0];
    const int z = rl[i + 1 < ns ? i + 1 : 0];
#endif
    st[k] = valid ? a : 0;
    en[k] = valid ? (i + 1 < ns ? z : n) : 0;
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
  for (int c0 = 0; c0 < n; c0 += kPPChunk) {
    double xv[EPT], pc[EPT];
#pragma unroll
    for (int e = 0; e < EPT; ++e) {
      xv[e] = static_cast<double>(gx(c[e]));  // 0 past the segment (c = -1)
      pc[e] = p[e];
    }
    fetch(c0 + kPPChunk < n ? c0 + kPPChunk : c0);
#pragma unroll
    for (int e = 0; e < EPT; ++e) {
      lp[threadIdx.x + e * kBlock] = pc[e];
      lx[threadIdx.x + e * kBlock] = xv[e];
    }
    __syncthreads();
    const int c1 = c0 + kPPChunk;
#pragma unroll
    for (int k = 0; k < 4; ++k) {
      const int lo = st[k] > c0 ? st[k] : c0;
      const int hi = en[k] < c1 ? en[k] : c1;
      double sk = sum[k];
      for (int j = lo; j < hi; ++j) sk = fma(lp[j - c0], lx[j - c0], sk);
      sum[k] = sk;
    }
    __syncthreads();
  }
}

template <typename XT>
__global__ __launch_bounds__(kBlock) void k_pp_product(int64_t S, int nblk, int ntiles, int pass,
                                                       const uint16_t* __restrict__ rel, const int2* __restrict__ seg,
                                                       const int* __restrict__ pcol, const double* __restrict__ pval,
                                                       const XT* __restrict__ x, double* __restrict__ part,
                                                       const Ctl* __restrict__ ctl) {
  if (ctl && ctl->done) return;
  __shared__ double lp[kPPChunk], lx[kPPChunk];
  // sliced copy: slice pass * 8 + w % 8 of tile w / 8; whole rows: tile w
  const bool sliced = nblk >= kNumXcd;
  const int b = sliced ? pass * kNumXcd + static_cast<int>(blockIdx.x % kNumXcd) : 0;
  const int t = static_cast<int>(sliced ? blockIdx.x / kNumXcd : blockIdx.x);
  if (b >= nblk || t >= ntiles) return;  // the same for the whole workgroup
  const int64_t s0 = static_cast<int64_t>(t) * kPPTile;
  const int ns = static_cast<int>(min<int64_t>(kPPTile, S - s0));
  double sum[4];
  pp_tile_sums<XT>(S, ntiles, b, t, s0, ns, rel, seg, pcol, pval, x, lp, lx, sum);
#pragma unroll
  for (int k = 0; k < 4; ++k) {
    const int i = threadIdx.x + k * kBlock;
#if MDP_NT_PARTS
    if (i < ns) __builtin_nontemporal_store(sum[k], part + static_cast<int64_t>(b) * S + s0 + i);
#else
    if (i < ns) part[static_cast<int64_t>(b) * S + s0 + i] = sum[k];
#endif
  }
}

// The unsliced copy (one slice): the product and its finish in one launch,
// no parts.  y = b + g P_pi x (a Horner step, or the Krylov product with
// b = x, g = -gamma), tile w; the same arithmetic as the two-kernel path.
template <typename XT>
__global__ __launch_bounds__(kBlock) void k_pp_axpy1(int64_t S, int ntiles, const uint16_t* __restrict__ rel,
                                                     const int2* __restrict__ seg, const int* __restrict__ pcol,
                                                     const double* __restrict__ pval, const XT* __restrict__ x,
                                                     const XT* __restrict__ bv, double g, XT* __restrict__ y,
                                                     const Ctl* __restrict__ ctl) {
  if (ctl && ctl->done) return;
  __shared__ double lp[kPPChunk], lx[kPPChunk];
  using AT = typename Acc<XT>::type;
  const int t = static_cast<int>(blockIdx.x);
  const int64_t s0 = static_cast<int64_t>(t) * kPPTile;
  const int ns = static_cast<int>(min<int64_t>(kPPTile, S - s0));
  double sum[4];
  pp_tile_sums<XT>(S, ntiles, 0, t, s0, ns, rel, seg, pcol, pval, x, lp, lx, sum);
  const AT gam = static_cast<AT>(g);
#pragma unroll
  for (int k = 0; k < 4; ++k) {
    const int i = threadIdx.x + k * kBlock;
    if (i < ns) y[s0 + i] = static_cast<XT>(fma(gam, static_cast<AT>(sum[k]), static_cast<AT>(bv[s0 + i])));
  }
}

// The unsliced copy: the Arnoldi product of step j and the Gram-Schmidt dot
// partials of its tile (tiles of kPPTile states, partials[i * ntiles + t]) in
// one launch; w as k_pp_arnoldi_finish forms it.
template <typename BT>
__global__ __launch_bounds__(kBlock) void k_pp_arnoldi1(int64_t S, int ntiles, const uint16_t* __restrict__ rel,
                                                        const int2* __restrict__ seg, const int* __restrict__ pcol,
                                                        const double* __restrict__ pval, BT* __restrict__ Ub,
                                                        int64_t ldu, int j, double gamma, const Ctl* __restrict__ ctl,
                                                        double* __restrict__ partials, const BT* __restrict__ xin) {
  if (ctl->done) return;
  static_assert(kPPChunk >= kPPTile, "the chunk staging doubles as the tile's w");
  __shared__ double lp[kPPChunk], lx[kPPChunk];
  using AT = typename Acc<BT>::type;
  const int t = static_cast<int>(blockIdx.x);
  const int64_t s0 = static_cast<int64_t>(t) * kPPTile;
  const int ns = static_cast<int>(min<int64_t>(kPPTile, S - s0));
  const BT* __restrict__ xj = xin ? xin : Ub + static_cast<int64_t>(j) * ldu;
  double sum[4];
  pp_tile_sums<BT>(S, ntiles, 0, t, s0, ns, rel, seg, pcol, pval, xj, lp, lx, sum);
  const AT gam = static_cast<AT>(gamma);
  BT* __restrict__ w = Ub + static_cast<int64_t>(j + 1) * ldu;
  const double cj = ctl->scale[j];
#pragma unroll
  for (int k = 0; k < 4; ++k) {
    const int i = threadIdx.x + k * kBlock;
    if (i < ns) {
      const int64_t s = s0 + i;
      const AT av = static_cast<AT>(xj[s]) - gam * static_cast<AT>(sum[k]);
      const BT wv = static_cast<BT>(cj * static_cast<double>(av));
      w[s] = wv;
      lp[i] = static_cast<double>(wv);  // the staging is free after the last chunk's barrier
    }
  }
  __syncthreads();
  cgs_dots_tile<BT, kPPTile>(Ub, ldu, j, s0, ns, lp, partials, t, ntiles);
}

// The rest of the Arnoldi step on the parts: (P_pi x)[s] is the sum of the
// slice parts in slice order, w = scale_j (x - gamma P_pi x) goes to U_{j+1},
// and the workgroup's dot partials with U_0..U_j go to partials, in the
// plain product's tiles and layout.
template <typename BT>
__global__ __launch_bounds__(kBlock) void k_pp_arnoldi_finish(int64_t S, int nblk, const double* __restrict__ part,
                                                              BT* __restrict__ Ub, int64_t ldu, int j, double gamma,
                                                              const Ctl* __restrict__ ctl,
                                                              double* __restrict__ partials,
                                                              const BT* __restrict__ xin) {
  if (ctl->done) return;
  using AT = typename Acc<BT>::type;
  __shared__ double w_lds[kApplyTile];
  const int tile = xcd_tile(blockIdx.x, gridDim.x);
  const int64_t s0 = static_cast<int64_t>(tile) * kApplyTile;
  const int ns = static_cast<int>(min<int64_t>(kApplyTile, S - s0));
  const AT gam = static_cast<AT>(gamma);
  const BT* __restrict__ xj = xin ? xin : Ub + static_cast<int64_t>(j) * ldu;
  BT* __restrict__ w = Ub + static_cast<int64_t>(j + 1) * ldu;
  const double cj = ctl->scale[j];
  for (int i = threadIdx.x; i < ns; i += kBlock) {
    const int64_t s = s0 + i;
    double pv = ld_part(part, S, 0, s);
    for (int b = 1; b < nblk; ++b) pv += ld_part(part, S, b, s);
    const AT av = static_cast<AT>(xj[s]) - gam * static_cast<AT>(pv);
    const BT wv = static_cast<BT>(cj * static_cast<double>(av));
    w[s] = wv;
    w_lds[i] = static_cast<double>(wv);
  }
  __syncthreads();
  cgs_dots_tile<BT>(Ub, ldu, j, s0, ns, w_lds, partials, tile, static_cast<int>(gridDim.x));
}

// One Horner step of the polynomial preconditioner on the parts:
// y = b + gamma P_pi x, as horner_tile forms it.  Exits at once when ctl is
// given and the GMRES cycle is done.
template <typename XT>
__global__ __launch_bounds__(kBlock) void k_pp_horner_finish(int64_t S, int nblk, const double* __restrict__ part,
                                                             const XT* __restrict__ b, double gamma,
                                                             XT* __restrict__ y, const Ctl* __restrict__ ctl) {
  if (ctl && ctl->done) return;
  using AT = typename Acc<XT>::type;
  const AT gam = static_cast<AT>(gamma);
  for (int64_t s = static_cast<int64_t>(blockIdx.x) * kBlock + threadIdx.x; s < S;
       s += static_cast<int64_t>(gridDim.x) * kBlock) {
    double pv = ld_part(part, S, 0, s);
    for (int k = 1; k < nblk; ++k) pv += ld_part(part, S, k, s);
    y[s] = static_cast<XT>(fma(gam, static_cast<AT>(pv), static_cast<AT>(b[s])));
  }
}

// The float64 residual r = g_pi - (x - gamma P_pi x) on the parts (a GMRES
// restart), with each tile's (max |r|, sum r^2) partial, in the tiles and
// layout of the row_ptr kernel.
template <typename YT>
__global__ __launch_bounds__(kBlock) void k_pp_residual_finish(int64_t S, int A, int nblk,
                                                               const double* __restrict__ part,
                                                               const double* __restrict__ cost,
                                                               const int* __restrict__ pi,
                                                               const double* __restrict__ x, double gamma,
                                                               YT* __restrict__ y, double4* __restrict__ partials) {
  const int tile = xcd_tile(blockIdx.x, gridDim.x);
  const int64_t s0 = static_cast<int64_t>(tile) * kApplyTile;
  const int ns = static_cast<int>(min<int64_t>(kApplyTile, S - s0));
  double dmax = 0.0, dsum = 0.0;
  for (int i = threadIdx.x; i < ns; i += kBlock) {
    const int64_t s = s0 + i;
    double pv = ld_part(part, S, 0, s);
    for (int k = 1; k < nblk; ++k) pv += ld_part(part, S, k, s);
    const double gc = cost[row_of(s, pi[s], A, S)];
    const double r = gc - (x[s] - gamma * pv);
    y[s] = static_cast<YT>(r);
    dmax = max_nan(dmax, fabs(r));
    dsum = fma(r, r, dsum);
  }
  block_max_sum(dmax, dsum);
  if (threadIdx.x == 0) partials[tile] = make_double4(dmax, dsum, 0.0, 0.0);
}

}  // namespace

// Set up (first call) and form the copy for policy pi; h->pp_ready says
// whether the partitioned products can run for it.
void pp_release(mdp_handle* h) {
  auto drop = [&](auto*& p) {
    handle_free(h, p);
    p = nullptr;
  };
  drop(h->pp_col);
  drop(h->pp_val);
  drop(h->pp_rel);
  drop(h->pp_seg);
  drop(h->pp_part);
  drop(h->pp_fill);
  drop(h->pp_snap);
}

hipError_t pp_prepare(mdp_handle* h, const int32_t* pi) {
  h->pp_ready = false;
  if (h->pp_state < 0) return hipSuccess;
  if (h->pp_state > 0 && h->pp_pi == pi && h->pp_gen == h->pi_gen) {
    h->pp_ready = true;
    return hipSuccess;
  }
  const int64_t S = h->S;
  if (h->pp_state == 0) {
    // slices only where the columns spread over a large vector (the handle
    // then carries the column-blocked copy); otherwise whole rows, the copy
    // being P_pi stored contiguously
    const int64_t passes = (S * static_cast<int64_t>(sizeof(double)) + kNumXcd * kPPSliceBytes - 1) /
                           (kNumXcd * kPPSliceBytes);
    const int64_t nblk = h->cb_blocks > 0 ? kNumXcd * passes : 1;
    const int64_t ntiles = (S + kPPTile - 1) / kPPTile;
    if (nblk > kPPMaxBlocks || nblk * ntiles > (int64_t{1} << 30)) {
      h->pp_state = -1;
      return hipSuccess;
    }
    // the longest row bounds every per-state count (8 bits) and every tile
    // segment (16 bits), and the copy's size
    hipError_t e = handle_alloc(h, reinterpret_cast<void**>(&h->pp_fill), 4 * sizeof(int));
    if (e == hipErrorOutOfMemory) {
      (void)hipGetLastError();
      h->pp_state = -1;
      return hipSuccess;
    }
    if (e != hipSuccess) return e;
    int64_t kmax = h->kfix;
    if (kmax == 0) {
      unsigned longest = 0;
      e = hipMemsetAsync(h->pp_fill, 0, sizeof(unsigned), h->stream);
      if (e == hipSuccess) {
        const int64_t g = std::min<int64_t>(4096, (h->rows + kBlock - 1) / kBlock);
        k_longest_row<<<static_cast<unsigned>(g), kBlock, 0, h->stream>>>(h->row_ptr, h->rows,
                                                                         reinterpret_cast<unsigned*>(h->pp_fill));
        e = hipGetLastError();
      }
      if (e == hipSuccess) e = copy_out(&longest, h->pp_fill, sizeof(unsigned), h->stream);
      if (e == hipSuccess) e = hipStreamSynchronize(h->stream);
      if (e != hipSuccess) return e;
      kmax = longest;
    }
    if (kmax > 255 || kmax * kPPTile > 65535) {
      pp_release(h);
      h->pp_state = -1;
      return hipSuccess;
    }
    h->pp_blocks = static_cast<int>(nblk);
    h->pp_slice = static_cast<int>((S + nblk - 1) / nblk);
    h->pp_ntiles = static_cast<int>(ntiles);
    h->pp_cap = std::min<int64_t>(h->nnz, S * kmax);
    e = handle_alloc(h, reinterpret_cast<void**>(&h->pp_rel), nblk * S * sizeof(uint16_t));
    if (e == hipSuccess) e = handle_alloc(h, reinterpret_cast<void**>(&h->pp_seg), nblk * ntiles * sizeof(int2));
    if (e == hipSuccess) e = handle_alloc(h, reinterpret_cast<void**>(&h->pp_part), nblk * S * sizeof(double));
    if (e == hipSuccess) e = handle_alloc(h, reinterpret_cast<void**>(&h->pp_col), h->pp_cap * sizeof(int));
    if (e == hipSuccess) e = handle_alloc(h, reinterpret_cast<void**>(&h->pp_val), h->pp_cap * sizeof(double));
    if (e == hipErrorOutOfMemory) {
      // no room for the copy: the products keep gathering through row_ptr
      (void)hipGetLastError();
      pp_release(h);
      h->pp_state = -1;
      return hipSuccess;
    }
    if (e != hipSuccess) return e;
    h->device_bytes += static_cast<int64_t>(nblk * S * (sizeof(uint16_t) + sizeof(double)) +
                                            nblk * ntiles * sizeof(int2) + h->pp_cap * 12);
    h->pp_state = 1;
  }
  // no host round trip: the segments are placed by atomic adds, and a policy
  // the copy already holds is found on the device (pp_fill[0]: entries placed,
  // pp_fill[1]: the policy differs from the last formation's)
  const RowIndex rix{h->row_ptr, h->kfix};
  hipError_t e = hipMemsetAsync(h->pp_fill, 0, 2 * sizeof(int), h->stream);
  if (e != hipSuccess) return e;
  int* changed = h->pp_fill + 1;
  {
    const bool first = h->pp_snap == nullptr;
    if (first) {
      e = handle_alloc(h, reinterpret_cast<void**>(&h->pp_snap), S * sizeof(int));
      if (e == hipErrorOutOfMemory) {
        // no snapshot: form the copy for every policy
        (void)hipGetLastError();
        h->pp_snap = nullptr;
        e = hipMemsetAsync(changed, 0xff, sizeof(int), h->stream);
        if (e != hipSuccess) return e;
      } else if (e != hipSuccess) {
        return e;
      } else {
        h->device_bytes += S * static_cast<int64_t>(sizeof(int));
      }
    }
    if (h->pp_snap) {
      const int64_t g = std::min<int64_t>(4096, (S + kBlock - 1) / kBlock);
      k_pp_policy_changed<<<static_cast<unsigned>(g), kBlock, 0, h->stream>>>(S, pi, h->pp_snap, first ? 1 : 0,
                                                                               changed);
      if ((e = hipGetLastError()) != hipSuccess) return e;
    }
  }
  // rows through row_ptr: bounds staged in LDS; uniform rows: computed per batch
  if (h->kfix > 0) {
    k_pp_place<false><<<h->pp_ntiles, kBlock, 0, h->stream>>>(S, h->A, rix, h->col, pi, h->pp_slice, h->pp_blocks,
                                                              h->pp_ntiles, h->pp_rel, h->pp_seg, h->pp_fill,
                                                              changed);
    k_pp_scatter<false><<<h->pp_ntiles, kBlock, 0, h->stream>>>(S, h->A, rix, h->col, h->val, pi, h->pp_slice,
                                                                h->pp_blocks, h->pp_ntiles, h->pp_seg, h->pp_rel,
                                                                h->pp_col, h->pp_val, changed);
  } else {
    k_pp_place<true><<<h->pp_ntiles, kBlock, 0, h->stream>>>(S, h->A, rix, h->col, pi, h->pp_slice, h->pp_blocks,
                                                             h->pp_ntiles, h->pp_rel, h->pp_seg, h->pp_fill,
                                                             changed);
    k_pp_scatter<true><<<h->pp_ntiles, kBlock, 0, h->stream>>>(S, h->A, rix, h->col, h->val, pi, h->pp_slice,
                                                               h->pp_blocks, h->pp_ntiles, h->pp_seg, h->pp_rel,
                                                               h->pp_col, h->pp_val, changed);
  }
  if ((e = hipGetLastError()) != hipSuccess) return e;
  h->pp_pi = pi;
  h->pp_gen = h->pi_gen;
  h->pp_ready = true;
  return hipSuccess;
}

namespace {
template <typename XT>
hipError_t pp_parts(mdp_handle* h, const XT* x, const Ctl* ctl) {
  const bool sliced = h->pp_blocks >= kNumXcd;
  const int passes = sliced ? h->pp_blocks / kNumXcd : 1;
  const int64_t grid = (sliced ? static_cast<int64_t>(kNumXcd) : int64_t{1}) * h->pp_ntiles;
  for (int p = 0; p < passes; ++p) {
    k_pp_product<XT><<<static_cast<unsigned>(grid), kBlock, 0, h->stream>>>(
        h->S, h->pp_blocks, h->pp_ntiles, p, h->pp_rel, h->pp_seg, h->pp_col, h->pp_val, x, h->pp_part, ctl);
  }
  return hipGetLastError();
}

// y = b + g P_pi x on the copy
template <typename XT>
hipError_t pp_axpy(mdp_handle* h, const XT* x, const XT* b, double g, XT* y, const Ctl* ctl) {
  if (h->pp_blocks == 1) {
    k_pp_axpy1<XT><<<static_cast<unsigned>(h->pp_ntiles), kBlock, 0, h->stream>>>(
        h->S, h->pp_ntiles, h->pp_rel, h->pp_seg, h->pp_col, h->pp_val, x, b, g, y, ctl);
    return hipGetLastError();
  }
  hipError_t e = pp_parts<XT>(h, x, ctl);
  if (e != hipSuccess) return e;
  const int64_t gr = std::min<int64_t>(8192, (h->S + kBlock - 1) / kBlock);
  k_pp_horner_finish<XT><<<static_cast<unsigned>(gr), kBlock, 0, h->stream>>>(h->S, h->pp_blocks, h->pp_part, b,
                                                                             g, y, ctl);
  return hipGetLastError();
}

template <typename BT>
hipError_t pp_arnoldi_apply(mdp_handle* h, BT* Ub, int j, const BT* xin, double* partials, int nb, int* nb_dots) {
  if (h->pp_blocks == 1) {
    *nb_dots = static_cast<int>(h->pp_ntiles);
    k_pp_arnoldi1<BT><<<static_cast<unsigned>(h->pp_ntiles), kBlock, 0, h->stream>>>(
        h->S, h->pp_ntiles, h->pp_rel, h->pp_seg, h->pp_col, h->pp_val, Ub, h->ldu, j, h->gamma, h->ctl, partials,
        xin);
    return hipGetLastError();
  }
  *nb_dots = nb;
  const BT* x = xin ? xin : Ub + static_cast<int64_t>(j) * h->ldu;
  hipError_t e = pp_parts<BT>(h, x, h->ctl);
  if (e != hipSuccess) return e;
  k_pp_arnoldi_finish<BT><<<nb, kBlock, 0, h->stream>>>(h->S, h->pp_blocks, h->pp_part, Ub, h->ldu, j, h->gamma,
                                                        h->ctl, partials, xin);
  return hipGetLastError();
}
}  // namespace

hipError_t launch_pp_op(mdp_handle* h, const double* x, double* y) {
  return pp_axpy<double>(h, x, x, -h->gamma, y, h->ctl);  // y = x + (-gamma) P_pi x
}

hipError_t launch_pp_residual(mdp_handle* h, const double* x, void* y, bool y_f32, double4* partials, int nb) {
  hipError_t e = pp_parts<double>(h, x, nullptr);
  if (e != hipSuccess) return e;
  if (y_f32)
    k_pp_residual_finish<float><<<nb, kBlock, 0, h->stream>>>(h->S, h->A, h->pp_blocks, h->pp_part, h->cost,
                                                              h->pp_pi, x, h->gamma, static_cast<float*>(y),
                                                              partials);
  else
    k_pp_residual_finish<double><<<nb, kBlock, 0, h->stream>>>(h->S, h->A, h->pp_blocks, h->pp_part, h->cost,
                                                               h->pp_pi, x, h->gamma, static_cast<double*>(y),
                                                               partials);
  return hipGetLastError();
}

hipError_t launch_pp_horner(mdp_handle* h, bool f32, const void* x, const void* b, void* y, const Ctl* ctl) {
  if (f32)
    return pp_axpy<float>(h, static_cast<const float*>(x), static_cast<const float*>(b), h->gamma,
                          static_cast<float*>(y), ctl);
  return pp_axpy<double>(h, static_cast<const double*>(x), static_cast<const double*>(b), h->gamma,
                         static_cast<double*>(y), ctl);
}

hipError_t launch_pp_arnoldi_apply(mdp_handle* h, bool basis_f32, int j, const void* xin, double* partials,
                                   int nb, int* nb_dots) {
  if (basis_f32)
    return pp_arnoldi_apply<float>(h, h->U32, j, static_cast<const float*>(xin), partials, nb, nb_dots);
  return pp_arnoldi_apply<double>(h, h->U64, j, static_cast<const double*>(xin), partials, nb, nb_dots);
}

}  // namespace mdp
