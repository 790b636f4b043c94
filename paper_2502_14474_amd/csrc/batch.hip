// Batched inexact policy iteration: many resident MDPs advanced together by
// persistent kernels that walk a work table of (MDP, tile) pairs.
//
// Every batched kernel calls the same tile bodies (device.h) as the
// single-MDP kernels, with the same tiling and the same fixed-order
// reductions into each MDP's own partials and control block, and the host
// takes the same decisions per MDP.  An MDP therefore gets bitwise the same
// iterates, policy and iteration counts alone and inside any batch.
//
// One round advances every unfinished MDP by one phase of the method:
//   1. MDPs that need a greedy step get a Bellman sweep (this also starts
//      their GMRES cycle from r0 = T v - v);
//   2. every MDP in policy evaluation runs one GMRES(m) cycle; the cycle's
//      Arnoldi steps are replayed from captured HIP graphs (one graph per
//      chunk of steps), each MDP leaving early once its cycle is done;
//   3. the cycle ends with x += V y and, where the inner tolerance is not
//      met, a float64 residual restart.
// New MDPs may join between rounds (continuous batching in the server).
#include <algorithm>
#include <chrono>
#include <cmath>
#include <cstring>
#include <limits>
#include <map>
#include <mutex>
#include <shared_mutex>
#include <vector>

#include "batch.h"
#include "device.h"

namespace mdp {

// ----------------------------------------------------------------------------
// device side
// ----------------------------------------------------------------------------

// Find the list position k with tstart[k] <= t < tstart[k+1] (uniform per
// workgroup, so the search runs on scalar registers).
__device__ __forceinline__ int find_item(const int* __restrict__ tstart, int n, int t) {
  int lo = 0, hi = n - 1;
  while (lo < hi) {
    const int mid = (lo + hi + 1) >> 1;
    if (tstart[mid] <= t) lo = mid;
    else hi = mid - 1;
  }
  return lo;
}

// Persistent loop: workgroup b takes the contiguous tile range
// [T*b/G, T*(b+1)/G) of the list and calls f(list position, local tile).
// Every listed MDP owns at least one tile, so tstart is strictly increasing.
template <typename F>
__device__ __forceinline__ void for_tiles(const WorkList* __restrict__ wl, F f) {
  const int n = wl->n;
  const int* tstart = wl->ts();
  const int T = tstart[n];
  const int t0 = static_cast<int>(static_cast<int64_t>(T) * blockIdx.x / gridDim.x);
  const int t1 = static_cast<int>(static_cast<int64_t>(T) * (blockIdx.x + 1) / gridDim.x);
  if (t0 >= t1) return;
  int k = find_item(tstart, n, t0);
  for (int t = t0; t < t1; ++t) {
    while (tstart[k + 1] <= t) ++k;
    f(k, t - tstart[k]);
  }
}

template <int L, int U, int PREC, bool GM>
__global__ __launch_bounds__(kBlock) void kb_bellman(const BDesc* __restrict__ d,
                                                     const WorkList* __restrict__ wl) {
  extern __shared__ double lds_d[];
  for_tiles(wl, [&](int k, int tl) {
    const BDesc& D = d[wl->it(k)];
    const int ts = D.A >= kSweepRows ? 1 : kSweepRows / D.A;
    auto* part = reinterpret_cast<double4*>(D.part);
    if (PREC == kF64) {
      if (GM && D.basis_f32)
        bellman_tile<L, U, double, double, false, float>(D.S, D.A, ts, RowIndex{D.row_ptr, D.kfix}, D.col, D.val,
                                                         nullptr, D.cost, D.v, D.gamma, nullptr,
                                                         D.pi, D.U32, part, tl, lds_d);
      else
        bellman_tile<L, U, double, double, false, double>(D.S, D.A, ts, RowIndex{D.row_ptr, D.kfix}, D.col, D.val,
                                                          nullptr, D.cost, D.v, D.gamma, nullptr,
                                                          D.pi, GM ? D.U64 : nullptr, part, tl,
                                                          lds_d);
    } else if (PREC == kF32) {
      bellman_tile<L, U, float, float, false, float>(D.S, D.A, ts, RowIndex{D.row_ptr, D.kfix},
                                                     reinterpret_cast<const int*>(D.cv32), D.cv32,
                                                     nullptr, D.cost, D.v32, D.gamma, nullptr,
                                                     D.pi, D.U32, part, tl, lds_d);
    } else {
      bellman_tile<L, U, __half, float, true, float>(D.S, D.A, ts, RowIndex{D.row_ptr, D.kfix}, D.col, D.val16,
                                                     D.corr16, D.cost, D.v32, D.gamma, nullptr,
                                                     D.pi, D.U32, part, tl, lds_d);
    }
    __syncthreads();
  });
}

// One workgroup per listed MDP: reduce its (max, sum, max) partials into its
// control block; kRedGmresStart starts a GMRES cycle.  `kind` selects which
// kernel produced the partials (0: sweep, 1: policy product).
__global__ __launch_bounds__(kBlock) void kb_reduce_ms(const BDesc* __restrict__ d,
                                                       const WorkList* __restrict__ wl, int kind,
                                                       int mode, int first_cycle) {
  for (int k = blockIdx.x; k < wl->n; k += gridDim.x) {
    const BDesc& D = d[wl->it(k)];
    reduce_ms_body(reinterpret_cast<const double4*>(D.part), kind == 0 ? D.nb_sweep : D.nb_apply,
                   mode, first_cycle, D.alpha, D.floor_rel, D.ctl);
    __syncthreads();
  }
}

// Float64 residual g_pi - (I - gamma P_pi) x of the inner iterate x = v,
// written into basis slot 0.
template <int L, int U>
__global__ __launch_bounds__(kBlock) void kb_residual(const BDesc* __restrict__ d,
                                                      const WorkList* __restrict__ wl) {
  for_tiles(wl, [&](int k, int tl) {
    const BDesc& D = d[wl->it(k)];
    auto* part = reinterpret_cast<double4*>(D.part);
    if (D.basis_f32)
      apply_tile<L, U, kApplyRes, double, double, float, false>(
          D.S, D.A, RowIndex{D.row_ptr, D.kfix}, D.col, D.val, nullptr, D.cost, D.pi, D.v, D.gamma, D.U32, part, tl);
    else
      apply_tile<L, U, kApplyRes, double, double, double, false>(
          D.S, D.A, RowIndex{D.row_ptr, D.kfix}, D.col, D.val, nullptr, D.cost, D.pi, D.v, D.gamma, D.U64, part, tl);
    __syncthreads();
  });
}

template <int L, int U, int PREC>
__global__ __launch_bounds__(kBlock) void kb_arnoldi_apply(const BDesc* __restrict__ d,
                                                           const WorkList* __restrict__ wl,
                                                           int j) {
  for_tiles(wl, [&](int k, int tl) {
    const BDesc& D = d[wl->it(k)];
    if (D.ctl->done) return;
    if (PREC == kF64)
      arnoldi_apply_tile<L, U, double, double, false>(D.S, D.A, RowIndex{D.row_ptr, D.kfix}, D.col, D.val, nullptr,
                                                      D.pi, D.U64, D.ldu, j, D.gamma, D.ctl,
                                                      D.part, tl, D.nb_apply);
    else if (PREC == kF32)
      arnoldi_apply_tile<L, U, float, float, false>(D.S, D.A, RowIndex{D.row_ptr, D.kfix},
                                                    reinterpret_cast<const int*>(D.cv32), D.cv32, nullptr,
                                                    D.pi, D.U32, D.ldu, j, D.gamma, D.ctl, D.part,
                                                    tl, D.nb_apply);
    else
      arnoldi_apply_tile<L, U, __half, float, true>(D.S, D.A, RowIndex{D.row_ptr, D.kfix}, D.col, D.val16,
                                                    D.corr16, D.pi, D.U32, D.ldu, j, D.gamma,
                                                    D.ctl, D.part, tl, D.nb_apply);
    __syncthreads();
  });
}

__global__ __launch_bounds__(kBlock) void kb_reduce_dots(const BDesc* __restrict__ d,
                                                         const WorkList* __restrict__ wl, int j) {
  const int work = wl->n * (j + 1);
  for (int w = blockIdx.x; w < work; w += gridDim.x) {
    const int k = w / (j + 1), i = w - k * (j + 1);
    const BDesc& D = d[wl->it(k)];
    if (D.ctl->done) continue;
    reduce_dots_body(D.part, D.nb_apply, j, D.ctl, i);
    __syncthreads();
  }
}

template <typename BT>
__global__ __launch_bounds__(kBlock) void kb_arnoldi_update(const BDesc* __restrict__ d,
                                                            const WorkList* __restrict__ wl,
                                                            int j) {
  for_tiles(wl, [&](int k, int tl) {
    const BDesc& D = d[wl->it(k)];
    if (D.ctl->done) return;
    BT* U = nullptr;
    if constexpr (sizeof(BT) == 8) U = D.U64;
    else U = D.U32;
    arnoldi_update_body<BT>(D.S, U, D.ldu, j, D.ctl, D.part, tl);
    __syncthreads();
  });
}

__global__ __launch_bounds__(kBlock) void kb_norm_givens(const BDesc* __restrict__ d,
                                                         const WorkList* __restrict__ wl, int j,
                                                         int m) {
  for (int k = blockIdx.x; k < wl->n; k += gridDim.x) {
    const BDesc& D = d[wl->it(k)];
    if (D.ctl->done) continue;
    norm_givens_body(D.part, D.nb_upd, j, m, D.ctl);
    __syncthreads();
  }
}

template <typename BT>
__global__ __launch_bounds__(kBlock) void kb_update_x(const BDesc* __restrict__ d,
                                                      const WorkList* __restrict__ wl) {
  for_tiles(wl, [&](int k, int tl) {
    const BDesc& D = d[wl->it(k)];
    const BT* U = nullptr;
    if constexpr (sizeof(BT) == 8) U = D.U64;
    else U = D.U32;
    gmres_update_x_body<BT, double>(D.S, D.v, U, D.ldu, D.ctl, tl);
    __syncthreads();
  });
}

// v -> float32 copy for low-precision sweeps (elementwise, per update tile).
__global__ __launch_bounds__(kBlock) void kb_cast(const BDesc* __restrict__ d,
                                                  const WorkList* __restrict__ wl) {
  for_tiles(wl, [&](int k, int tl) {
    const BDesc& D = d[wl->it(k)];
    const int64_t s0 = static_cast<int64_t>(tl) * kUpdTile;
    for (int i = threadIdx.x; i < kUpdTile; i += kBlock) {
      const int64_t s = s0 + i;
      if (s < D.S) D.v32[s] = static_cast<float>(D.v[s]);
    }
  });
}

// Copy the control-block header of every listed MDP into one array.
__global__ void kb_headers(const BDesc* __restrict__ d, const WorkList* __restrict__ wl,
                           Ctl* __restrict__ out) {
  constexpr int W = static_cast<int>(kCtlHeaderBytes / sizeof(uint32_t));
  const int total = wl->n * W;
  for (int i = blockIdx.x * blockDim.x + threadIdx.x; i < total; i += gridDim.x * blockDim.x) {
    const int k = i / W, w = i - k * W;
    const uint32_t* src = reinterpret_cast<const uint32_t*>(d[wl->it(k)].ctl);
    reinterpret_cast<uint32_t*>(out + k)[w] = src[w];
  }
}

// ----------------------------------------------------------------------------
// host side
// ----------------------------------------------------------------------------
namespace {

template <int L> constexpr int rows_in_flight_b() { return L >= 32 ? 2 : MDP_UNROLL; }

template <typename F>
hipError_t with_lanes_b(int L, F&& f) {
  switch (L) {
    case 2: return f(std::integral_constant<int, 2>{});
    case 4: return f(std::integral_constant<int, 4>{});
    case 8: return f(std::integral_constant<int, 8>{});
    case 16: return f(std::integral_constant<int, 16>{});
    case 32: return f(std::integral_constant<int, 32>{});
    case 64: return f(std::integral_constant<int, 64>{});
    default: return hipErrorInvalidValue;
  }
}

int nb_of(int64_t n, int per) { return static_cast<int>((n + per - 1) / per); }

}  // namespace

BatchEngine::~BatchEngine() { release(); }

void BatchEngine::release() {
  for (auto& g : graphs) {
    for (auto& e : g.second.exec) (void)hipGraphExecDestroy(e);
  }
  graphs.clear();
  lib_free(descs_d);
  lib_free(lists_d);
  lib_free(hdr_d);
  lib_host_free(hdr_h);
  lib_host_free(lists_h);
  lib_host_free(descs_h);
  descs_h = nullptr;
  descs_d = nullptr;
  lists_d = nullptr;
  hdr_d = nullptr;
  hdr_h = nullptr;
  lists_h = nullptr;
  cap = 0;
}

mdp_status BatchEngine::reserve(int n) {
  if (n <= cap) return MDP_OK;
  release();
  const int want = std::max(n, 16);
  const size_t list_bytes = WorkList::bytes(want);
  hipError_t e = lib_malloc(reinterpret_cast<void**>(&descs_d), sizeof(BDesc) * want);
  if (e == hipSuccess) e = lib_malloc(reinterpret_cast<void**>(&lists_d), list_bytes * kNumLists);
  if (e == hipSuccess) e = lib_malloc(reinterpret_cast<void**>(&hdr_d), sizeof(Ctl) * want);
  if (e == hipSuccess) e = lib_host_malloc(reinterpret_cast<void**>(&hdr_h), sizeof(Ctl) * want);
  if (e == hipSuccess) e = lib_host_malloc(reinterpret_cast<void**>(&lists_h), list_bytes * kNumLists);
  if (e == hipSuccess) e = lib_host_malloc(reinterpret_cast<void**>(&descs_h), sizeof(BDesc) * want);
  if (e != hipSuccess) {
    release();  // all or nothing: cap stays 0, so a later call allocates again
    MDP_HIP(e);
  }
  cap = want;
  std::memset(descs_h, 0, sizeof(BDesc) * cap);
  return MDP_OK;
}

WorkList* BatchEngine::list_d(int slot) const {
  return reinterpret_cast<WorkList*>(reinterpret_cast<char*>(lists_d) + WorkList::bytes(cap) * slot);
}
WorkList* BatchEngine::list_h(int slot) const {
  return reinterpret_cast<WorkList*>(reinterpret_cast<char*>(lists_h) + WorkList::bytes(cap) * slot);
}

void BatchEngine::fill_desc(int i) {
  BatchItem& it = *items[i];
  mdp_handle* h = it.h;
  BDesc& D = descs_h[i];
  D.S = h->S;
  D.A = h->A;
  D.gamma = h->gamma;
  D.row_ptr = h->row_ptr;
  D.kfix = h->kfix;
  D.col = h->col;
  D.val = h->val;
  D.cv32 = h->cv32;
  D.val16 = h->val16;
  D.corr16 = h->corr16;
  D.cost = h->cost;
  D.v = h->v;
  D.v32 = h->v32;
  D.pi = h->pi;
  D.U64 = h->U64;
  D.U32 = h->U32;
  D.ldu = h->ldu;
  D.part = h->part.buf;
  D.ctl = h->ctl;
  D.alpha = it.alpha;
  D.floor_rel = floor_of(prec);
  D.basis_f32 = prec != kF64 ? 1 : 0;
  D.nb_sweep = nb_of(h->S, sweep_tile_states(h->A));
  D.nb_apply = nb_of(h->S, kApplyTile);
  D.nb_upd = nb_of(h->S, kUpdTile);
}

// Build work list `slot` over the given items; tiles per item from `per`.
int BatchEngine::build_list(int slot, const std::vector<int>& idx, int kind) {
  WorkList* w = list_h(slot);
  w->n = static_cast<int>(idx.size());
  w->cap = cap;
  int t = 0;
  for (size_t k = 0; k < idx.size(); ++k) {
    const BDesc& D = descs_h[idx[k]];
    w->items()[k] = idx[k];
    w->tss()[k] = t;
    t += kind == 0 ? D.nb_sweep : (kind == 1 ? D.nb_apply : D.nb_upd);
  }
  w->tss()[idx.size()] = t;
  return t;
}

mdp_status BatchEngine::upload(int nitems, int nlists) {
  MDP_HIP(hipMemcpyAsync(descs_d, descs_h, sizeof(BDesc) * nitems, hipMemcpyHostToDevice,
                         stream));
  MDP_HIP(hipMemcpyAsync(lists_d, lists_h, WorkList::bytes(cap) * nlists, hipMemcpyHostToDevice,
                         stream));
  return MDP_OK;
}

mdp_status BatchEngine::headers(int slot, int n) {
  if (n == 0) return MDP_OK;
  kb_headers<<<std::min(1024, (n * 32 + 255) / 256), 256, 0, stream>>>(descs_d, list_d(slot), hdr_d);
  MDP_HIP(hipGetLastError());
  MDP_HIP(hipMemcpyAsync(hdr_h, hdr_d, sizeof(Ctl) * n, hipMemcpyDeviceToHost, stream));
  MDP_HIP(hipStreamSynchronize(stream));
  return MDP_OK;
}

static int persistent_grid(int total) { return std::max(1, std::min(total, 2048)); }

// Grids of the captured Arnoldi steps (graph replays keep their launch
// shapes, and the kernels walk their work lists grid-stride): the round's work
// rounded up to a power of two, capped at 4 workgroups per CU on the big
// kernels and fewer on the per-MDP reductions.  The grids are part of the
// graph key, so a smaller batch replays graphs with smaller grids.
constexpr int kGraphGridBig = 1024;
constexpr int kGraphGridReduce = 512;
constexpr int kGraphGridSmall = 64;

static int pow2_grid(int work, int cap) {
  int g = 1;
  while (g < work && g < cap) g <<= 1;
  return g;
}

// Arnoldi steps [j0, j1) of the current cycle for the lanes classes `cls`.
hipError_t BatchEngine::enqueue_steps(const std::vector<int>& cls_lanes, int j0, int j1, int m,
                                      const GraphKey* fixed, int tiles_apply_max, int tiles_upd,
                                      int n_items) {
  // Captured steps take the key's grids and read every count from the work
  // lists; direct launches size each grid to the work.
  auto grid = [&](int work, int fixed_size) { return fixed ? fixed_size : persistent_grid(work); };
  const int g_apply = fixed ? fixed->g_apply : 0, g_upd = fixed ? fixed->g_upd : 0;
  const int g_small = fixed ? fixed->g_small : 0;
  for (int j = j0; j < j1; ++j) {
    for (size_t c = 0; c < cls_lanes.size(); ++c) {
      const int L = cls_lanes[c];
      hipError_t e = with_lanes_b(L, [&](auto Lc) -> hipError_t {
        constexpr int LL = decltype(Lc)::value;
        constexpr int UU = rows_in_flight_b<LL>();
        const int g = grid(tiles_apply_max, g_apply);
        if (prec == kF64)
          kb_arnoldi_apply<LL, UU, kF64><<<g, kBlock, 0, stream>>>(descs_d, list_d(kListApply0 + c), j);
        else if (prec == kF32)
          kb_arnoldi_apply<LL, UU, kF32><<<g, kBlock, 0, stream>>>(descs_d, list_d(kListApply0 + c), j);
        else
          kb_arnoldi_apply<LL, UU, kF16><<<g, kBlock, 0, stream>>>(descs_d, list_d(kListApply0 + c), j);
        return hipGetLastError();
      });
      if (e != hipSuccess) return e;
    }
    kb_reduce_dots<<<grid(n_items * (j + 1), kGraphGridReduce), kBlock, 0, stream>>>(descs_d, list_d(kListGm), j);
    const int gu = grid(tiles_upd, g_upd);
    if (prec == kF64)
      kb_arnoldi_update<double><<<gu, kBlock, 0, stream>>>(descs_d, list_d(kListGmUpd), j);
    else
      kb_arnoldi_update<float><<<gu, kBlock, 0, stream>>>(descs_d, list_d(kListGmUpd), j);
    kb_norm_givens<<<grid(n_items, g_small), kBlock, 0, stream>>>(descs_d, list_d(kListGm), j, m);
    hipError_t e = hipGetLastError();
    if (e != hipSuccess) return e;
  }
  return hipSuccess;
}

mdp_status BatchEngine::sweep_phase(const mdp_solve_opts& o, std::vector<int>& need) {
  // items needing a sweep, grouped by (lanes, sweep precision)
  for (int i : need) ++items[i]->h->pi_gen;  // their policies are written
  while (!need.empty()) {
    for (int i : need) fill_desc(i);  // tile counts come from the descriptors
    std::map<std::pair<int, int>, std::vector<int>> groups;
    for (int i : need) groups[{items[i]->h->lanes, items[i]->lowp_sweep ? static_cast<int>(prec) : 0}].push_back(i);
    int slot = kListSweep0;
    std::vector<std::pair<std::pair<int, int>, int>> launch;
    for (auto& g : groups) {
      if (slot >= kListSweep0 + 3 * kMaxClasses) return fail(MDP_E_NOTSUP, "too many sweep classes in a batch");
      const int tiles = build_list(slot, g.second, 0);
      launch.push_back({g.first, tiles});
      ++slot;
    }
    const int ncast_tiles = [&]() {
      std::vector<int> c;
      for (int i : need)
        if (items[i]->lowp_sweep) c.push_back(i);
      return build_list(kListCast, c, 2);
    }();
    build_list(kListAll, need, 0);
    MDP_TRY(upload(static_cast<int>(items.size()), kNumLists));
    if (ncast_tiles > 0) {
      kb_cast<<<persistent_grid(ncast_tiles), kBlock, 0, stream>>>(descs_d, list_d(kListCast));
      MDP_HIP(hipGetLastError());
    }
    slot = kListSweep0;
    for (auto& l : launch) {
      const int L = l.first.first, sp = l.first.second, tiles = l.second;
      size_t lds = 0;
      for (int i : groups[l.first]) {
        const int A = items[i]->h->A;
        const int ts = sweep_tile_states(A);
        lds = std::max(lds, static_cast<size_t>(ts) * A * sizeof(double) +
                                (static_cast<size_t>(ts) * A + 1) * sizeof(int));
      }
      const WorkList* wl = list_d(slot);
      hipError_t e = with_lanes_b(L, [&](auto Lc) -> hipError_t {
        constexpr int LL = decltype(Lc)::value;
        constexpr int UU = rows_in_flight_b<LL>();
        const int grid = persistent_grid(tiles);
        if (sp == kF64)
          kb_bellman<LL, UU, kF64, true><<<grid, kBlock, lds, stream>>>(descs_d, wl);
        else if (sp == kF32)
          kb_bellman<LL, UU, kF32, true><<<grid, kBlock, lds, stream>>>(descs_d, wl);
        else
          kb_bellman<LL, UU, kF16, true><<<grid, kBlock, lds, stream>>>(descs_d, wl);
        return hipGetLastError();
      });
      MDP_HIP(e);
      ++slot;
    }
    kb_reduce_ms<<<persistent_grid(static_cast<int>(need.size())), kBlock, 0, stream>>>(
        descs_d, list_d(kListAll), 0, kRedGmresStart, 1);
    MDP_HIP(hipGetLastError());
    MDP_TRY(headers(kListAll, static_cast<int>(need.size())));
    std::vector<int> redo;
    for (size_t k = 0; k < need.size(); ++k) {
      BatchItem& it = *items[need[k]];
      const Ctl& c = hdr_h[k];
      const Prec sp = it.lowp_sweep ? prec : kF64;
      it.sweeps += 1;
      it.bytes += bytes_sweep(it.h, bval_of(sp), sp == kF64 ? 8 : 4, true, prec != kF64 ? 4 : 8);
      const double res = c.res_max, tv_max = c.aux_max;
      if (!std::isfinite(res)) {
        it.status = MDP_E_NUMERIC;
        it.state = BatchItem::kDone;
        continue;
      }
      if (it.lowp_sweep) {
        const double uP = sp == kF16 ? 4.9e-4 : 6.0e-8;
        if (res <= std::max(1e-5, 16.0 * uP) * tv_max || res <= 10.0 * o.atol ||
            res > 0.5 * it.prev_lowp_res) {
          it.lowp_sweep = false;
          redo.push_back(need[k]);
          continue;
        }
        it.prev_lowp_res = res;
      }
      it.history.push_back(res);
      it.res = res;
      const bool cert_ok = o.rtol_cert <= 0.0 || res <= o.rtol_cert * (1.0 - it.h->gamma) * tv_max;
      if (!it.lowp_sweep && res <= o.atol && cert_ok) {
        it.status = MDP_OK;
        it.state = BatchItem::kDone;
        continue;
      }
      if (it.k >= o.max_outer) {
        it.status = MDP_W_MAXITER;
        it.state = BatchItem::kDone;
        continue;
      }
      if (res > it.prev_res) it.alpha = std::max(it.alpha * 0.5, 1e-12);
      it.prev_res = res;
      it.state = BatchItem::kGmres;
      it.eval_steps = 0;
    }
    need.swap(redo);
  }
  return MDP_OK;
}

mdp_status BatchEngine::cycle_phase(const mdp_solve_opts& o, std::vector<int>& gm) {
  if (gm.empty()) return MDP_OK;
  const int m = o.restart;
  for (int i : gm) fill_desc(i);  // tile counts come from the descriptors
  std::map<int, std::vector<int>> cls;
  for (int i : gm) cls[items[i]->h->lanes].push_back(i);
  if (static_cast<int>(cls.size()) > kMaxClasses) return fail(MDP_E_NOTSUP, "too many lane classes in a batch");
  std::vector<int> lanes;
  int slot = kListApply0, tiles_apply_max = 0;
  for (auto& c : cls) {
    lanes.push_back(c.first);
    tiles_apply_max = std::max(tiles_apply_max, build_list(slot++, c.second, 1));
  }
  build_list(kListGm, gm, 1);
  const int tiles_upd = build_list(kListGmUpd, gm, 2);
  MDP_TRY(upload(static_cast<int>(items.size()), kNumLists));
  const int n = static_cast<int>(gm.size());
  const int se = std::max(1, o.sync_every > 0 ? o.sync_every : 6);

  // The Arnoldi steps come from HIP graphs captured once per configuration
  // (precision, lane classes, m, chunk length, grid sizes) and replayed each
  // round; the work lists they read are refreshed before every replay.
  GraphKey key{static_cast<int>(prec), lanes, m, se, pow2_grid(tiles_apply_max, kGraphGridBig),
               pow2_grid(tiles_upd, kGraphGridBig), pow2_grid(n, kGraphGridSmall)};
  auto git = graphs.find(key);
  if (use_graphs && git == graphs.end()) {
    std::unique_lock<std::shared_mutex> cap_guard(alloc_lock());
    ChunkGraphs cg;
    for (int j0 = 0; j0 < m; j0 += se) {
      hipGraph_t g;
      MDP_HIP(hipStreamBeginCapture(stream, hipStreamCaptureModeThreadLocal));
      hipError_t e = enqueue_steps(lanes, j0, std::min(m, j0 + se), m, &key, tiles_apply_max,
                                   tiles_upd, n);
      hipGraph_t gout = nullptr;
      hipError_t e2 = hipStreamEndCapture(stream, &gout);
      MDP_HIP(e);
      MDP_HIP(e2);
      g = gout;
      hipGraphExec_t ex;
      MDP_HIP(hipGraphInstantiate(&ex, g, nullptr, nullptr, 0));
      (void)hipGraphDestroy(g);
      cg.exec.push_back(ex);
    }
    git = graphs.emplace(key, std::move(cg)).first;
    if (graphs.size() > 64) {  // bound the cache: drop everything but this one
      ChunkGraphs keep = std::move(git->second);
      for (auto& g : graphs)
        for (auto& e : g.second.exec) (void)hipGraphExecDestroy(e);
      graphs.clear();
      git = graphs.emplace(key, std::move(keep)).first;
    }
  }
  int chunk = 0;
  for (int j0 = 0; j0 < m; j0 += se, ++chunk) {
    if (use_graphs) {
      MDP_HIP(hipGraphLaunch(git->second.exec[chunk], stream));
    } else {
      MDP_HIP(enqueue_steps(lanes, j0, std::min(m, j0 + se), m, nullptr, tiles_apply_max, tiles_upd,
                            n));
    }
    MDP_TRY(headers(kListGm, n));
    bool all_done = true;
    for (int k = 0; k < n; ++k) all_done = all_done && hdr_h[k].done;
    if (all_done) break;
  }
  // x += V y
  if (prec == kF64)
    kb_update_x<double><<<persistent_grid(tiles_upd), kBlock, 0, stream>>>(descs_d, list_d(kListGmUpd));
  else
    kb_update_x<float><<<persistent_grid(tiles_upd), kBlock, 0, stream>>>(descs_d, list_d(kListGmUpd));
  MDP_HIP(hipGetLastError());
  MDP_TRY(headers(kListGm, n));
  const int bb = prec == kF64 ? 8 : 4;
  std::vector<int> restart, last_j(items.size(), 0);
  for (int k = 0; k < n; ++k) {
    BatchItem& it = *items[gm[k]];
    const Ctl& c = hdr_h[k];
    const int done_j = c.j;
    last_j[gm[k]] = done_j;
    for (int jj = 0; jj < done_j; ++jj)
      it.bytes += bytes_arnoldi_apply(it.h, bval_of(prec), bb, jj) + bytes_arnoldi_update(it.h, bb, jj);
    it.applies += done_j;
    it.eval_steps = c.steps;
    if (!std::isfinite(c.res_est)) {
      it.status = MDP_E_NUMERIC;
      it.state = BatchItem::kDone;
      continue;
    }
    if ((c.converged && prec == kF64) || c.steps >= o.max_inner) {
      it.finish_eval();
      continue;
    }
    restart.push_back(gm[k]);
  }
  if (!restart.empty()) {
    std::map<int, std::vector<int>> rc;
    for (int i : restart) rc[items[i]->h->lanes].push_back(i);
    int s = kListApply0;
    std::vector<std::pair<int, int>> rl;
    for (auto& c : rc) rl.push_back({c.first, build_list(s++, c.second, 1)});
    build_list(kListGm, restart, 1);
    MDP_TRY(upload(static_cast<int>(items.size()), kNumLists));
    s = kListApply0;
    for (auto& c : rl) {
      hipError_t e = with_lanes_b(c.first, [&](auto Lc) -> hipError_t {
        constexpr int LL = decltype(Lc)::value;
        constexpr int UU = rows_in_flight_b<LL>();
        kb_residual<LL, UU><<<persistent_grid(c.second), kBlock, 0, stream>>>(descs_d, list_d(s));
        return hipGetLastError();
      });
      MDP_HIP(e);
      ++s;
    }
    kb_reduce_ms<<<persistent_grid(static_cast<int>(restart.size())), kBlock, 0, stream>>>(
        descs_d, list_d(kListGm), 1, kRedGmresStart, 0);
    MDP_HIP(hipGetLastError());
    MDP_TRY(headers(kListGm, static_cast<int>(restart.size())));
    for (size_t k = 0; k < restart.size(); ++k) {
      BatchItem& it = *items[restart[k]];
      const Ctl& c = hdr_h[k];
      it.applies += 1;
      it.refinements += prec == kF64 ? 0 : 1;
      it.bytes += bytes_apply(it.h, 8, 8, bb);
      if (!std::isfinite(c.beta)) {
        it.status = MDP_E_NUMERIC;
        it.state = BatchItem::kDone;
        continue;
      }
      if (c.converged || (last_j[restart[k]] == 0 && c.done)) it.finish_eval();
    }
  }
  return MDP_OK;
}

void BatchItem::finish_eval() {
  inner += eval_steps;
  k += 1;
  state = kSweep;
}

mdp_status BatchEngine::round(const mdp_solve_opts& o) {
  std::vector<int> need, gm;
  for (size_t i = 0; i < items.size(); ++i)
    if (items[i]->state == BatchItem::kSweep) need.push_back(static_cast<int>(i));
  last_swept = static_cast<int>(need.size());
  MDP_TRY(sweep_phase(o, need));
  last_sweep_end_ms = std::chrono::duration<double, std::milli>(
                          std::chrono::steady_clock::now().time_since_epoch()).count();
  for (size_t i = 0; i < items.size(); ++i)
    if (items[i]->state == BatchItem::kGmres) gm.push_back(static_cast<int>(i));
  MDP_TRY(cycle_phase(o, gm));
  return MDP_OK;
}

}  // namespace mdp
