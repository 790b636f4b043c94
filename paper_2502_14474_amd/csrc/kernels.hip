// HIP kernels of the single-MDP path and their launchers.  The kernel bodies
// live in device.h and are shared with the batched kernels, so one MDP gives
// bitwise the same results alone and inside a batch.
#include "device.h"

namespace mdp {

template <int L, int U, typename VT, typename XT, bool CORR, typename RT>
__global__ __launch_bounds__(kBlock) void k_bellman(
    int64_t S, int A, int tile_states, const int* __restrict__ row_ptr, int kfix,
    const int* __restrict__ col, const VT* __restrict__ val, const double* __restrict__ corr,
    const double* __restrict__ cost, const XT* __restrict__ v, double gamma,
    double* __restrict__ Tv, int* __restrict__ pi, RT* __restrict__ r0,
    double4* __restrict__ partials) {
  extern __shared__ double lds_d[];
  bellman_tile<L, U, VT, XT, CORR, RT>(S, A, tile_states, RowIndex{row_ptr, kfix}, col, val, corr, cost, v, gamma,
                                       Tv, pi, r0, partials, xcd_tile(blockIdx.x, gridDim.x),
                                       lds_d);
}

template <int L, int U, int MODE, typename VT, typename XT, typename YT, bool CORR>
__global__ __launch_bounds__(kBlock) void k_policy_apply(
    int64_t S, int A, const int* __restrict__ row_ptr, int kfix, const int* __restrict__ col,
    const VT* __restrict__ val, const double* __restrict__ corr,
    const double* __restrict__ cost, const int* __restrict__ pi, const XT* __restrict__ x,
    double gamma, YT* __restrict__ y, double4* __restrict__ partials,
    const Ctl* __restrict__ ctl, const int* __restrict__ cur /* Richardson ping-pong or null */,
    const XT* __restrict__ x_alt, YT* __restrict__ y_alt) {
  if (ctl && ctl->done) return;
  if (cur && *cur) {  // Richardson: odd steps read the second buffer
    const XT* t = x_alt;
    x_alt = x;
    x = t;
    YT* u = y_alt;
    y_alt = y;
    y = u;
  }
  apply_tile<L, U, MODE, VT, XT, YT, CORR>(S, A, RowIndex{row_ptr, kfix}, col, val, corr, cost, pi, x, gamma, y,
                                           partials, xcd_tile(blockIdx.x, gridDim.x));
}

template <int L, int U, typename VT, typename BT, bool CORR>
__global__ __launch_bounds__(kBlock) void k_arnoldi_apply(
    int64_t S, int A, const int* __restrict__ row_ptr, int kfix, const int* __restrict__ col,
    const VT* __restrict__ val, const double* __restrict__ corr, const int* __restrict__ pi,
    BT* __restrict__ Ub, int64_t ldu, int j, double gamma, const Ctl* __restrict__ ctl,
    double* __restrict__ partials, const BT* __restrict__ xin) {
  if (ctl->done) return;
  arnoldi_apply_tile<L, U, VT, BT, CORR>(S, A, RowIndex{row_ptr, kfix}, col, val, corr, pi, Ub, ldu, j, gamma,
                                         ctl, partials, xcd_tile(blockIdx.x, gridDim.x),
                                         gridDim.x, xin);
}

// Horner step y = b + gamma P_pi x of the polynomial preconditioner; exits at
// once when ctl is given and the current GMRES cycle is done.
template <int L, int U, typename VT, typename XT, bool CORR>
__global__ __launch_bounds__(kBlock) void k_horner(int64_t S, int A, const int* __restrict__ row_ptr, int kfix,
                                                   const int* __restrict__ col, const VT* __restrict__ val,
                                                   const double* __restrict__ corr, const int* __restrict__ pi,
                                                   const XT* __restrict__ x, const XT* __restrict__ b,
                                                   double gamma, XT* __restrict__ y,
                                                   const Ctl* __restrict__ ctl) {
  if (ctl && ctl->done) return;
  horner_tile<L, U, VT, XT, CORR>(S, A, RowIndex{row_ptr, kfix}, col, val, corr, pi, x, b, gamma, y,
                                  xcd_tile(blockIdx.x, gridDim.x));
}

template <typename T>
__global__ __launch_bounds__(kBlock) void k_zero(T* __restrict__ x, int64_t n) {
  for (int64_t i = static_cast<int64_t>(blockIdx.x) * kBlock + threadIdx.x; i < n;
       i += static_cast<int64_t>(gridDim.x) * kBlock)
    x[i] = T(0);
}

// x += q (q in the basis precision)
template <typename T>
__global__ __launch_bounds__(kBlock) void k_add_to(double* __restrict__ x, const T* __restrict__ q, int64_t n) {
  for (int64_t i = static_cast<int64_t>(blockIdx.x) * kBlock + threadIdx.x; i < n;
       i += static_cast<int64_t>(gridDim.x) * kBlock)
    x[i] += static_cast<double>(q[i]);
}

__global__ __launch_bounds__(kBlock) void k_reduce_dots(const double* __restrict__ partials,
                                                        int nb, int j, Ctl* __restrict__ ctl) {
  if (ctl->done) return;
  reduce_dots_body(partials, nb, j, ctl, blockIdx.x);
}

template <typename BT>
__global__ __launch_bounds__(kBlock) void k_arnoldi_update(int64_t S, BT* __restrict__ Ub,
                                                           int64_t ldu, int j,
                                                           const Ctl* __restrict__ ctl,
                                                           double* __restrict__ partials) {
  if (ctl->done) return;
  arnoldi_update_body<BT>(S, Ub, ldu, j, ctl, partials, blockIdx.x);
}

__global__ __launch_bounds__(kBlock) void k_norm_givens(const double* __restrict__ partials,
                                                        int nb, int j, int m,
                                                        Ctl* __restrict__ ctl, int gs2) {
  if (ctl->done) return;
  norm_givens_body(partials, nb, j, m, ctl, gs2 != 0);
}

template <typename BT>
__global__ __launch_bounds__(kBlock) void k_cgs2_dots(int64_t S, const BT* __restrict__ Ub, int64_t ldu, int j,
                                                     const Ctl* __restrict__ ctl, double* __restrict__ partials) {
  if (ctl->done) return;
  cgs2_dots_tile<BT>(S, Ub, ldu, j, partials, xcd_tile(blockIdx.x, gridDim.x), gridDim.x);
}

__global__ __launch_bounds__(kBlock) void k_reduce_dots2(const double* __restrict__ partials, int nb, int j,
                                                        Ctl* __restrict__ ctl) {
  if (ctl->done) return;
  reduce_dots2_body(partials, nb, j, ctl, blockIdx.x);
}

template <typename BT, typename XT>
__global__ __launch_bounds__(kBlock) void k_gmres_update_x(int64_t S, XT* __restrict__ x,
                                                           const BT* __restrict__ Ub,
                                                           int64_t ldu,
                                                           const Ctl* __restrict__ ctl) {
  gmres_update_x_body<BT, XT>(S, x, Ub, ldu, ctl, blockIdx.x);
}

__global__ __launch_bounds__(kBlock) void k_reduce_ms(const double4* __restrict__ partials,
                                                      int nb, int mode, int first_cycle,
                                                      double alpha, double floor_rel,
                                                      Ctl* __restrict__ ctl) {
  if (mode == kRedRichardson && ctl->done) return;
  reduce_ms_body(partials, nb, mode, first_cycle, alpha, floor_rel, ctl);
}

__global__ void k_ctl_reset(Ctl* ctl, double tol) {
  if (threadIdx.x == 0 && blockIdx.x == 0) {
    ctl->res_max = 0.0;
    ctl->sumsq = 0.0;
    ctl->beta = 0.0;
    ctl->tol = tol;
    ctl->res_est = 0.0;
    ctl->beta0 = 0.0;
    ctl->tol_cycle = tol;
    ctl->aux_max = 0.0;
    ctl->orth_loss = 0.0;
    ctl->j = 0;
    ctl->done = 0;
    ctl->converged = 0;
    ctl->breakdown = 0;
    ctl->bad_policy = 0;
    ctl->steps = 0;
    ctl->rich_cur = 0;
    ctl->pad0 = 0;
  }
}

__global__ void k_rich_begin(Ctl* ctl, double tol, int cur, int steps) {
  if (threadIdx.x == 0 && blockIdx.x == 0) {
    ctl->tol = tol;
    ctl->rich_cur = cur;
    ctl->steps = steps;
    ctl->converged = 0;
    ctl->done = 0;
  }
}

__global__ __launch_bounds__(kBlock) void k_check_policy(int64_t S, int A,
                                                         const int* __restrict__ pi,
                                                         Ctl* __restrict__ ctl) {
  const int64_t s = static_cast<int64_t>(blockIdx.x) * kBlock + threadIdx.x;
  int bad = 0;
  if (s < S) bad = (pi[s] < 0 || pi[s] >= A) ? 1 : 0;
  bad = wave_sum(bad);
  if ((threadIdx.x & (kWave - 1)) == 0 && bad) atomicAdd(&ctl->bad_policy, bad);
}

__global__ __launch_bounds__(kBlock) void k_to_f32(const double* __restrict__ a,
                                                   float* __restrict__ b, int64_t n) {
  for (int64_t i = static_cast<int64_t>(blockIdx.x) * kBlock + threadIdx.x; i < n;
       i += static_cast<int64_t>(gridDim.x) * kBlock)
    b[i] = static_cast<float>(a[i]);
}

// The packed float32 copy: groups of 8 lanes per row copy its columns to
// words [2 st, st + en) and its values, rounded to float32, to [st + en, 2 en)
// (word indices up to 2*nnz, so they are formed in 64 bits).
__global__ __launch_bounds__(kBlock) void k_pack_f32(int64_t rows, const int* __restrict__ row_ptr, int kfix,
                                                    const int* __restrict__ col, const double* __restrict__ val,
                                                    float* __restrict__ cv) {
  constexpr int G = 8;
  int* __restrict__ cvi = reinterpret_cast<int*>(cv);
  const int l = threadIdx.x % G;
  for (int64_t r = (static_cast<int64_t>(blockIdx.x) * kBlock + threadIdx.x) / G; r < rows;
       r += static_cast<int64_t>(gridDim.x) * (kBlock / G)) {
    const int st = kfix > 0 ? static_cast<int>(r) * kfix : row_ptr[r];
    const int en = kfix > 0 ? st + kfix : row_ptr[r + 1];
    // word indices reach 2*nnz, beyond int32 once nnz >= 2^30: 64-bit sums
    for (int e = st + l; e < en; e += G) {
      cvi[static_cast<int64_t>(st) + e] = col[e];
      cv[static_cast<int64_t>(en) + e] = static_cast<float>(val[e]);
    }
  }
}

// One thread per row: float16 values (round to nearest even) and the row
// correction c_r = 1 - sum_j double(fp16(p_rj)) summed in entry order.
__global__ __launch_bounds__(kBlock) void k_to_f16_rows(int64_t rows,
                                                        const int* __restrict__ row_ptr,
                                                        const double* __restrict__ a,
                                                        __half* __restrict__ h,
                                                        double* __restrict__ corr) {
  for (int64_t r = static_cast<int64_t>(blockIdx.x) * kBlock + threadIdx.x; r < rows;
       r += static_cast<int64_t>(gridDim.x) * kBlock) {
    double sum = 0.0;
    for (int e = row_ptr[r]; e < row_ptr[r + 1]; ++e) {
      const __half hv = __ushort_as_half(f64_to_f16_bits(a[e]));
      h[e] = hv;
      sum += static_cast<double>(__half2float(hv));
    }
    corr[r] = 1.0 - sum;
  }
}

}  // namespace mdp

namespace mdp {

__global__ __launch_bounds__(kBlock) void k_i64_to_i32(const int64_t* __restrict__ a,
                                                       int32_t* __restrict__ b, int64_t n) {
  for (int64_t i = static_cast<int64_t>(blockIdx.x) * kBlock + threadIdx.x; i < n;
       i += static_cast<int64_t>(gridDim.x) * kBlock)
    b[i] = static_cast<int32_t>(a[i]);
}

// ----------------------------------------------------------------------------
// launchers
// ----------------------------------------------------------------------------
namespace {

// Event pair around one launch while the handle's profiler is on.
struct Prof {
  mdp_handle* h;
  int kind;
  double bytes;
  int tag;
  hipEvent_t a;
  Prof(mdp_handle* hh, int k, double b, int t = -1) : h(hh), kind(k), bytes(b), tag(t) {
    prof_begin(h, kind, &a);
  }
  ~Prof() { prof_end(h, kind, a, bytes, tag); }
};

template <int L> constexpr int rows_in_flight() { return L >= 32 ? 2 : MDP_UNROLL; }

template <typename F>
hipError_t with_lanes(int L, F&& f) {
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

inline int grid_for(int64_t n, int per) { return static_cast<int>((n + per - 1) / per); }
inline int grid_stride(int64_t n) {
  const int64_t g = (n + kBlock - 1) / kBlock;
  return static_cast<int>(g < 8192 ? (g > 0 ? g : 1) : 8192);
}

hipError_t reduce_into_ctl(mdp_handle* h, int nb, int red_mode, int first_cycle, double alpha,
                           double floor_rel) {
  if (red_mode == kRedNone) return hipSuccess;
  Prof pf(h, MDP_K_REDUCE, 0.0);
  k_reduce_ms<<<1, kBlock, 0, h->stream>>>(reinterpret_cast<const double4*>(h->part.buf), nb,
                                            red_mode, first_cycle, alpha, floor_rel, h->ctl);
  return hipGetLastError();
}

}  // namespace

size_t partials_doubles(int64_t S, int A, int m) {
  const int64_t nb_sweep = (S + sweep_tile_states(A) - 1) / sweep_tile_states(A);
  const int64_t nb_apply = (S + kApplyTile - 1) / kApplyTile;
  const int64_t nb_upd = (S + kUpdTile - 1) / kUpdTile;
  int64_t need = 4 * nb_sweep;
  need = need > 4 * nb_apply ? need : 4 * nb_apply;
  need = need > (m + 1) * nb_apply ? need : (m + 1) * nb_apply;
  need = need > nb_upd ? need : nb_upd;
  return static_cast<size_t>(need);
}

hipError_t launch_bellman(mdp_handle* h, Prec prec, const void* v, double* Tv, int32_t* pi,
                          void* r0, bool r0_f32, int red_mode, int first_cycle, double alpha,
                          double floor_rel) {
  ++h->pi_gen;  // a policy is written
  const int ts = sweep_tile_states(h->A);
  const int nb = grid_for(h->S, ts);
  auto* part = reinterpret_cast<double4*>(h->part.buf);
  hipError_t e;
  if (prec == kF64 && h->cb_blocks > 0) {
    {
      Prof pf(h, MDP_K_BELLMAN, bytes_sweep(h, 8, 8, r0 != nullptr, r0_f32 ? 4 : 8));
      e = launch_bellman_cb(h, static_cast<const double*>(v), Tv, pi, r0, r0_f32, part, nb);
    }
    if (e != hipSuccess) return e;
    return reduce_into_ctl(h, nb, red_mode, first_cycle, alpha, floor_rel);
  }
  if (prec == kF64 && h->flat_sweep) {
    {
      Prof pf(h, MDP_K_BELLMAN, bytes_sweep(h, 8, 8, r0 != nullptr, r0_f32 ? 4 : 8));
      e = launch_bellman_flat(h, static_cast<const double*>(v), Tv, pi, r0, r0_f32, part, nb);
    }
    if (e != hipSuccess) return e;
    return reduce_into_ctl(h, nb, red_mode, first_cycle, alpha, floor_rel);
  }
  {
    Prof pf(h, MDP_K_BELLMAN, bytes_sweep(h, prec == kF64 ? 8 : (prec == kF32 ? 4 : 2), prec == kF64 ? 8 : 4, r0 != nullptr, r0_f32 ? 4 : 8) + (prec == kF16 ? h->rows * 8.0 : 0.0));
    e = with_lanes(h->lanes, [&](auto Lc) -> hipError_t {
    constexpr int L = decltype(Lc)::value;
    constexpr int U = rows_in_flight<L>();
    if (prec == kF64) {
      const size_t lds = static_cast<size_t>(ts) * h->A * sizeof(double) +
                         (static_cast<size_t>(ts) * h->A + 1) * sizeof(int);
      if (r0_f32)
        k_bellman<L, U, double, double, false, float><<<nb, kBlock, lds, h->stream>>>(
            h->S, h->A, ts, h->row_ptr, h->kfix, h->col, h->val, nullptr, h->cost,
            static_cast<const double*>(v), h->gamma, Tv, pi, static_cast<float*>(r0), part);
      else
        k_bellman<L, U, double, double, false, double><<<nb, kBlock, lds, h->stream>>>(
            h->S, h->A, ts, h->row_ptr, h->kfix, h->col, h->val, nullptr, h->cost,
            static_cast<const double*>(v), h->gamma, Tv, pi, static_cast<double*>(r0), part);
    } else if (prec == kF32) {
      const size_t lds = static_cast<size_t>(ts) * h->A * sizeof(double) +
                         (static_cast<size_t>(ts) * h->A + 1) * sizeof(int);
      k_bellman<L, U, float, float, false, float><<<nb, kBlock, lds, h->stream>>>(
          h->S, h->A, ts, h->row_ptr, h->kfix, reinterpret_cast<const int*>(h->cv32), h->cv32, nullptr, h->cost,
          static_cast<const float*>(v), h->gamma, Tv, pi, static_cast<float*>(r0), part);
    } else {
      const size_t lds = static_cast<size_t>(ts) * h->A * sizeof(double) +
                         (static_cast<size_t>(ts) * h->A + 1) * sizeof(int);
      k_bellman<L, U, __half, float, true, float><<<nb, kBlock, lds, h->stream>>>(
          h->S, h->A, ts, h->row_ptr, h->kfix, h->col, h->val16, h->corr16, h->cost,
          static_cast<const float*>(v), h->gamma, Tv, pi, static_cast<float*>(r0), part);
    }
    return hipGetLastError();
  });
  }
  if (e != hipSuccess) return e;
  return reduce_into_ctl(h, nb, red_mode, first_cycle, alpha, floor_rel);
}

hipError_t launch_apply(mdp_handle* h, int mode, const int32_t* pi, const double* x, void* y,
                        bool y_f32, int red_mode, int first_cycle, double alpha,
                        double floor_rel) {
  const int nb = grid_for(h->S, kApplyTile);
  auto* part = reinterpret_cast<double4*>(h->part.buf);
  hipError_t e;
  if (mode == kApplyRes && h->pp_ready && pi == h->pp_pi) {
    Prof pf(h, MDP_K_POLICY_APPLY, bytes_apply(h, 8, 8, y_f32 ? 4 : 8));
    e = launch_pp_residual(h, x, y, y_f32, part, nb);  // on the policy's copy
  } else {
    Prof pf(h, MDP_K_POLICY_APPLY, bytes_apply(h, 8, 8, y_f32 ? 4 : 8));
    e = with_lanes(h->lanes, [&](auto Lc) -> hipError_t {
    constexpr int L = decltype(Lc)::value;
    constexpr int U = rows_in_flight<L>();
#define MDP_APPLY_ARGS(YT)                                                                 \
  h->S, h->A, h->row_ptr, h->kfix, h->col, h->val, nullptr, h->cost, pi, x, h->gamma,              \
      static_cast<YT*>(y), part, nullptr, nullptr, nullptr, nullptr
    if (mode == kApplyOp)
      k_policy_apply<L, U, kApplyOp, double, double, double, false>
          <<<nb, kBlock, 0, h->stream>>>(MDP_APPLY_ARGS(double));
    else if (mode == kApplyT)
      k_policy_apply<L, U, kApplyT, double, double, double, false>
          <<<nb, kBlock, 0, h->stream>>>(MDP_APPLY_ARGS(double));
    else if (y_f32)
      k_policy_apply<L, U, kApplyRes, double, double, float, false>
          <<<nb, kBlock, 0, h->stream>>>(MDP_APPLY_ARGS(float));
    else
      k_policy_apply<L, U, kApplyRes, double, double, double, false>
          <<<nb, kBlock, 0, h->stream>>>(MDP_APPLY_ARGS(double));
#undef MDP_APPLY_ARGS
    return hipGetLastError();
  });
  }
  if (e != hipSuccess) return e;
  return reduce_into_ctl(h, nb, red_mode, first_cycle, alpha, floor_rel);
}

hipError_t launch_richardson_step(mdp_handle* h, const int32_t* pi, double* buf0, double* buf1) {
  const int nb = grid_for(h->S, kApplyTile);
  auto* part = reinterpret_cast<double4*>(h->part.buf);
  hipError_t e;
  {
    Prof pf(h, MDP_K_POLICY_APPLY, bytes_apply(h, 8, 8, 8));
    e = with_lanes(h->lanes, [&](auto Lc) -> hipError_t {
    constexpr int L = decltype(Lc)::value;
    constexpr int U = rows_in_flight<L>();
    // current iterate in buf[rich_cur]; the kernel swaps roles when rich_cur == 1
    k_policy_apply<L, U, kApplyT, double, double, double, false><<<nb, kBlock, 0, h->stream>>>(
        h->S, h->A, h->row_ptr, h->kfix, h->col, h->val, nullptr, h->cost, pi, buf0, h->gamma, buf1,
        part, h->ctl, &h->ctl->rich_cur, buf1, buf0);
    return hipGetLastError();
  });
  }
  if (e != hipSuccess) return e;
  return reduce_into_ctl(h, nb, kRedRichardson, 0, 0.0, 0.0);
}

// y = b + gamma P_pi x in the arithmetic of `prec` (x, b, y: double* for kF64,
// float* otherwise); ctl may be null (no early exit).
hipError_t launch_horner(mdp_handle* h, Prec prec, const int32_t* pi, const void* x, const void* b, void* y,
                         const Ctl* ctl) {
  const int nb = grid_for(h->S, kApplyTile);
  Prof pf(h, MDP_K_POLICY_APPLY, bytes_apply(h, bval_of(prec), prec == kF64 ? 8 : 4, prec == kF64 ? 8 : 4) +
                                     h->S * (prec == kF64 ? 8.0 : 4.0) + (prec == kF16 ? h->S * 8.0 : 0.0));
  if ((prec == kF64 || prec == kF32) && h->pp_ready && pi == h->pp_pi)
    return launch_pp_horner(h, prec == kF32, x, b, y, ctl);  // on the policy's copy
  return with_lanes(h->lanes, [&](auto Lc) -> hipError_t {
    constexpr int L = decltype(Lc)::value;
    constexpr int U = rows_in_flight<L>();
    if (prec == kF64)
      k_horner<L, U, double, double, false><<<nb, kBlock, 0, h->stream>>>(
          h->S, h->A, h->row_ptr, h->kfix, h->col, h->val, nullptr, pi, static_cast<const double*>(x),
          static_cast<const double*>(b), h->gamma, static_cast<double*>(y), ctl);
    else if (prec == kF32)
      k_horner<L, U, float, float, false><<<nb, kBlock, 0, h->stream>>>(
          h->S, h->A, h->row_ptr, h->kfix, reinterpret_cast<const int*>(h->cv32), h->cv32, nullptr, pi,
          static_cast<const float*>(x), static_cast<const float*>(b), h->gamma, static_cast<float*>(y), ctl);
    else
      k_horner<L, U, __half, float, true><<<nb, kBlock, 0, h->stream>>>(
          h->S, h->A, h->row_ptr, h->kfix, h->col, h->val16, h->corr16, pi, static_cast<const float*>(x),
          static_cast<const float*>(b), h->gamma, static_cast<float*>(y), ctl);
    return hipGetLastError();
  });
}

// Basis slot i of the basis precision of `prec`.
void* basis_slot(mdp_handle* h, Prec prec, int i) {
  if (prec == kF64) return h->U64 + static_cast<int64_t>(i) * h->ldu;
  return h->U32 + static_cast<int64_t>(i) * h->ldu;
}

// M^-1 u = sum_{i<deg} (gamma P_pi)^i u by deg - 1 Horner steps from u, using
// the two scratch slots a and b; returns the slot holding the result (u itself
// when deg <= 1).
void* precond_apply(mdp_handle* h, Prec prec, const int32_t* pi, void* u, int a, int b, int deg,
                    const Ctl* ctl, hipError_t* err) {
  void* cur = u;
  *err = hipSuccess;
  for (int k = 1; k < deg && *err == hipSuccess; ++k) {
    void* nxt = basis_slot(h, prec, (k & 1) ? a : b);
    *err = launch_horner(h, prec, pi, cur, u, nxt, ctl);
    cur = nxt;
  }
  return cur;
}

hipError_t launch_arnoldi_step(mdp_handle* h, Prec prec, const int32_t* pi, int j, int m, int deg, bool gs2) {
  const int nb = grid_for(h->S, kApplyTile);
  hipError_t e;
  const Prec bprec = prec == kF64 ? kF64 : kF32;
  // polynomial preconditioning (deg > 1): the product runs on q = M^-1 U_j,
  // built in basis slots m + 1 and m + 2
  const void* xin = nullptr;
  if (deg > 1) {
    xin = precond_apply(h, prec, pi, basis_slot(h, bprec, j), m + 1, m + 2, deg, h->ctl, &e);
    if (e != hipSuccess) return e;
  }
  int nb_dots = nb;  // tiles of the dot partials
  if ((prec == kF64 || prec == kF32) && h->pp_ready && pi == h->pp_pi) {
    // the XCD-partitioned product on the policy's copy (same outputs)
    Prof pf(h, MDP_K_ARNOLDI_APPLY, bytes_arnoldi_apply(h, 8, prec == kF64 ? 8 : 4, j), j);
    e = launch_pp_arnoldi_apply(h, prec == kF32, j, xin, h->part.buf, nb, &nb_dots);
  } else {
    Prof pf(h, MDP_K_ARNOLDI_APPLY, bytes_arnoldi_apply(h, prec == kF64 ? 8 : (prec == kF32 ? 4 : 2), prec == kF64 ? 8 : 4, j) + (prec == kF16 ? h->S * 8.0 : 0.0), j);
    e = with_lanes(h->lanes, [&](auto Lc) -> hipError_t {
    constexpr int L = decltype(Lc)::value;
    constexpr int U = rows_in_flight<L>();
    if (prec == kF64)
      k_arnoldi_apply<L, U, double, double, false><<<nb, kBlock, 0, h->stream>>>(
          h->S, h->A, h->row_ptr, h->kfix, h->col, h->val, nullptr, pi, h->U64, h->ldu, j, h->gamma,
          h->ctl, h->part.buf, static_cast<const double*>(xin));
    else if (prec == kF32)
      k_arnoldi_apply<L, U, float, float, false><<<nb, kBlock, 0, h->stream>>>(
          h->S, h->A, h->row_ptr, h->kfix, reinterpret_cast<const int*>(h->cv32), h->cv32, nullptr, pi, h->U32,
          h->ldu, j, h->gamma,
          h->ctl, h->part.buf, static_cast<const float*>(xin));
    else
      k_arnoldi_apply<L, U, __half, float, true><<<nb, kBlock, 0, h->stream>>>(
          h->S, h->A, h->row_ptr, h->kfix, h->col, h->val16, h->corr16, pi, h->U32, h->ldu, j, h->gamma,
          h->ctl, h->part.buf, static_cast<const float*>(xin));
    return hipGetLastError();
  });
  }
  if (e != hipSuccess) return e;
  {
    Prof pf(h, MDP_K_REDUCE, 0.0, j);
    k_reduce_dots<<<j + 1, kBlock, 0, h->stream>>>(h->part.buf, nb_dots, j, h->ctl);
  }
  if ((e = hipGetLastError()) != hipSuccess) return e;
  const int nbu = grid_for(h->S, kUpdTile);
  {
  Prof pf(h, MDP_K_ARNOLDI_UPDATE, bytes_arnoldi_update(h, prec == kF64 ? 8 : 4, j), j);
  if (prec == kF64)
    k_arnoldi_update<double><<<nbu, kBlock, 0, h->stream>>>(h->S, h->U64, h->ldu, j, h->ctl,
                                                             h->part.buf);
  else
    k_arnoldi_update<float><<<nbu, kBlock, 0, h->stream>>>(h->S, h->U32, h->ldu, j, h->ctl,
                                                            h->part.buf);
  }
  if ((e = hipGetLastError()) != hipSuccess) return e;
  if (gs2) {
    {
      Prof pf(h, MDP_K_ARNOLDI_UPDATE, h->S * (j + 2.0) * (prec == kF64 ? 8.0 : 4.0), j);
      if (prec == kF64)
        k_cgs2_dots<double><<<nb, kBlock, 0, h->stream>>>(h->S, h->U64, h->ldu, j, h->ctl, h->part.buf);
      else
        k_cgs2_dots<float><<<nb, kBlock, 0, h->stream>>>(h->S, h->U32, h->ldu, j, h->ctl, h->part.buf);
    }
    if ((e = hipGetLastError()) != hipSuccess) return e;
    {
      Prof pf(h, MDP_K_REDUCE, 0.0, j);
      k_reduce_dots2<<<j + 1, kBlock, 0, h->stream>>>(h->part.buf, nb, j, h->ctl);
    }
    if ((e = hipGetLastError()) != hipSuccess) return e;
    {
      Prof pf(h, MDP_K_ARNOLDI_UPDATE, bytes_arnoldi_update(h, prec == kF64 ? 8 : 4, j), j);
      if (prec == kF64)
        k_arnoldi_update<double><<<nbu, kBlock, 0, h->stream>>>(h->S, h->U64, h->ldu, j, h->ctl, h->part.buf);
      else
        k_arnoldi_update<float><<<nbu, kBlock, 0, h->stream>>>(h->S, h->U32, h->ldu, j, h->ctl, h->part.buf);
    }
    if ((e = hipGetLastError()) != hipSuccess) return e;
  }
  Prof pf(h, MDP_K_REDUCE, 0.0, j);
  k_norm_givens<<<1, kBlock, 0, h->stream>>>(h->part.buf, nbu, j, m, h->ctl, gs2 ? 1 : 0);
  return hipGetLastError();
}

hipError_t launch_gmres_update_x(mdp_handle* h, Prec prec, double* x) {
  const int nbu = grid_for(h->S, kUpdTile);
  Prof pf(h, MDP_K_GMRES_UPDATE_X, 0.0);
  if (prec == kF64)
    k_gmres_update_x<double, double><<<nbu, kBlock, 0, h->stream>>>(h->S, x, h->U64, h->ldu,
                                                                     h->ctl);
  else
    k_gmres_update_x<float, double><<<nbu, kBlock, 0, h->stream>>>(h->S, x, h->U32, h->ldu,
                                                                    h->ctl);
  return hipGetLastError();
}

// End of a preconditioned GMRES cycle: x += M^-1 (V y).  V y goes to basis
// slot m + 1 (in the basis precision), M^-1 uses slots m + 2 and m + 3.
hipError_t launch_precond_update_x(mdp_handle* h, Prec prec, const int32_t* pi, double* x, int m, int deg) {
  const Prec bprec = prec == kF64 ? kF64 : kF32;
  const int nbu = grid_for(h->S, kUpdTile);
  void* t = basis_slot(h, bprec, m + 1);
  hipError_t e;
  {
    Prof pf(h, MDP_K_GMRES_UPDATE_X, 0.0);
    if (bprec == kF64) {
      k_zero<double><<<grid_stride(h->S), kBlock, 0, h->stream>>>(static_cast<double*>(t), h->S);
      k_gmres_update_x<double, double><<<nbu, kBlock, 0, h->stream>>>(h->S, static_cast<double*>(t), h->U64,
                                                                       h->ldu, h->ctl);
    } else {
      k_zero<float><<<grid_stride(h->S), kBlock, 0, h->stream>>>(static_cast<float*>(t), h->S);
      k_gmres_update_x<float, float><<<nbu, kBlock, 0, h->stream>>>(h->S, static_cast<float*>(t), h->U32,
                                                                     h->ldu, h->ctl);
    }
    if ((e = hipGetLastError()) != hipSuccess) return e;
  }
  void* q = precond_apply(h, prec, pi, t, m + 2, m + 3, deg, nullptr, &e);
  if (e != hipSuccess) return e;
  Prof pf(h, MDP_K_GMRES_UPDATE_X, 0.0);
  if (bprec == kF64)
    k_add_to<double><<<grid_stride(h->S), kBlock, 0, h->stream>>>(x, static_cast<const double*>(q), h->S);
  else
    k_add_to<float><<<grid_stride(h->S), kBlock, 0, h->stream>>>(x, static_cast<const float*>(q), h->S);
  return hipGetLastError();
}

hipError_t launch_check_policy(mdp_handle* h, const int32_t* pi) {
  Prof pf(h, MDP_K_OTHER, 0.0);
  k_check_policy<<<grid_for(h->S, kBlock), kBlock, 0, h->stream>>>(h->S, h->A, pi, h->ctl);
  return hipGetLastError();
}

hipError_t launch_ctl_reset(mdp_handle* h, double tol) {
  Prof pf(h, MDP_K_OTHER, 0.0);
  k_ctl_reset<<<1, 64, 0, h->stream>>>(h->ctl, tol);
  return hipGetLastError();
}

hipError_t launch_rich_begin(mdp_handle* h, double tol, int cur, int steps) {
  Prof pf(h, MDP_K_OTHER, 0.0);
  k_rich_begin<<<1, 64, 0, h->stream>>>(h->ctl, tol, cur, steps);
  return hipGetLastError();
}

hipError_t launch_build_lowp(mdp_handle* h, int which) {
  if (which & MDP_BUILD_FP32) {
    k_pack_f32<<<grid_stride(h->rows), kBlock, 0, h->stream>>>(h->rows, h->row_ptr, h->kfix, h->col, h->val,
                                                                h->cv32);
    hipError_t e = hipGetLastError();
    if (e != hipSuccess) return e;
  }
  if (which & MDP_BUILD_FP16) {
    k_to_f16_rows<<<grid_stride(h->rows), kBlock, 0, h->stream>>>(h->rows, h->row_ptr, h->val,
                                                                   h->val16, h->corr16);
    return hipGetLastError();
  }
  return hipSuccess;
}

hipError_t launch_cast_f32(hipStream_t st, const double* src, float* dst, int64_t n) {
  k_to_f32<<<grid_stride(n), kBlock, 0, st>>>(src, dst, n);
  return hipGetLastError();
}

hipError_t launch_i64_to_i32(hipStream_t st, const int64_t* src, int32_t* dst, int64_t n) {
  k_i64_to_i32<<<grid_stride(n), kBlock, 0, st>>>(src, dst, n);
  return hipGetLastError();
}

}  // namespace mdp
