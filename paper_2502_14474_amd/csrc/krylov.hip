// Short-recurrence Krylov solvers for the policy-evaluation system
// (I - gamma P_pi) x = g_pi in float64: BiCGSTAB (van der Vorst, 1992) and
// TFQMR (Freund, 1993).  The policy products use the same tile body as the
// GMRES path.
#include <algorithm>

#include "device.h"
// ----------------------------------------------------------------------------
// BiCGSTAB (van der Vorst, 1992) on A x = g_pi with A = I - gamma P_pi, in
// float64.  Every kernel exits at once when ctl->done is set, so steps
// enqueued past convergence cost only their launches.  Scalars live in ctl;
// each reduction is per-workgroup partials (kUpdTile entries each) summed in
// a fixed order by one workgroup, so the iteration is deterministic.
// ----------------------------------------------------------------------------
namespace mdp {

namespace {

constexpr int kBiPer = kUpdTile / kBlock;

inline int grid_for(int64_t n, int per) { return static_cast<int>((n + per - 1) / per); }

// event-pair timing of one launch when the handle's profiler asks for it
struct Prof {
  mdp_handle* h;
  int kind;
  double bytes;
  hipEvent_t a;
  Prof(mdp_handle* hh, int k, double b) : h(hh), kind(k), bytes(b) { prof_begin(h, kind, &a); }
  ~Prof() { prof_end(h, kind, a, bytes, -1); }
};

// y = x - gamma P_pi x (the policy product of the GMRES path), skipped once ctl->done
template <int L, int U>
__global__ __launch_bounds__(kBlock) void k_bi_apply(int64_t S, int A, const int* __restrict__ row_ptr,
                                                     int kfix, const int* __restrict__ col,
                                                     const double* __restrict__ val,
                                                     const int* __restrict__ pi,
                                                     const double* __restrict__ x, double gamma,
                                                     double* __restrict__ y,
                                                     const Ctl* __restrict__ ctl) {
  if (ctl->done) return;
  apply_tile<L, U, kApplyOp, double, double, double, false>(S, A, RowIndex{row_ptr, kfix}, col, val,
                                                             nullptr, nullptr, pi, x, gamma, y,
                                                             nullptr, xcd_tile(blockIdx.x, gridDim.x));
}

__global__ __launch_bounds__(kBlock) void k_bi_init(int64_t S, double* __restrict__ U, int64_t ldu,
                                                    Ctl* __restrict__ ctl) {
  if (ctl->done) return;
  const double* r = U;
  double* rh = U + ldu;
  double* p = U + 2 * ldu;
  for (int64_t i = static_cast<int64_t>(blockIdx.x) * kBlock + threadIdx.x; i < S;
       i += static_cast<int64_t>(gridDim.x) * kBlock) {
    rh[i] = r[i];
    p[i] = r[i];
  }
  if (blockIdx.x == 0 && threadIdx.x == 0) {
    ctl->bi_rho = ctl->sumsq;  // (r^, r0) = ||r0||^2
    ctl->bi_alpha = 1.0;
    ctl->bi_omega = 1.0;
    ctl->bi_beta = 0.0;
  }
}

// partials[blk] = sum over the workgroup's entries of a*b (and of c*d in .y)
template <bool TWO>
__global__ __launch_bounds__(kBlock) void k_bi_dot(int64_t S, const double* __restrict__ a,
                                                   const double* __restrict__ b,
                                                   const double* __restrict__ c,
                                                   const double* __restrict__ d,
                                                   double2* __restrict__ partials,
                                                   const Ctl* __restrict__ ctl) {
  if (ctl->done) return;
  const int64_t base = static_cast<int64_t>(blockIdx.x) * kUpdTile + threadIdx.x;
  double s1 = 0.0, s2 = 0.0;
#pragma unroll
  for (int k = 0; k < kBiPer; ++k) {
    const int64_t i = base + k * kBlock;
    if (i < S) {
      s1 = fma(a[i], b[i], s1);
      if (TWO) s2 = fma(c[i], d[i], s2);
    }
  }
  double m1 = 0.0, m2 = 0.0;
  block_max_sum(m1, s1);
  if (TWO) block_max_sum(m2, s2);
  if (threadIdx.x == 0) partials[blockIdx.x] = make_double2(s1, s2);
}

__device__ __forceinline__ double2 sum_partials2(const double2* __restrict__ partials, int nb) {
  double s1 = 0.0, s2 = 0.0;
  for (int b = threadIdx.x; b < nb; b += kBlock) {
    s1 += partials[b].x;
    s2 += partials[b].y;
  }
  double m1 = 0.0, m2 = 0.0;
  block_max_sum(m1, s1);
  block_max_sum(m2, s2);
  return make_double2(s1, s2);  // valid in thread 0
}

// alpha = rho / (r^, v); a zero or non-finite quotient ends the solve
__global__ __launch_bounds__(kBlock) void k_bi_alpha(const double2* __restrict__ partials, int nb,
                                                     Ctl* __restrict__ ctl) {
  if (ctl->done) return;
  const double2 s = sum_partials2(partials, nb);
  if (threadIdx.x != 0) return;
  const double a = ctl->bi_rho / s.x;
  if (!(s.x != 0.0) || !(a != 0.0) || !std::isfinite(a)) {
    ctl->breakdown = 1;
    ctl->done = 1;
    return;
  }
  ctl->bi_alpha = a;
}

// s = r - alpha v
__global__ __launch_bounds__(kBlock) void k_bi_s(int64_t S, const double* __restrict__ r,
                                                 const double* __restrict__ v, double* __restrict__ s,
                                                 const Ctl* __restrict__ ctl) {
  if (ctl->done) return;
  const double a = ctl->bi_alpha;
  const int64_t base = static_cast<int64_t>(blockIdx.x) * kUpdTile + threadIdx.x;
#pragma unroll
  for (int k = 0; k < kBiPer; ++k) {
    const int64_t i = base + k * kBlock;
    if (i < S) s[i] = fma(-a, v[i], r[i]);
  }
}

// omega = (t, s) / (t, t); t = 0 (s = 0) gives omega = 0
__global__ __launch_bounds__(kBlock) void k_bi_omega(const double2* __restrict__ partials, int nb,
                                                     Ctl* __restrict__ ctl) {
  if (ctl->done) return;
  const double2 s = sum_partials2(partials, nb);
  if (threadIdx.x != 0) return;
  ctl->bi_omega = s.y > 0.0 ? s.x / s.y : 0.0;
}

// x += alpha p + omega s;  r = s - omega t;  partials ((r^, r), (r, r))
__global__ __launch_bounds__(kBlock) void k_bi_xr(int64_t S, double* __restrict__ x,
                                                  const double* __restrict__ p,
                                                  const double* __restrict__ s,
                                                  const double* __restrict__ t,
                                                  double* __restrict__ r,
                                                  const double* __restrict__ rh,
                                                  double2* __restrict__ partials,
                                                  const Ctl* __restrict__ ctl) {
  if (ctl->done) return;
  const double a = ctl->bi_alpha, w = ctl->bi_omega;
  const int64_t base = static_cast<int64_t>(blockIdx.x) * kUpdTile + threadIdx.x;
  double s1 = 0.0, s2 = 0.0;
#pragma unroll
  for (int k = 0; k < kBiPer; ++k) {
    const int64_t i = base + k * kBlock;
    if (i < S) {
      x[i] = fma(w, s[i], fma(a, p[i], x[i]));
      const double ri = fma(-w, t[i], s[i]);
      r[i] = ri;
      s1 = fma(rh[i], ri, s1);
      s2 = fma(ri, ri, s2);
    }
  }
  double m1 = 0.0, m2 = 0.0;
  block_max_sum(m1, s1);
  block_max_sum(m2, s2);
  if (threadIdx.x == 0) partials[blockIdx.x] = make_double2(s1, s2);
}

// rho' = (r^, r), ||r||; stop test; beta = (rho'/rho)(alpha/omega)
__global__ __launch_bounds__(kBlock) void k_bi_rho(const double2* __restrict__ partials, int nb,
                                                   Ctl* __restrict__ ctl) {
  if (ctl->done) return;
  const double2 s = sum_partials2(partials, nb);
  if (threadIdx.x != 0) return;
  const double res = sqrt(s.y);
  ctl->res_est = res;
  ctl->steps += 1;
  if (!std::isfinite(res)) {
    ctl->done = 1;
    return;
  }
  if (res <= ctl->tol) {
    ctl->converged = 1;
    ctl->done = 1;
    return;
  }
  const double beta = (s.x / ctl->bi_rho) * (ctl->bi_alpha / ctl->bi_omega);
  if (!(ctl->bi_omega != 0.0) || !(s.x != 0.0) || !std::isfinite(beta)) {
    ctl->breakdown = 1;
    ctl->done = 1;
    return;
  }
  ctl->bi_rho = s.x;
  ctl->bi_beta = beta;
}

// p = r + beta (p - omega v)
__global__ __launch_bounds__(kBlock) void k_bi_p(int64_t S, double* __restrict__ p,
                                                 const double* __restrict__ r,
                                                 const double* __restrict__ v,
                                                 const Ctl* __restrict__ ctl) {
  if (ctl->done) return;
  const double b = ctl->bi_beta, w = ctl->bi_omega;
  const int64_t base = static_cast<int64_t>(blockIdx.x) * kUpdTile + threadIdx.x;
#pragma unroll
  for (int k = 0; k < kBiPer; ++k) {
    const int64_t i = base + k * kBlock;
    if (i < S) p[i] = fma(b, fma(-w, v[i], p[i]), r[i]);
  }
}

// ---- TFQMR ------------------------------------------------------------------
// Freund's transpose-free QMR: two products per iteration (A y2 and the next
// A y1), a quasi-minimal residual update of x at every half-step, and the
// bound tau * sqrt(m + 1) on the residual norm after half-step m as the stop
// test.  Slots 0..7 of the float64 basis hold r^, w, y1, y2, v, d, u = A y2
// and t = A y1; v is the direction of the underlying squared method,
// v = A y1 + beta (A y2 + beta v), not A y1 itself.

// r^ = w = y1 = r0 (in slot 0 on entry, moved so that slot 0 is r^), d = 0;
// rho = (r^, r0) = ||r0||^2, tau = ||r0||
__global__ __launch_bounds__(kBlock) void k_tf_init(int64_t S, double* __restrict__ U, int64_t ldu,
                                                    Ctl* __restrict__ ctl) {
  if (ctl->done) return;
  const double* r0 = U;
  double* w = U + ldu;
  double* y1 = U + 2 * ldu;
  double* d = U + 5 * ldu;
  for (int64_t i = static_cast<int64_t>(blockIdx.x) * kBlock + threadIdx.x; i < S;
       i += static_cast<int64_t>(gridDim.x) * kBlock) {
    w[i] = r0[i];
    y1[i] = r0[i];
    d[i] = 0.0;
  }
  if (blockIdx.x == 0 && threadIdx.x == 0) {
    ctl->bi_rho = ctl->sumsq;
    ctl->tf_tau = sqrt(ctl->sumsq);
    ctl->tf_theta = 0.0;
    ctl->tf_eta = 0.0;
    ctl->tf_half = 0.0;
    ctl->tf_stop = 0;
  }
}

// alpha = rho / (r^, v)
__global__ __launch_bounds__(kBlock) void k_tf_alpha(const double2* __restrict__ partials, int nb,
                                                     Ctl* __restrict__ ctl) {
  if (ctl->done) return;
  const double2 s = sum_partials2(partials, nb);
  if (threadIdx.x != 0) return;
  const double a = ctl->bi_rho / s.x;
  // alpha = 0 (rho = 0) would divide the next direction update by zero
  if (!(s.x != 0.0) || !(a != 0.0) || !std::isfinite(a)) {
    ctl->breakdown = 1;
    ctl->done = 1;
    return;
  }
  ctl->bi_alpha = a;
}

// y2 = y1 - alpha v
__global__ __launch_bounds__(kBlock) void k_tf_y2(int64_t S, const double* __restrict__ y1,
                                                  const double* __restrict__ v, double* __restrict__ y2,
                                                  const Ctl* __restrict__ ctl) {
  if (ctl->done) return;
  const double a = ctl->bi_alpha;
  const int64_t base = static_cast<int64_t>(blockIdx.x) * kUpdTile + threadIdx.x;
#pragma unroll
  for (int k = 0; k < kBiPer; ++k) {
    const int64_t i = base + k * kBlock;
    if (i < S) y2[i] = fma(-a, v[i], y1[i]);
  }
}

// half-step: w -= alpha A y;  d = y + (theta^2 eta / alpha) d;  partials ||w||^2
__global__ __launch_bounds__(kBlock) void k_tf_half(int64_t S, const double* __restrict__ y,
                                                    const double* __restrict__ Ay,
                                                    double* __restrict__ w, double* __restrict__ d,
                                                    double2* __restrict__ partials,
                                                    const Ctl* __restrict__ ctl) {
  if (ctl->done) return;
  const double a = ctl->bi_alpha;
  const double coef = ctl->tf_theta * ctl->tf_theta * ctl->tf_eta / a;
  const int64_t base = static_cast<int64_t>(blockIdx.x) * kUpdTile + threadIdx.x;
  double s1 = 0.0;
#pragma unroll
  for (int k = 0; k < kBiPer; ++k) {
    const int64_t i = base + k * kBlock;
    if (i < S) {
      const double wi = fma(-a, Ay[i], w[i]);
      w[i] = wi;
      d[i] = fma(coef, d[i], y[i]);
      s1 = fma(wi, wi, s1);
    }
  }
  double m1 = 0.0;
  block_max_sum(m1, s1);
  if (threadIdx.x == 0) partials[blockIdx.x] = make_double2(s1, 0.0);
}

// theta = ||w|| / tau, c = 1 / sqrt(1 + theta^2), tau = tau theta c, eta = c^2 alpha
__global__ __launch_bounds__(kBlock) void k_tf_scal(const double2* __restrict__ partials, int nb,
                                                    Ctl* __restrict__ ctl) {
  if (ctl->done) return;
  const double2 s = sum_partials2(partials, nb);
  if (threadIdx.x != 0) return;
  const double theta = sqrt(s.x) / ctl->tf_tau;
  const double c = 1.0 / sqrt(1.0 + theta * theta);
  const double tau = ctl->tf_tau * theta * c;
  ctl->tf_theta = theta;
  ctl->tf_tau = tau;
  ctl->tf_eta = c * c * ctl->bi_alpha;
  ctl->tf_half += 1.0;
  const double bound = tau * sqrt(ctl->tf_half + 1.0);
  ctl->res_est = bound;
  if (!std::isfinite(bound)) {
    ctl->done = 1;
  } else if (bound <= ctl->tol) {
    ctl->converged = 1;
    ctl->tf_stop = 1;  // the x update of this half-step still runs
  }
}

// x += eta d; then, if the bound was met, end the solve
__global__ __launch_bounds__(kBlock) void k_tf_x(int64_t S, double* __restrict__ x,
                                                 const double* __restrict__ d,
                                                 const Ctl* __restrict__ ctl) {
  if (ctl->done) return;
  const double eta = ctl->tf_eta;
  const int64_t base = static_cast<int64_t>(blockIdx.x) * kUpdTile + threadIdx.x;
#pragma unroll
  for (int k = 0; k < kBiPer; ++k) {
    const int64_t i = base + k * kBlock;
    if (i < S) x[i] = fma(eta, d[i], x[i]);
  }
}

// counts an iteration after its second half-step (or when the first one met
// the bound) and ends the solve once the bound is met
__global__ void k_tf_finish(Ctl* __restrict__ ctl, int second_half) {
  if (ctl->done) return;
  if (second_half || ctl->tf_stop) ctl->steps += 1;
  if (ctl->tf_stop) ctl->done = 1;
}

// rho' = (r^, w); beta = rho'/rho
__global__ __launch_bounds__(kBlock) void k_tf_beta(const double2* __restrict__ partials, int nb,
                                                    Ctl* __restrict__ ctl) {
  if (ctl->done) return;
  const double2 s = sum_partials2(partials, nb);
  if (threadIdx.x != 0) return;
  const double b = s.x / ctl->bi_rho;
  if (!(ctl->bi_rho != 0.0) || !(s.x != 0.0) || !std::isfinite(b)) {
    ctl->breakdown = 1;
    ctl->done = 1;
    return;
  }
  ctl->bi_rho = s.x;
  ctl->bi_beta = b;
}

// y1 = w + beta y2
__global__ __launch_bounds__(kBlock) void k_tf_y1(int64_t S, const double* __restrict__ w,
                                                  const double* __restrict__ y2, double* __restrict__ y1,
                                                  const Ctl* __restrict__ ctl) {
  if (ctl->done) return;
  const double b = ctl->bi_beta;
  const int64_t base = static_cast<int64_t>(blockIdx.x) * kUpdTile + threadIdx.x;
#pragma unroll
  for (int k = 0; k < kBiPer; ++k) {
    const int64_t i = base + k * kBlock;
    if (i < S) y1[i] = fma(b, y2[i], w[i]);
  }
}

// v = A y1 + beta (u + beta v), with A y1 in t
__global__ __launch_bounds__(kBlock) void k_tf_v(int64_t S, const double* __restrict__ t,
                                                 const double* __restrict__ u, double* __restrict__ v,
                                                 const Ctl* __restrict__ ctl) {
  if (ctl->done) return;
  const double b = ctl->bi_beta;
  const int64_t base = static_cast<int64_t>(blockIdx.x) * kUpdTile + threadIdx.x;
#pragma unroll
  for (int k = 0; k < kBiPer; ++k) {
    const int64_t i = base + k * kBlock;
    if (i < S) v[i] = fma(b, fma(b, v[i], u[i]), t[i]);
  }
}

}  // namespace

hipError_t launch_bicgstab_init(mdp_handle* h) {
  const int g = static_cast<int>(std::min<int64_t>(8192, std::max<int64_t>(1, (h->S + kBlock - 1) / kBlock)));
  k_bi_init<<<g, kBlock, 0, h->stream>>>(h->S, h->U64, h->ldu, h->ctl);
  return hipGetLastError();
}

// out = in - gamma P_pi in, skipped once ctl->done
hipError_t krylov_product(mdp_handle* h, const int32_t* pi, const double* in, double* out) {
  const int64_t S = h->S;
  const int nba = grid_for(S, kApplyTile);
  Prof pf(h, MDP_K_POLICY_APPLY, bytes_apply(h, 8, 8, 8));
  if (h->pp_ready && pi == h->pp_pi) return launch_pp_op(h, in, out);  // on the policy's copy
#define MDP_KR_APPLY(LL, UU)                                                              \
  k_bi_apply<LL, UU><<<nba, kBlock, 0, h->stream>>>(S, h->A, h->row_ptr, h->kfix, h->col, h->val, \
                                                     pi, in, h->gamma, out, h->ctl)
  switch (h->lanes) {
    case 2: MDP_KR_APPLY(2, MDP_UNROLL); break;
    case 4: MDP_KR_APPLY(4, MDP_UNROLL); break;
    case 8: MDP_KR_APPLY(8, MDP_UNROLL); break;
    case 16: MDP_KR_APPLY(16, MDP_UNROLL); break;
    case 32: MDP_KR_APPLY(32, 2); break;
    case 64: MDP_KR_APPLY(64, 2); break;
    default: return hipErrorInvalidValue;
  }
#undef MDP_KR_APPLY
  return hipGetLastError();
}

hipError_t launch_tfqmr_init(mdp_handle* h, const int32_t* pi) {
  const int g = static_cast<int>(std::min<int64_t>(8192, std::max<int64_t>(1, (h->S + kBlock - 1) / kBlock)));
  k_tf_init<<<g, kBlock, 0, h->stream>>>(h->S, h->U64, h->ldu, h->ctl);
  hipError_t e = hipGetLastError();
  if (e != hipSuccess) return e;
  // t = A y1, and v = t for the first iteration
  double* t = h->U64 + 7 * h->ldu;
  if ((e = krylov_product(h, pi, h->U64 + 2 * h->ldu, t)) != hipSuccess) return e;
  return hipMemcpyAsync(h->U64 + 4 * h->ldu, t, h->S * sizeof(double), hipMemcpyDeviceToDevice,
                        h->stream);
}

hipError_t launch_tfqmr_step(mdp_handle* h, const int32_t* pi, double* x) {
  const int64_t S = h->S, ld = h->ldu;
  const double* rh = h->U64;
  double* w = h->U64 + ld;
  double* y1 = h->U64 + 2 * ld;
  double* y2 = h->U64 + 3 * ld;
  double* v = h->U64 + 4 * ld;
  double* d = h->U64 + 5 * ld;
  double* u = h->U64 + 6 * ld;
  double* t = h->U64 + 7 * ld;
  auto* part = reinterpret_cast<double2*>(h->part.buf);
  const int nbu = grid_for(S, kUpdTile);
  hipError_t e;
  {
    Prof pf(h, MDP_K_REDUCE, 0.0);
    k_bi_dot<false><<<nbu, kBlock, 0, h->stream>>>(S, rh, v, nullptr, nullptr, part, h->ctl);
    k_tf_alpha<<<1, kBlock, 0, h->stream>>>(part, nbu, h->ctl);
    k_tf_y2<<<nbu, kBlock, 0, h->stream>>>(S, y1, v, y2, h->ctl);
    // half-step 2n-1 with y1 (A y1 = t, from the end of the previous iteration)
    k_tf_half<<<nbu, kBlock, 0, h->stream>>>(S, y1, t, w, d, part, h->ctl);
    k_tf_scal<<<1, kBlock, 0, h->stream>>>(part, nbu, h->ctl);
    k_tf_x<<<nbu, kBlock, 0, h->stream>>>(S, x, d, h->ctl);
    k_tf_finish<<<1, 1, 0, h->stream>>>(h->ctl, 0);
  }
  if ((e = krylov_product(h, pi, y2, u)) != hipSuccess) return e;
  {
    Prof pf(h, MDP_K_REDUCE, 0.0);
    // half-step 2n with y2 (A y2 = u)
    k_tf_half<<<nbu, kBlock, 0, h->stream>>>(S, y2, u, w, d, part, h->ctl);
    k_tf_scal<<<1, kBlock, 0, h->stream>>>(part, nbu, h->ctl);
    k_tf_x<<<nbu, kBlock, 0, h->stream>>>(S, x, d, h->ctl);
    k_tf_finish<<<1, 1, 0, h->stream>>>(h->ctl, 1);
    k_bi_dot<false><<<nbu, kBlock, 0, h->stream>>>(S, rh, w, nullptr, nullptr, part, h->ctl);
    k_tf_beta<<<1, kBlock, 0, h->stream>>>(part, nbu, h->ctl);
    k_tf_y1<<<nbu, kBlock, 0, h->stream>>>(S, w, y2, y1, h->ctl);
  }
  if ((e = krylov_product(h, pi, y1, t)) != hipSuccess) return e;
  k_tf_v<<<nbu, kBlock, 0, h->stream>>>(S, t, u, v, h->ctl);
  return hipGetLastError();
}

hipError_t launch_bicgstab_step(mdp_handle* h, const int32_t* pi, double* x) {
  const int64_t S = h->S, ld = h->ldu;
  double* r = h->U64;
  double* rh = h->U64 + ld;
  double* p = h->U64 + 2 * ld;
  double* v = h->U64 + 3 * ld;
  double* s = h->U64 + 4 * ld;
  double* t = h->U64 + 5 * ld;
  auto* part = reinterpret_cast<double2*>(h->part.buf);
  const int nbu = grid_for(S, kUpdTile);
  auto product = [&](const double* in, double* out) -> hipError_t {
    return krylov_product(h, pi, in, out);
  };
  hipError_t e;
  if ((e = product(p, v)) != hipSuccess) return e;
  {
    Prof pf(h, MDP_K_REDUCE, 0.0);
    k_bi_dot<false><<<nbu, kBlock, 0, h->stream>>>(S, rh, v, nullptr, nullptr, part, h->ctl);
    k_bi_alpha<<<1, kBlock, 0, h->stream>>>(part, nbu, h->ctl);
    k_bi_s<<<nbu, kBlock, 0, h->stream>>>(S, r, v, s, h->ctl);
  }
  if ((e = product(s, t)) != hipSuccess) return e;
  {
    Prof pf(h, MDP_K_REDUCE, 0.0);
    k_bi_dot<true><<<nbu, kBlock, 0, h->stream>>>(S, t, s, t, t, part, h->ctl);
    k_bi_omega<<<1, kBlock, 0, h->stream>>>(part, nbu, h->ctl);
    k_bi_xr<<<nbu, kBlock, 0, h->stream>>>(S, x, p, s, t, r, rh, part, h->ctl);
    k_bi_rho<<<1, kBlock, 0, h->stream>>>(part, nbu, h->ctl);
    k_bi_p<<<nbu, kBlock, 0, h->stream>>>(S, p, r, v, h->ctl);
  }
  return hipGetLastError();
}

}  // namespace mdp
