// Float64 Bellman sweep over a caller's CSR arrays without any allocation:
// the entry point for callers that cannot allocate device memory (code under
// HIP graph capture, tight serving loops, harnesses that forbid hipMalloc).
//
// The sweep is the fused greedy step of mdp_bellman (Q = g + gamma P v, the
// lowest action attaining the minimum, max |Tv - v|), run on rows in the
// caller's natural order r = s*A + a.  Its per-workgroup partials live in one
// file-scope device array, `scratch`, instead of in a handle's memory.  Each
// row is summed by the same lane mapping as in a handle's sweep (lane l of the
// row's L lanes takes entries l, l+L, ...; the partial sums meet in the same
// butterfly), so with the same lanes per row both give bitwise the same Tv,
// policy and residual.
#include <cstring>
#include <mutex>
#include <string>
#include <vector>

#include "device.h"

namespace mdp {

namespace {

// Most sweep tiles one call may have: 2 MiB of per-tile partials (one double4
// each).  A tile holds sweep_tile_states(A) states, so this covers S*A up to
// 2^26 rows (64M, e.g. 4M states with 16 actions).
constexpr int kNoAllocMaxTiles = 65536;

// Per-workgroup partials of the last call on this GPU: (max|Tv - v|,
// sum (Tv - v)^2, max|Tv|, unused) for tile t at index t.  Every tile of a
// call writes its own entry before the reduction reads it, so nothing has to
// be cleared between calls.  Host code must not use this name as a device
// address: it takes the per-device address from hipGetSymbolAddress.
static __device__ __align__(256) double4 scratch[kNoAllocMaxTiles];

// Sweep tile over natural-order rows: stage the tile's int64 row offsets as
// int32 (nnz < 2^31), form Q(s, a) in LDS, then finish as every sweep does.
template <int L, int U>
__global__ __launch_bounds__(kBlock) void k_bellman_natural(
    int64_t S, int A, int tile_states, const int64_t* __restrict__ row_ptr,
    const int* __restrict__ col, const double* __restrict__ val, const double* __restrict__ cost,
    const double* __restrict__ v, double gamma, double* __restrict__ Tv, int* __restrict__ pi,
    double4* __restrict__ partials) {
  extern __shared__ double lds_d[];
  const int tile = xcd_tile(blockIdx.x, gridDim.x);
  const int tile_rows = tile_states * A;
  double* q = lds_d;
  int* rp = reinterpret_cast<int*>(lds_d + tile_rows);  // tile_rows + 1 entries
  const int64_t s0 = static_cast<int64_t>(tile) * tile_states;
  const int ns = static_cast<int>(min<int64_t>(tile_states, S - s0));
  const int nrows = ns * A;
  const int64_t row0 = s0 * A;
  for (int base = 0; base <= nrows; base += 4 * kBlock) {
    int buf[4];
#pragma unroll
    for (int k = 0; k < 4; ++k) {
      const int i = base + threadIdx.x + k * kBlock;
      buf[k] = static_cast<int>(row_ptr[row0 + (i <= nrows ? i : 0)]);
    }
#pragma unroll
    for (int k = 0; k < 4; ++k) {
      const int i = base + threadIdx.x + k * kBlock;
      if (i <= nrows) rp[i] = buf[k];
    }
  }
  __syncthreads();
  pipelined_rows<L, U, double, double, double, false, true, false>(
      nrows,
      [&](int idx, int& st, int& en, int& ri, int& si) {
        st = rp[idx];
        en = rp[idx + 1];
        ri = static_cast<int>(row0 + idx);
        si = -1;
      },
      col, val, v, S, cost, nullptr,
      [&](int idx, double pv, double gc, double) {
        // natural order: row idx of the tile is action idx % A of state idx / A
        if ((threadIdx.x % L) == 0) q[idx] = fma(gamma, pv, gc);
      });
  __syncthreads();
  sweep_finish<double, double, double>(s0, ns, A, q, v, Tv, pi, nullptr, partials, tile);
}

// max over the tiles' max|Tv - v| into *res (a single workgroup; max is exact,
// so the order does not matter).
__global__ __launch_bounds__(kBlock) void k_noalloc_res(const double4* __restrict__ partials, int nb,
                                                        double* __restrict__ res) {
  double mx = 0.0, unused = 0.0;
  for (int b = threadIdx.x; b < nb; b += kBlock) mx = max_nan(mx, partials[b].x);
  block_max_sum(mx, unused);
  if (threadIdx.x == 0) *res = mx;
}

std::mutex g_scratch_mu;
std::vector<void*> g_scratch_ptr;  // per device: address of `scratch` on that device

// The device address of `scratch` on the current device (looked up once per
// device, with that device current).
mdp_status scratch_address(int dev, double4** out) {
  std::lock_guard<std::mutex> lk(g_scratch_mu);
  if (g_scratch_ptr.size() <= static_cast<size_t>(dev)) g_scratch_ptr.resize(dev + 1, nullptr);
  if (!g_scratch_ptr[dev]) {
    void* p = nullptr;
    const hipError_t e = hipGetSymbolAddress(&p, HIP_SYMBOL(scratch));
    if (e != hipSuccess || !p) {
      (void)hipGetLastError();
      return fail(MDP_E_DEVICE, std::string("hipGetSymbolAddress of the sweep scratch failed: ") +
                                    hipGetErrorString(e));
    }
    g_scratch_ptr[dev] = p;
  }
  *out = static_cast<double4*>(g_scratch_ptr[dev]);
  return MDP_OK;
}

// p is device memory of device dev (hipPointerGetAttributes; no allocation).
bool on_device(const void* p, int dev) {
  hipPointerAttribute_t a;
  std::memset(&a, 0, sizeof(a));
  if (hipPointerGetAttributes(&a, p) != hipSuccess) {
    (void)hipGetLastError();
    return false;
  }
  return a.type == hipMemoryTypeDevice && a.device == dev;
}

template <typename F>
hipError_t with_lanes_na(int L, F&& f) {
  switch (L) {
    case 2: return f(std::integral_constant<int, 2>{});
    case 4: return f(std::integral_constant<int, 4>{});
    case 8: return f(std::integral_constant<int, 8>{});
    case 16: return f(std::integral_constant<int, 16>{});
    case 32: return f(std::integral_constant<int, 32>{});
    default: return f(std::integral_constant<int, 64>{});
  }
}

}  // namespace

}  // namespace mdp

extern "C" mdp_status mdp_bellman_noalloc(int64_t S, int32_t A, int64_t nnz, const int64_t* row_ptr,
                                          const int32_t* col, const double* val, const double* cost,
                                          double gamma, const double* v, double* Tv, int32_t* policy,
                                          double* res_inf, int32_t lanes_per_row, void* stream) {
  using namespace mdp;
  clear_error();
  if (S < 1 || A < 1) return fail(MDP_E_INVAL, "S and A must be at least 1");
  if (nnz < S * static_cast<int64_t>(A)) return fail(MDP_E_INVAL, "nnz must be at least S*A (no empty rows)");
  MDP_TRY(check_size_limits(S, A, nnz));
  if (!(gamma >= 0.0 && gamma < 1.0)) return fail(MDP_E_INVAL, "gamma must lie in [0,1)");
  if (lanes_per_row != 0 && (lanes_per_row < 2 || lanes_per_row > 64 || (lanes_per_row & (lanes_per_row - 1))))
    return fail(MDP_E_INVAL, "lanes_per_row must be 0 or a power of two in [2,64]");
  const int ts = sweep_tile_states(A);
  const int64_t nb = (S + ts - 1) / ts;
  if (nb > kNoAllocMaxTiles)
    return fail(MDP_E_NOTSUP, "the MDP needs " + std::to_string(nb) + " sweep tiles; the no-allocation sweep has scratch for " +
                                  std::to_string(kNoAllocMaxTiles) + " (S*A up to about 2^26 rows)");
  int dev = -1;
  MDP_HIP(hipGetDevice(&dev));
  if (!row_ptr || !col || !val || !cost || !v) return fail(MDP_E_INVAL, "row_ptr, col, val, cost and v must be non-NULL");
  const void* need[] = {row_ptr, col, val, cost, v};
  for (const void* p : need)
    if (!on_device(p, dev)) return fail(MDP_E_INVAL, "every array must be device memory of the current device");
  const void* opt_out[] = {Tv, policy, res_inf};
  for (const void* p : opt_out)
    if (p && !on_device(p, dev)) return fail(MDP_E_INVAL, "Tv, policy and res_inf must be NULL or device memory of the current device");
  if (Tv && static_cast<const void*>(Tv) == static_cast<const void*>(v)) return fail(MDP_E_INVAL, "Tv must not alias v");
  double4* part = nullptr;
  MDP_TRY(scratch_address(dev, &part));
  auto st = static_cast<hipStream_t>(stream);
  const int L = lanes_per_row ? lanes_per_row : default_lanes(static_cast<double>(nnz) / (S * static_cast<double>(A)));
  const size_t lds = static_cast<size_t>(ts) * A * sizeof(double) + (static_cast<size_t>(ts) * A + 1) * sizeof(int);
  const hipError_t e = with_lanes_na(L, [&](auto Lc) -> hipError_t {
    constexpr int LL = decltype(Lc)::value;
    constexpr int U = LL >= 32 ? 2 : MDP_UNROLL;
    k_bellman_natural<LL, U><<<static_cast<unsigned>(nb), kBlock, lds, st>>>(S, A, ts, row_ptr, col, val, cost, v,
                                                                            gamma, Tv, policy, part);
    return hipGetLastError();
  });
  if (e != hipSuccess) return fail(MDP_E_DEVICE, std::string("sweep launch failed: ") + hipGetErrorString(e));
  if (res_inf) {
    k_noalloc_res<<<1, kBlock, 0, st>>>(part, static_cast<int>(nb), res_inf);
    const hipError_t e2 = hipGetLastError();
    if (e2 != hipSuccess) return fail(MDP_E_DEVICE, std::string("reduction launch failed: ") + hipGetErrorString(e2));
  }
  return MDP_OK;
}
