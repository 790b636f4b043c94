// C-ABI entry points: validation, handle life cycle, and the host side of the
// inexact policy iteration (outer loop, inner-solver control, precision
// schedule).  The arithmetic itself runs in the kernels of kernels.hip.
#include <algorithm>
#include <chrono>
#include <cmath>
#include <cstring>
#include <limits>
#include <memory>
#include <mutex>
#include <new>
#include <thread>
#include <vector>

#include "batch.h"
#include "internal.h"

namespace mdp {

std::shared_mutex& alloc_lock() {
  static std::shared_mutex mu;
  return mu;
}

hipError_t lib_malloc(void** p, size_t bytes) {
  std::shared_lock<std::shared_mutex> g(alloc_lock());
  return hipMalloc(p, bytes);
}

void lib_free(void* p) {
  if (!p) return;
  std::shared_lock<std::shared_mutex> g(alloc_lock());
  (void)hipFree(p);
}

hipError_t lib_host_malloc(void** p, size_t bytes) {
  std::shared_lock<std::shared_mutex> g(alloc_lock());
  return hipHostMalloc(p, bytes, hipHostMallocDefault);
}

void lib_host_free(void* p) {
  if (!p) return;
  std::shared_lock<std::shared_mutex> g(alloc_lock());
  (void)hipHostFree(p);
}

// Device memory of handles, and staging memory at create time, come from the
// handle's arena when it has one (arena.cpp; servers admit into one), else
// from a stream-ordered pool that the library creates once per device and
// keeps until the process ends.  hipFree waits for the whole device, so a
// solve ending beside others would wait for them; the pool frees in stream
// order.  (The runtime's pool hands most freed memory back at the next
// synchronisation, whatever its release threshold, so a handle created after
// others were destroyed usually takes fresh memory from the device.)
constexpr uint64_t kPoolKeepBytes = uint64_t{2} << 30;

namespace {
struct DevicePool {
  hipMemPool_t pool = nullptr;
};
std::mutex g_pool_mu;
std::vector<DevicePool> g_pools;

hipError_t pool_locked(int dev, DevicePool** out) {
  if (dev < 0) return hipErrorInvalidDevice;
  if (g_pools.size() <= static_cast<size_t>(dev)) g_pools.resize(dev + 1);
  DevicePool& d = g_pools[dev];
  if (!d.pool) {
    hipMemPoolProps props;
    std::memset(&props, 0, sizeof(props));
    props.allocType = hipMemAllocationTypePinned;
    props.handleTypes = hipMemHandleTypeNone;
    props.location.type = hipMemLocationTypeDevice;
    props.location.id = dev;
    hipMemPool_t p = nullptr;
    hipError_t e = hipMemPoolCreate(&p, &props);
    if (e != hipSuccess) return e;
    uint64_t keep = kPoolKeepBytes;
    e = hipMemPoolSetAttribute(p, hipMemPoolAttrReleaseThreshold, &keep);
    if (e != hipSuccess) {
      (void)hipMemPoolDestroy(p);
      return e;
    }
    d.pool = p;
  }
  *out = &d;
  return hipSuccess;
}
}  // namespace

hipError_t device_pool(int dev, hipMemPool_t* out) {
  std::lock_guard<std::mutex> lk(g_pool_mu);
  DevicePool* d = nullptr;
  hipError_t e = pool_locked(dev, &d);
  if (e == hipSuccess) *out = d->pool;
  return e;
}

hipError_t handle_alloc(mdp_handle* h, void** p, size_t bytes) {
  if (h->dev_arena) {
    *p = h->dev_arena->alloc(bytes);
    if (*p) return hipSuccess;  // arena ranges are 256-byte aligned
  }
  hipMemPool_t pool = nullptr;
  hipError_t e = device_pool(h->device, &pool);
  if (e != hipSuccess) return e;
  {
    std::shared_lock<std::shared_mutex> g(alloc_lock());
    e = hipMallocFromPoolAsync(p, std::max<size_t>(bytes, 1), pool, h->stream);
  }
  // after this, the memory may be used from any stream
  if (e == hipSuccess) e = hipStreamSynchronize(h->stream);
  if (e == hipSuccess && (reinterpret_cast<uintptr_t>(*p) & 255) != 0) {
    handle_free(h, *p);
    *p = nullptr;
    e = hipErrorInvalidValue;  // the kernels assume 256-byte aligned arrays
  }
  return e;
}

void handle_free(mdp_handle* h, void* p) {
  if (!p) return;
  if (DeviceArena* a = arena_of(p)) {
    a->free(p, h->destroying ? nullptr : h->stream);
    return;
  }
  std::shared_lock<std::shared_mutex> g(alloc_lock());
  (void)hipFreeAsync(p, h->stream);
}

// Streams of handles are recycled per device, and the pinned host mirrors of
// their control blocks come from slabs kept until the process ends: stream
// creation and destruction cost a few hundred microseconds each, and
// hipHostFree waits for the device, which would hold a server's retirement
// behind the solves running beside it.
constexpr size_t kMaxCachedStreams = 64;
constexpr int kCtlSlab = 256;

namespace {
std::mutex g_recycle_mu;
std::vector<std::vector<hipStream_t>> g_streams;
std::vector<Ctl*> g_ctl_free;
}  // namespace

hipError_t stream_take(int dev, hipStream_t* out) {
  {
    std::lock_guard<std::mutex> lk(g_recycle_mu);
    if (dev >= 0 && static_cast<size_t>(dev) < g_streams.size() && !g_streams[dev].empty()) {
      *out = g_streams[dev].back();
      g_streams[dev].pop_back();
      return hipSuccess;
    }
  }
  std::shared_lock<std::shared_mutex> g(alloc_lock());
  return hipStreamCreateWithFlags(out, hipStreamNonBlocking);
}

void stream_give(int dev, hipStream_t st) {
  {
    std::lock_guard<std::mutex> lk(g_recycle_mu);
    if (dev >= 0) {
      if (g_streams.size() <= static_cast<size_t>(dev)) g_streams.resize(dev + 1);
      if (g_streams[dev].size() < kMaxCachedStreams) {
        g_streams[dev].push_back(st);
        return;
      }
    }
  }
  std::shared_lock<std::shared_mutex> g(alloc_lock());
  (void)hipStreamDestroy(st);
}

Ctl* ctl_slot_take() {
  std::lock_guard<std::mutex> lk(g_recycle_mu);
  if (g_ctl_free.empty()) {
    void* slab = nullptr;
    if (lib_host_malloc(&slab, sizeof(Ctl) * kCtlSlab) != hipSuccess) return nullptr;
    for (int i = kCtlSlab - 1; i >= 0; --i) g_ctl_free.push_back(static_cast<Ctl*>(slab) + i);
  }
  Ctl* c = g_ctl_free.back();
  g_ctl_free.pop_back();
  return c;
}

void ctl_slot_give(Ctl* c) {
  if (!c) return;
  std::lock_guard<std::mutex> lk(g_recycle_mu);
  g_ctl_free.push_back(c);
}

// Lanes per CSR row when neither the caller nor the autotuner's cache gives a
// width: the smallest power of two in [2, 64] that covers the mean row length.
int default_lanes(double mean_row) {
  int L = 2;
  while (L < 64 && L < mean_row) L <<= 1;
  return L;
}

// Engines of mdp_solve_batch are kept per device between calls, so that the
// HIP graphs they capture are replayed by later calls of the same
// configuration.  A call leases an idle engine (or makes one) and hands it
// back; concurrent calls lease different engines.  Engines stay until the
// process ends; each holds its work tables and at most 64 graph sets.
namespace {
std::mutex g_engine_mu;
std::vector<std::vector<std::unique_ptr<BatchEngine>>> g_engines;
}  // namespace

EngineLease::EngineLease(int dev) : dev(dev) {
  std::lock_guard<std::mutex> lk(g_engine_mu);
  if (dev >= 0 && static_cast<size_t>(dev) < g_engines.size() && !g_engines[dev].empty()) {
    eng = g_engines[dev].back().release();
    g_engines[dev].pop_back();
  } else {
    eng = new (std::nothrow) BatchEngine();
  }
}

EngineLease::~EngineLease() {
  if (!eng) return;
  eng->items.clear();
  std::lock_guard<std::mutex> lk(g_engine_mu);
  if (dev < 0) {
    delete eng;
    return;
  }
  if (g_engines.size() <= static_cast<size_t>(dev)) g_engines.resize(dev + 1);
  g_engines[dev].emplace_back(eng);
}

namespace {
thread_local std::string g_err;

struct BusyGuard {
  mdp_handle* h;
  bool ok;
  explicit BusyGuard(mdp_handle* hh) : h(hh) {
    int expect = 0;
    ok = h->busy.compare_exchange_strong(expect, 1);
  }
  ~BusyGuard() {
    if (ok) h->busy.store(0);
  }
};

double now_ms() {
  using namespace std::chrono;
  return duration<double, std::milli>(steady_clock::now().time_since_epoch()).count();
}

template <typename T>
hipError_t dev_alloc(mdp_handle* h, T** p, size_t n) {
  const size_t bytes = std::max<size_t>(1, n) * sizeof(T);
  hipError_t e = handle_alloc(h, reinterpret_cast<void**>(p), bytes);
  if (e == hipSuccess) h->device_bytes += static_cast<int64_t>(bytes);
  return e;
}

template <typename T>
void dev_free(mdp_handle* h, T*& p) {
  handle_free(h, p);
  p = nullptr;
}

hipError_t staging_alloc(int dev, hipStream_t st, size_t bytes, char** out) {
  if (DeviceArena* a = current_arena(); a && a->device() == dev) {
    *out = static_cast<char*>(a->alloc(bytes));
    if (*out) return hipSuccess;
  }
  hipMemPool_t pool = nullptr;
  hipError_t e = device_pool(dev, &pool);
  if (e != hipSuccess) return e;
  std::shared_lock<std::shared_mutex> g(alloc_lock());
  return hipMallocFromPoolAsync(reinterpret_cast<void**>(out), std::max<size_t>(bytes, 1), pool, st);
}

hipError_t staging_free(char* p, hipStream_t st) {
  if (DeviceArena* a = arena_of(p)) {
    a->free(p, st);
    return hipSuccess;
  }
  std::shared_lock<std::shared_mutex> g(alloc_lock());
  return hipFreeAsync(p, st);
}

}  // namespace

namespace {
std::mutex g_stage_mu;
std::vector<StageBlock> g_stage_free;
}  // namespace

bool stage_take(StageBlock* b) {
  {
    std::lock_guard<std::mutex> lk(g_stage_mu);
    if (!g_stage_free.empty()) {
      *b = g_stage_free.back();
      g_stage_free.pop_back();
      return true;
    }
  }
  StageBlock n;
  void* p = nullptr;
  if (lib_host_malloc(&p, kStageBlockBytes) != hipSuccess) return false;
  hipError_t e;
  {
    std::shared_lock<std::shared_mutex> g(alloc_lock());
    e = hipEventCreateWithFlags(&n.ev, hipEventDisableTiming);
  }
  if (e != hipSuccess) {
    lib_host_free(p);
    return false;
  }
  n.p = static_cast<char*>(p);
  *b = n;
  return true;
}

void stage_give(const StageBlock& b) {
  if (!b.p) return;
  std::lock_guard<std::mutex> lk(g_stage_mu);
  g_stage_free.push_back(b);
}

bool host_pageable(const void* p) {
  if (!p) return false;
  hipPointerAttribute_t a;
  std::memset(&a, 0, sizeof(a));
  if (hipPointerGetAttributes(&a, p) != hipSuccess) {
    (void)hipGetLastError();
    return true;
  }
  return a.type == hipMemoryTypeUnregistered;
}

namespace {
// Two blocks per staged copy, so that the host side of one chunk overlaps the
// transfer of the other; handed back once the stream has drained them.
struct StagePair {
  StageBlock b[2];
  bool ok = false;
  StagePair() {
    ok = stage_take(&b[0]);
    if (ok && !stage_take(&b[1])) {
      stage_give(b[0]);
      b[0] = StageBlock();
      ok = false;
    }
  }
  ~StagePair() {
    stage_give(b[0]);
    stage_give(b[1]);
  }
};
}  // namespace

hipError_t copy_in(void* dst, const void* src, size_t bytes, hipStream_t st) {
  if (bytes == 0) return hipSuccess;
  if (!host_pageable(src)) return hipMemcpyAsync(dst, src, bytes, hipMemcpyDefault, st);
  if (host_pageable(dst)) {  // host to host
    std::memcpy(dst, src, bytes);
    return hipSuccess;
  }
  StagePair sp;
  if (!sp.ok) return hipErrorOutOfMemory;
  hipError_t e = hipSuccess;
  bool used[2] = {false, false};
  int k = 0;
  for (size_t off = 0; off < bytes && e == hipSuccess; off += kStageBlockBytes, k ^= 1) {
    const size_t c = std::min(kStageBlockBytes, bytes - off);
    if (used[k]) e = hipEventSynchronize(sp.b[k].ev);  // the block's previous chunk has left
    if (e != hipSuccess) break;
    std::memcpy(sp.b[k].p, static_cast<const char*>(src) + off, c);
    e = hipMemcpyAsync(static_cast<char*>(dst) + off, sp.b[k].p, c, hipMemcpyDefault, st);
    if (e == hipSuccess) e = hipEventRecord(sp.b[k].ev, st);
    used[k] = true;
  }
  const hipError_t es = hipStreamSynchronize(st);  // the blocks go back idle
  return e != hipSuccess ? e : es;
}

hipError_t copy_out(void* dst, const void* src, size_t bytes, hipStream_t st) {
  if (bytes == 0) return hipSuccess;
  if (!host_pageable(dst)) return hipMemcpyAsync(dst, src, bytes, hipMemcpyDefault, st);
  if (host_pageable(src)) {  // host to host
    std::memcpy(dst, src, bytes);
    return hipSuccess;
  }
  StagePair sp;
  if (!sp.ok) return hipErrorOutOfMemory;
  hipError_t e = hipSuccess;
  size_t prev_off = 0, prev_c = 0;
  bool pending = false;
  int k = 0;
  // chunk i goes into block k while chunk i-1 leaves block k^1 for dst
  for (size_t off = 0; off < bytes && e == hipSuccess; off += kStageBlockBytes, k ^= 1) {
    const size_t c = std::min(kStageBlockBytes, bytes - off);
    e = hipMemcpyAsync(sp.b[k].p, static_cast<const char*>(src) + off, c, hipMemcpyDefault, st);
    if (e == hipSuccess) e = hipEventRecord(sp.b[k].ev, st);
    if (e == hipSuccess && pending) {
      e = hipEventSynchronize(sp.b[k ^ 1].ev);
      if (e == hipSuccess) std::memcpy(static_cast<char*>(dst) + prev_off, sp.b[k ^ 1].p, prev_c);
    }
    pending = e == hipSuccess;
    prev_off = off;
    prev_c = c;
  }
  if (e == hipSuccess && pending) {
    e = hipEventSynchronize(sp.b[k ^ 1].ev);
    if (e == hipSuccess) std::memcpy(static_cast<char*>(dst) + prev_off, sp.b[k ^ 1].p, prev_c);
  }
  const hipError_t es = hipStreamSynchronize(st);
  return e != hipSuccess ? e : es;
}

namespace {

// Copy a caller policy to device memory and check its range.
mdp_status load_policy(mdp_handle* h, const int32_t* policy, int32_t* dst) {
  if (!policy) return fail(MDP_E_INVAL, "policy is NULL");
  ++h->pi_gen;  // a policy is written
  if (!is_device_ptr(policy)) {
    for (int64_t s = 0; s < h->S; ++s)
      if (policy[s] < 0 || policy[s] >= h->A)
        return fail(MDP_E_INVAL, "policy entry outside [0,A) at state " + std::to_string(s));
    MDP_HIP(copy_in(dst, policy, h->S * sizeof(int32_t), h->stream));
    return MDP_OK;
  }
  MDP_HIP(hipMemcpyAsync(dst, policy, h->S * sizeof(int32_t), hipMemcpyDeviceToDevice, h->stream));
  MDP_HIP(launch_ctl_reset(h, 0.0));
  MDP_HIP(launch_check_policy(h, dst));
  MDP_TRY(sync_ctl(h));
  if (h->ctl_host->bad_policy)
    return fail(MDP_E_INVAL, std::to_string(h->ctl_host->bad_policy) + " policy entries outside [0,A)");
  return MDP_OK;
}

mdp_status load_vec(mdp_handle* h, const double* src, double* dst) {
  if (src) {
    MDP_HIP(copy_in(dst, src, h->S * sizeof(double), h->stream));
    if (h->maximize) MDP_HIP(launch_negate(h->stream, dst, h->S));
  } else {
    MDP_HIP(hipMemsetAsync(dst, 0, h->S * sizeof(double), h->stream));
  }
  return MDP_OK;
}

mdp_status store(mdp_handle* h, void* dst, const void* src, size_t bytes) {
  if (dst && dst != src) MDP_HIP(copy_out(dst, src, bytes, h->stream));
  return MDP_OK;
}

// Copy a value vector out; src is device scratch of the handle and is turned
// into reward terms in place first when the handle maximises.
mdp_status store_values(mdp_handle* h, double* dst, double* src) {
  if (h->maximize) MDP_HIP(launch_negate(h->stream, src, h->S));
  return store(h, dst, src, h->S * sizeof(double));
}

struct InnerResult {
  int64_t steps = 0;
  int64_t applies = 0;
  int64_t refinements = 0;
  double bytes = 0;
  double orth_loss = 0;
  bool converged = false;
};

// Float64 and float32 products of an inner solve on a large handle use the
// copy of P_pi for its policy (formed at the first inner solve of the
// policy, kept for the next), cut by XCD when the handle carries a
// column-blocked copy, else contiguous when its rows are short.  The scope
// takes the copy out of the products when the inner solve ends.
struct PolicyCopyScope {
  mdp_handle* h;
  ~PolicyCopyScope() { h->pp_ready = false; }
};
hipError_t policy_copy_begin(mdp_handle* h, const int32_t* pi, int policy_copy) {
  const bool short_rows = h->S >= kPolicyCopyMinStates && h->nnz <= kPolicyCopyMaxRowMean * h->rows;
  if (policy_copy != 0 && (h->cb_blocks > 0 || short_rows)) return pp_prepare(h, pi);
  return hipSuccess;
}

// GMRES(m) on (I - gamma P_pi) x = g_pi.  On entry basis slot 0 holds the
// residual of x and ctl holds a started cycle (kRedGmresStart).  Arnoldi steps
// run in `prec`; every restart recomputes the residual in float64 from the
// float64 P, so the mixed-precision variants are iterative refinement.
mdp_status gmres_inner(mdp_handle* h, Prec prec, const int32_t* pi, double* x, int m,
                       int64_t max_iter, int sync_every, double alpha, InnerResult* out, int deg = 1,
                       bool gs2 = false, int policy_copy = -1) {
  const Prec bprec = prec == kF64 ? kF64 : kF32;
  const int bb = bprec == kF64 ? 8 : 4;
  PolicyCopyScope pp_scope{h};
  if (prec == kF64 || prec == kF32) MDP_HIP(policy_copy_begin(h, pi, policy_copy));
  for (;;) {
    int j = 0;
    const size_t rec0 = h->prof_pending.size();
    MDP_TRY(sync_ctl(h));
    // Steps are enqueued in chunks between host checks.  After the first
    // chunk the chunk length follows the observed contraction of the
    // residual estimate, so that few steps are enqueued past the end of the
    // cycle (they exit at once, but each still costs a launch).
    //
    // While the host reads a snapshot of the control header, one more step is
    // already queued behind it, so the device does not idle during the host's
    // round trip; a step queued past the end of the cycle exits at once and
    // leaves the control block unchanged.
    int chunk = sync_every;
    int j_prev = 0;
    double est_prev = h->ctl_host->beta;
    bool stale = false;  // steps were queued after the last snapshot
    while (!h->ctl_host->done && j < m) {
      for (int b = 0; b < chunk && j < m; ++b, ++j) {
        MDP_HIP(launch_arnoldi_step(h, prec, pi, j, m, deg, gs2));
      }
      const int j_snap = j;
      MDP_TRY(ctl_snapshot(h));
      if (j < m) {
        MDP_HIP(launch_arnoldi_step(h, prec, pi, j, m, deg, gs2));
        ++j;
      }
      stale = j > j_snap;
      MDP_TRY(ctl_wait(h));
      const double est = h->ctl_host->res_est, goal = h->ctl_host->tol_cycle;
      chunk = sync_every;
      if (j_snap > j_prev && est > 0.0 && est < est_prev && goal > 0.0) {
        const double rate = std::pow(est / est_prev, 1.0 / (j_snap - j_prev));
        if (rate < 1.0) {
          const double need = std::ceil(std::log(goal / est) / std::log(rate)) - (j - j_snap);
          chunk = static_cast<int>(std::min(16.0, std::max(1.0, need)));
        }
      }
      j_prev = j_snap;
      est_prev = est;
    }
    // the header is final unless the last snapshot missed queued steps that did work
    if (stale && !h->ctl_host->done) MDP_TRY(sync_ctl(h));
    const int done_j = h->ctl_host->j;
    prof_discard_steps(h, rec0, done_j);
    // a preconditioned step also makes deg - 1 Horner products (y = b + gamma P_pi x)
    const double horner_bytes = bytes_apply(h, bval_of(prec), bb, bb) + h->S * (double)bb;
    for (int jj = 0; jj < done_j; ++jj)
      out->bytes += bytes_arnoldi_apply(h, bval_of(prec), bb, jj) + bytes_arnoldi_update(h, bb, jj) +
                    (deg - 1) * horner_bytes;
    out->applies += static_cast<int64_t>(done_j) * deg;
    if (done_j > 0) {
      if (deg > 1) {
        MDP_HIP(launch_precond_update_x(h, prec, pi, x, m, deg));
        out->applies += deg - 1;
        out->bytes += h->S * (16.0 + done_j * (double)bb) + (deg - 1) * horner_bytes;
      } else {
        MDP_HIP(launch_gmres_update_x(h, bprec, x));
        out->bytes += h->S * (16.0 + done_j * (double)bb);
      }
    }
    out->steps = h->ctl_host->steps;
    out->orth_loss = std::max(out->orth_loss, h->ctl_host->orth_loss);
    if (gs2)  // the second pass reads the basis and the new vector once more and updates again
      for (int jj = 0; jj < done_j; ++jj) out->bytes += h->S * (jj + 2.0) * bb + bytes_arnoldi_update(h, bb, jj);
    const double est = h->ctl_host->res_est;
    if (!std::isfinite(est)) return fail(MDP_E_NUMERIC, "non-finite GMRES residual");
    if (h->ctl_host->converged && prec == kF64) {
      out->converged = true;
      return MDP_OK;
    }
    if (out->steps >= max_iter) return MDP_OK;
    // restart: true residual in float64 into basis slot 0, next cycle
    void* slot0 = bprec == kF64 ? static_cast<void*>(h->U64) : static_cast<void*>(h->U32);
    MDP_HIP(launch_apply(h, kApplyRes, pi, x, slot0, bprec != kF64, kRedGmresStart, 0, alpha,
                         floor_of(prec)));
    out->applies += 1;
    out->refinements += prec == kF64 ? 0 : 1;
    out->bytes += bytes_apply(h, 8, 8, bb);
    MDP_TRY(sync_ctl(h));
    if (!std::isfinite(h->ctl_host->beta)) return fail(MDP_E_NUMERIC, "non-finite residual");
    if (h->ctl_host->converged) {
      out->converged = true;
      return MDP_OK;
    }
    if (done_j == 0 && h->ctl_host->done) {
      // the residual cannot be reduced further in this arithmetic
      return MDP_OK;
    }
  }
}

// Richardson x <- g_pi + gamma P_pi x on the pair (buf0, buf1), starting from
// ctl->rich_cur; stops at ctl->tol or after max_iter total steps.  Returns the
// buffer holding the last iterate.
mdp_status richardson_inner(mdp_handle* h, const int32_t* pi, double* buf0, double* buf1,
                            int64_t max_iter, int sync_every, InnerResult* out, double** last) {
  MDP_TRY(sync_ctl(h));
  while (!h->ctl_host->done && h->ctl_host->steps < max_iter) {
    const int64_t left = max_iter - h->ctl_host->steps;
    const int64_t n = std::min<int64_t>(sync_every, left);
    for (int64_t i = 0; i < n; ++i) MDP_HIP(launch_richardson_step(h, pi, buf0, buf1));
    MDP_TRY(sync_ctl(h));
    if (!std::isfinite(h->ctl_host->res_est)) return fail(MDP_E_NUMERIC, "non-finite Richardson difference");
  }
  out->steps = h->ctl_host->steps;
  out->applies = out->steps;
  out->bytes += out->steps * bytes_apply(h, 8, 8, 8);
  out->converged = h->ctl_host->converged != 0;
  *last = h->ctl_host->rich_cur ? buf1 : buf0;
  return MDP_OK;
}

// BiCGSTAB (or TFQMR) from x (residual r0 in basis slot 0, its norm and the
// tolerance in ctl); stops at ctl->tol, at a breakdown, or after max_iter
// iterations.
mdp_status bicgstab_inner(mdp_handle* h, const int32_t* pi, double* x, int64_t max_iter,
                          int sync_every, InnerResult* out, bool tfqmr = false, int policy_copy = -1) {
  PolicyCopyScope pp_scope{h};
  MDP_HIP(policy_copy_begin(h, pi, policy_copy));
  if (tfqmr)
    MDP_HIP(launch_tfqmr_init(h, pi));
  else
    MDP_HIP(launch_bicgstab_init(h));
  MDP_TRY(sync_ctl(h));
  int64_t launched = 0;
  while (!h->ctl_host->done && launched < max_iter) {
    const int64_t n = std::min<int64_t>(sync_every, max_iter - launched);
    for (int64_t i = 0; i < n; ++i) {
      if (tfqmr)
        MDP_HIP(launch_tfqmr_step(h, pi, x));
      else
        MDP_HIP(launch_bicgstab_step(h, pi, x));
    }
    launched += n;
    MDP_TRY(sync_ctl(h));
    if (!std::isfinite(h->ctl_host->res_est)) return fail(MDP_E_NUMERIC, "non-finite Krylov residual");
  }
  out->steps = h->ctl_host->steps;
  out->applies += 2 * out->steps;
  // two products, two dot passes (2 and 4 vectors), s (3), x/r (7 vectors), p (4)
  out->bytes += out->steps * (2.0 * bytes_apply(h, 8, 8, 8) + 20.0 * h->S * 8.0);
  out->converged = h->ctl_host->converged != 0;
  return MDP_OK;
}

void stats_begin(mdp_stats* st) {
  if (!st) return;
  double* hist = st->history;
  int64_t cap = st->history_cap;
  size_t sz = st->struct_size;
  std::memset(st, 0, std::min(sz, sizeof(mdp_stats)));
  st->struct_size = sz;
  st->history = hist;
  st->history_cap = cap;
}

bool stats_ok(const mdp_stats* st) { return !st || st->struct_size >= sizeof(mdp_stats); }

}  // namespace

// ---- validation -------------------------------------------------------------
mdp_status check_size_limits(int64_t S, int32_t A, int64_t nnz) {
  if (A > 4096) return fail(MDP_E_NOTSUP, "A above 4096 is not supported");
  if (S * static_cast<int64_t>(A) >= (int64_t{1} << 31) - 1)
    return fail(MDP_E_NOTSUP, "S*A must be below 2^31");
  if (S > kMaxStates) return fail(MDP_E_NOTSUP, "S must be below 2^29");
  if (nnz > kMaxNnz) return fail(MDP_E_NOTSUP, "nnz must be at most 2^31 - 4096");
  return MDP_OK;
}

// Structure of row_ptr; checked in every mode, since kernels index rows by it.
mdp_status validate_row_ptr(int64_t S, int32_t A, const int64_t* rp) {
  const int64_t rows = S * A;
  if (rp[0] != 0) return fail(MDP_E_INVAL, "row_ptr[0] must be 0");
  for (int64_t r = 0; r < rows; ++r)
    if (rp[r + 1] <= rp[r])
      return fail(MDP_E_INVAL, "row_ptr must increase (row " + std::to_string(r) +
                                   " of state " + std::to_string(r / A) + " is empty or decreasing)");
  return check_size_limits(S, A, rp[rows]);
}

// The first failure of the entry checks, as a message; shared by the host and
// device checks so that both report alike.  why: 1 column, 2 probability, 3 sum.
mdp_status entry_failure(int64_t cost_row, int64_t entry_row, int why) {
  if (cost_row >= 0) return fail(MDP_E_INVAL, "non-finite cost at row " + std::to_string(cost_row));
  const char* w = why == 1 ? "column index outside [0,S)"
                  : why == 2 ? "negative or non-finite probability"
                             : "row does not sum to 1";
  return fail(MDP_E_INVAL, std::string(w) + " in row " + std::to_string(entry_row));
}

// Entries and costs on host arrays (row_ptr already checked).
mdp_status validate_entries_host(int64_t S, int32_t A, const int64_t* rp, const int32_t* col,
                                 const double* val, const double* cost) {
  const int64_t rows = S * A;
  for (int64_t r = 0; r < rows; ++r)
    if (!std::isfinite(cost[r])) return entry_failure(r, -1, 0);
  const unsigned nt = std::max(1u, std::min(16u, std::thread::hardware_concurrency()));
  std::vector<int64_t> bad(nt, -1);
  std::vector<int> why(nt, 0);
  std::vector<std::thread> th;
  for (unsigned t = 0; t < nt; ++t) {
    th.emplace_back([&, t]() {
      const int64_t r0 = rows * t / nt, r1 = rows * (t + 1) / nt;
      for (int64_t r = r0; r < r1; ++r) {
        // the library's row-sum order: eight interleaved partials, combined
        // as ((p0+p4)+(p2+p6)) + ((p1+p5)+(p3+p7)), as the device check does
        double p[8] = {0.0, 0.0, 0.0, 0.0, 0.0, 0.0, 0.0, 0.0};
        for (int64_t e = rp[r]; e < rp[r + 1]; ++e) {
          if (col[e] < 0 || col[e] >= S) { bad[t] = r; why[t] = 1; return; }
          if (!(val[e] >= 0.0) || !std::isfinite(val[e])) { bad[t] = r; why[t] = 2; return; }
          p[(e - rp[r]) % 8] += val[e];
        }
        const double sum = ((p[0] + p[4]) + (p[2] + p[6])) + ((p[1] + p[5]) + (p[3] + p[7]));
        const double len = static_cast<double>(rp[r + 1] - rp[r]);
        if (std::fabs(sum - 1.0) > 1e-12 * std::max(1.0, len)) { bad[t] = r; why[t] = 3; return; }
      }
    });
  }
  for (auto& x : th) x.join();
  for (unsigned t = 0; t < nt; ++t)
    if (bad[t] >= 0) return entry_failure(-1, bad[t], why[t]);
  return MDP_OK;
}

mdp_status validate_host(int64_t S, int32_t A, const int64_t* rp, const int32_t* col,
                         const double* val, const double* cost) {
  MDP_TRY(validate_row_ptr(S, A, rp));
  return validate_entries_host(S, A, rp, col, val, cost);
}

bool is_device_ptr(const void* p) {
  if (!p) return false;
  hipPointerAttribute_t a;
  std::memset(&a, 0, sizeof(a));
  if (hipPointerGetAttributes(&a, p) != hipSuccess) {
    (void)hipGetLastError();
    return false;
  }
  return a.type == hipMemoryTypeDevice;
}

mdp_status sync_ctl(mdp_handle* h) {
  MDP_HIP(hipMemcpyAsync(h->ctl_host, h->ctl, kCtlHeaderBytes, hipMemcpyDeviceToHost, h->stream));
  MDP_HIP(hipStreamSynchronize(h->stream));
  return MDP_OK;
}

mdp_status ctl_snapshot(mdp_handle* h) {
  MDP_HIP(hipMemcpyAsync(h->ctl_host, h->ctl, kCtlHeaderBytes, hipMemcpyDeviceToHost, h->stream));
  MDP_HIP(hipEventRecord(h->ctl_event, h->stream));
  return MDP_OK;
}

mdp_status ctl_wait(mdp_handle* h) {
  MDP_HIP(hipEventSynchronize(h->ctl_event));
  return MDP_OK;
}

mdp_status ensure_basis(mdp_handle* h, Prec prec, int m) {
  if (prec == kF64) {
    if (h->basis_m64 >= m) return MDP_OK;
    dev_free(h, h->U64);
    MDP_HIP(dev_alloc(h, &h->U64, static_cast<size_t>(m + 1) * h->ldu));
    h->basis_m64 = m;
  } else {
    if (h->basis_m32 >= m) return MDP_OK;
    dev_free(h, h->U32);
    MDP_HIP(dev_alloc(h, &h->U32, static_cast<size_t>(m + 1) * h->ldu));
    h->basis_m32 = m;
  }
  return MDP_OK;
}

mdp_status ensure_lowp(mdp_handle* h, Prec prec) {
  if (prec == kF32 && !h->cv32) {
    MDP_HIP(dev_alloc(h, &h->cv32, 2 * h->nnz));
    MDP_HIP(launch_build_lowp(h, MDP_BUILD_FP32));
  }
  if (prec == kF16 && !h->val16) {
    MDP_HIP(dev_alloc(h, &h->val16, h->nnz));
    MDP_HIP(dev_alloc(h, &h->corr16, h->rows));
    MDP_HIP(launch_build_lowp(h, MDP_BUILD_FP16));
  }
  if (prec != kF64 && !h->v32) MDP_HIP(dev_alloc(h, &h->v32, h->S));
  return MDP_OK;
}

Prec prec_of(int p) { return p == MDP_MIXED_FP16 ? kF16 : (p == MDP_MIXED_FP32 ? kF32 : kF64); }
int bval_of(Prec p) { return p == kF64 ? 8 : (p == kF32 ? 4 : 2); }
double floor_of(Prec p) { return p == kF64 ? 0.0 : (p == kF32 ? 1e-6 : 1e-3); }

double bytes_sweep(const mdp_handle* h, int bval, int bv, bool r0, int br) {
  // CSR values + columns, row offsets, costs, v gathered (counted once), Tv and pi out
  return static_cast<double>(h->nnz) * (bval + 4) + (h->rows + 1) * 4.0 + h->rows * 8.0 +
         h->S * static_cast<double>(bv) + h->S * 12.0 + (r0 ? h->S * static_cast<double>(br) : 0.0);
}
double bytes_apply(const mdp_handle* h, int bval, int bx, int by) {
  // selected rows (values + columns), pi, two row offsets, g_pi, x (once), y
  const double nnz_pi = static_cast<double>(h->nnz) / h->rows * h->S;
  return nnz_pi * (bval + 4) + h->S * (4.0 + 8.0 + 8.0 + bx + by);
}
double bytes_arnoldi_apply(const mdp_handle* h, int bval, int bb, int j) {
  // product (x read once, w written) + one pass over U_0..U_j for the dots
  const double nnz_pi = static_cast<double>(h->nnz) / h->rows * h->S;
  return nnz_pi * (bval + 4) + h->S * (4.0 + 8.0 + 2.0 * bb) + h->S * static_cast<double>(bb) * (j + 1);
}
double bytes_arnoldi_update(const mdp_handle* h, int bb, int j) {
  // U_0..U_j read, w read and written
  return h->S * static_cast<double>(bb) * (j + 3);
}

void prof_begin(mdp_handle* h, int kind, hipEvent_t* a) {
  *a = nullptr;
  if (!(h->prof_mask & (1 << kind))) return;
  if (h->prof_seen[kind]++ % h->prof_every != 0) return;
  if (h->prof_pool.empty()) {
    hipEvent_t e;
    if (hipEventCreate(&e) != hipSuccess) return;
    h->prof_pool.push_back(e);
  }
  *a = h->prof_pool.back();
  h->prof_pool.pop_back();
  (void)hipEventRecord(*a, h->stream);
}

void prof_end(mdp_handle* h, int kind, hipEvent_t a, double bytes, int tag) {
  if (!a) return;
  hipEvent_t b;
  if (h->prof_pool.empty()) {
    if (hipEventCreate(&b) != hipSuccess) return;
  } else {
    b = h->prof_pool.back();
    h->prof_pool.pop_back();
  }
  (void)hipEventRecord(b, h->stream);
  h->prof_pending.push_back({kind, tag, a, b, bytes});
  if (h->prof_pending.size() >= (size_t{1} << 20)) prof_resolve(h);
}

void prof_discard_steps(mdp_handle* h, size_t from, int min_tag) {
  if (from > h->prof_pending.size()) return;  // resolved in between: keep
  size_t w = from;
  for (size_t r = from; r < h->prof_pending.size(); ++r) {
    auto& rec = h->prof_pending[r];
    if (rec.tag >= 0 && rec.tag >= min_tag) {
      h->prof_pool.push_back(rec.a);
      h->prof_pool.push_back(rec.b);
    } else {
      h->prof_pending[w++] = rec;
    }
  }
  h->prof_pending.resize(w);
}

void prof_resolve(mdp_handle* h) {
  if (h->prof_pending.empty()) return;
  (void)hipEventSynchronize(h->prof_pending.back().b);
  for (auto& r : h->prof_pending) {
    float ms = 0.f;
    if (hipEventElapsedTime(&ms, r.a, r.b) == hipSuccess) {
      h->prof_ms[r.kind] += ms;
      h->prof_launches[r.kind] += 1;
      h->prof_bytes[r.kind] += r.bytes;
    }
    h->prof_pool.push_back(r.a);
    h->prof_pool.push_back(r.b);
  }
  h->prof_pending.clear();
}

mdp_status fail(mdp_status st, const std::string& msg) {
  g_err = msg;
  return st;
}
void clear_error() { g_err.clear(); }

}  // namespace mdp

using namespace mdp;

extern "C" {

const char* mdp_last_error(void) { return g_err.c_str(); }
const char* mdp_version(void) { return "mdp-mi355x 0.1 (gfx950)"; }

void mdp_default_create_opts(mdp_create_opts* o) {
  if (!o) return;
  std::memset(o, 0, sizeof(*o));
  o->struct_size = sizeof(*o);
  o->stream = nullptr;
  o->device = -1;
  o->validate = 1;
  o->low_precision = 0;
  o->lanes_per_row = 0;
  o->col_blocks = -1;
}

void mdp_default_eval_opts(mdp_eval_opts* o) {
  if (!o) return;
  std::memset(o, 0, sizeof(*o));
  o->struct_size = sizeof(*o);
  o->inner = MDP_INNER_GMRES;
  o->restart = 30;
  o->precision = MDP_FP64;
  o->sync_every = 0;
  o->rtol = 1e-10;
  o->max_iter = 10000;
  o->precond_degree = 1;
  o->gs_passes = 1;
  o->policy_copy = -1;
}

void mdp_default_solve_opts(mdp_solve_opts* o) {
  if (!o) return;
  std::memset(o, 0, sizeof(*o));
  o->struct_size = sizeof(*o);
  o->inner = MDP_INNER_GMRES;
  o->restart = 30;
  o->precision = MDP_FP64;
  o->sync_every = 0;
  o->alpha = 1e-4;
  o->atol = 1e-8;
  o->rtol_cert = 0.0;
  o->max_outer = 1000;
  o->max_inner = 10000;
  o->launch = MDP_LAUNCH_AUTO;
  o->precond_degree = 1;
  o->gs_passes = 1;
  o->policy_copy = -1;
}

mdp_status mdp_destroy(mdp_t h) {
  if (!h) return MDP_OK;
  if (h->stream) (void)hipStreamSynchronize(h->stream);
  h->destroying = true;
  if (h->arena) {  // the arrays inside it go with it
    dev_free(h, h->arena);
    h->row_ptr = h->col = nullptr;
    h->val = h->cost = h->v = h->Tv = h->x2 = h->io = nullptr;
    h->pi = h->pi_io = nullptr;
    h->part.buf = nullptr;
    h->ctl = nullptr;
  }
  dev_free(h, h->row_ptr);
  dev_free(h, h->col);
  dev_free(h, h->val);
  dev_free(h, h->cost);
  dev_free(h, h->cv32);
  dev_free(h, h->val16);
  dev_free(h, h->corr16);
  dev_free(h, h->cost32);
  dev_free(h, h->cb_col);
  dev_free(h, h->cb_val);
  dev_free(h, h->cb_rel);
  dev_free(h, h->cb_off);
  dev_free(h, h->cb_acc);
  dev_free(h, h->v);
  dev_free(h, h->Tv);
  dev_free(h, h->x2);
  dev_free(h, h->io);
  dev_free(h, h->pi);
  dev_free(h, h->pi_io);
  dev_free(h, h->v32);
  dev_free(h, h->x32a);
  dev_free(h, h->x32b);
  dev_free(h, h->U64);
  dev_free(h, h->U32);
  dev_free(h, h->part.buf);
  dev_free(h, h->ctl);
  pp_release(h);
  ctl_slot_give(h->ctl_host);
  prof_resolve(h);
  {
    std::shared_lock<std::shared_mutex> g(alloc_lock());
    if (h->ctl_event) (void)hipEventDestroy(h->ctl_event);
    for (auto e : h->prof_pool) (void)hipEventDestroy(e);
  }
  if (h->own_stream && h->stream) {
    // idle once the frees queued on it have run; the next handle may reuse it
    if (hipStreamSynchronize(h->stream) == hipSuccess) {
      stream_give(h->device, h->stream);
    } else {
      std::shared_lock<std::shared_mutex> g(alloc_lock());
      (void)hipStreamDestroy(h->stream);
    }
  }
  delete h;
  return MDP_OK;
}

mdp_status mdp_create(int64_t S, int32_t A, const int64_t* row_ptr, const int32_t* col,
                      const double* val, const double* cost, double gamma,
                      const mdp_create_opts* opt, mdp_t* out) {
  clear_error();
  if (!out) return fail(MDP_E_INVAL, "out is NULL");
  *out = nullptr;
  mdp_create_opts o;
  mdp_default_create_opts(&o);
  if (opt) {
    if (opt->struct_size < sizeof(mdp_create_opts)) return fail(MDP_E_INVAL, "mdp_create_opts.struct_size too small");
    o = *opt;
  }
  if (S < 1 || A < 1) return fail(MDP_E_INVAL, "S and A must be at least 1");
  MDP_TRY(check_size_limits(S, A, -1));
  if (!(gamma >= 0.0 && gamma < 1.0)) return fail(MDP_E_INVAL, "gamma must lie in [0,1)");
  if (!row_ptr || !col || !val || !cost) return fail(MDP_E_INVAL, "NULL MDP array");
  if (o.lanes_per_row != 0 &&
      (o.lanes_per_row < 2 || o.lanes_per_row > 64 || (o.lanes_per_row & (o.lanes_per_row - 1))))
    return fail(MDP_E_INVAL, "lanes_per_row must be 0 or a power of two in [2,64]");
  if (o.low_precision & ~(MDP_BUILD_FP32 | MDP_BUILD_FP16))
    return fail(MDP_E_INVAL, "unknown low_precision bits");
  if (o.objective != MDP_MINIMIZE_COST && o.objective != MDP_MAXIMIZE_REWARD)
    return fail(MDP_E_INVAL, "unknown objective");
  if (o.validate < MDP_VALIDATE_NONE || o.validate > MDP_VALIDATE_DEVICE)
    return fail(MDP_E_INVAL, "validate must be MDP_VALIDATE_NONE, _HOST or _DEVICE");
  if (o.col_blocks < -1 || o.col_blocks > kMaxColBlocks)
    return fail(MDP_E_INVAL, "col_blocks must be -1, 0 or 1.." + std::to_string(kMaxColBlocks));
  const int64_t rows = S * A;

  const bool dev_in = is_device_ptr(row_ptr) || is_device_ptr(col) || is_device_ptr(val) ||
                      is_device_ptr(cost);
  std::vector<int64_t> h_rp;
  const int64_t* rp_host = row_ptr;
  int64_t nnz = 0;
  if (dev_in) {
    // stage through the host for validation
    h_rp.resize(rows + 1);
    MDP_HIP(copy_out(h_rp.data(), row_ptr, (rows + 1) * sizeof(int64_t), static_cast<hipStream_t>(o.stream)));
    rp_host = h_rp.data();
  }
  nnz = rp_host[rows];
  if (nnz < rows) return fail(MDP_E_INVAL, "row_ptr[S*A] smaller than the number of rows");
  MDP_TRY(check_size_limits(S, A, nnz));
  MDP_TRY(validate_row_ptr(S, A, rp_host));
  if (o.validate == MDP_VALIDATE_HOST) {
    if (dev_in) {
      std::vector<int32_t> c(nnz);
      std::vector<double> v(nnz), g(rows);
      hipStream_t cs = static_cast<hipStream_t>(o.stream);
      MDP_HIP(copy_out(c.data(), col, nnz * sizeof(int32_t), cs));
      MDP_HIP(copy_out(v.data(), val, nnz * sizeof(double), cs));
      MDP_HIP(copy_out(g.data(), cost, rows * sizeof(double), cs));
      MDP_TRY(validate_entries_host(S, A, rp_host, c.data(), v.data(), g.data()));
    } else {
      MDP_TRY(validate_entries_host(S, A, rp_host, col, val, cost));
    }
  }

  auto* h = new mdp_handle();
  auto bail = [&](mdp_status st) {
    std::string keep = g_err;
    mdp_destroy(h);
    g_err = keep;
    return st;
  };
#define CHK(call)                                                                         \
  do {                                                                                    \
    hipError_t e_ = (call);                                                               \
    if (e_ != hipSuccess)                                                                 \
      return bail(fail(e_ == hipErrorOutOfMemory ? MDP_E_NOMEM : MDP_E_DEVICE,            \
                       std::string(#call) + ": " + hipGetErrorString(e_)));               \
  } while (0)
  h->S = S;
  h->A = A;
  h->rows = rows;
  h->nnz = nnz;
  h->gamma = gamma;
  h->lanes = o.lanes_per_row ? o.lanes_per_row : default_lanes(static_cast<double>(nnz) / rows);
  {
    const int64_t k0 = rp_host[1] - rp_host[0];
    bool uniform = k0 > 0 && rp_host[rows] == k0 * rows;
    for (int64_t r = 0; uniform && r <= rows; ++r) uniform = rp_host[r] == r * k0;
    h->kfix = uniform ? static_cast<int32_t>(k0) : 0;
  }
  if (o.device >= 0) CHK(hipSetDevice(o.device));
  CHK(hipGetDevice(&h->device));
  if (DeviceArena* a = current_arena()) h->dev_arena = a->device() == h->device ? a : nullptr;
  if (o.lanes_per_row == 0) {
    const int tuned = tune_lookup(h);  // width measured earlier for this class, if any
    if (tuned) h->lanes = tuned;
  }
  if (o.stream) {
    h->stream = static_cast<hipStream_t>(o.stream);
  } else {
    CHK(stream_take(h->device, &h->stream));
    h->own_stream = true;
  }
  h->ldu = (S + 255) / 256 * 256;
  // One allocation holds the CSR arrays, the S-vectors, the partials and the
  // control block: one pool call and one stream sync per create, one free.
  h->part.cap = partials_doubles(S, A, kMaxRestart);
  {
    auto up = [](size_t b) { return (b + 255) / 256 * 256; };
    const size_t sz[] = {static_cast<size_t>(rows + 1) * sizeof(int32_t), static_cast<size_t>(nnz) * sizeof(int32_t),
                         static_cast<size_t>(nnz) * sizeof(double),       static_cast<size_t>(rows) * sizeof(double),
                         static_cast<size_t>(S) * sizeof(double),         static_cast<size_t>(S) * sizeof(double),
                         static_cast<size_t>(S) * sizeof(double),         static_cast<size_t>(S) * sizeof(double),
                         static_cast<size_t>(S) * sizeof(int32_t),        static_cast<size_t>(S) * sizeof(int32_t),
                         h->part.cap * sizeof(double),                    sizeof(Ctl)};
    size_t total = 0;
    for (size_t b : sz) total += up(b);
    CHK(dev_alloc(h, &h->arena, total));
    char* at = h->arena;
    int k = 0;
    auto take = [&]() {
      char* q = at;
      at += up(sz[k++]);
      return q;
    };
    h->row_ptr = reinterpret_cast<int32_t*>(take());
    h->col = reinterpret_cast<int32_t*>(take());
    h->val = reinterpret_cast<double*>(take());
    h->cost = reinterpret_cast<double*>(take());
    h->v = reinterpret_cast<double*>(take());
    h->Tv = reinterpret_cast<double*>(take());
    h->x2 = reinterpret_cast<double*>(take());
    h->io = reinterpret_cast<double*>(take());
    h->pi = reinterpret_cast<int32_t*>(take());
    h->pi_io = reinterpret_cast<int32_t*>(take());
    h->part.buf = reinterpret_cast<double*>(take());
    h->ctl = reinterpret_cast<Ctl*>(take());
  }
  // Rows are stored in the tile-by-tile, action-major order of row_of():
  // the natural arrays go to a staging block and one kernel moves them.
  // Device validation reads the natural arrays before they move.
  const bool permute = A > 1 && sweep_tile_states(A) > 1;
  {
    // staging: [verdicts | natural col | val | cost | int32 row_ptr | int64
    // row_ptr]; natural arrays only when the rows are permuted, the int64 copy
    // only when row_ptr is host memory (it is narrowed on the device)
    auto up = [](size_t b) { return (b + 255) / 256 * 256; };
    const bool on_dev = o.validate == MDP_VALIDATE_DEVICE;
    const bool rp_dev = is_device_ptr(row_ptr);
    const int vblocks = on_dev ? validate_blocks(rows) : 0;
    const size_t o_col = up(static_cast<size_t>(vblocks) * 3 * sizeof(int64_t));
    const size_t o_val = o_col + up(nnz * sizeof(int32_t));
    const size_t o_cost = o_val + up(nnz * sizeof(double));
    const size_t o_rp = o_cost + up(rows * sizeof(double));
    const size_t o_rp64 = up(permute ? o_rp + (rows + 1) * sizeof(int32_t) : o_col);
    const size_t bytes = rp_dev ? (permute ? o_rp + (rows + 1) * sizeof(int32_t) : o_col)
                                : o_rp64 + (rows + 1) * sizeof(int64_t);
    char* stage = nullptr;
    if (bytes > 0) CHK(staging_alloc(h->device, h->stream, bytes, &stage));
    int32_t* rp_nat = permute ? reinterpret_cast<int32_t*>(stage + o_rp) : h->row_ptr;
    int32_t* col_nat = permute ? reinterpret_cast<int32_t*>(stage + o_col) : h->col;
    double* val_nat = permute ? reinterpret_cast<double*>(stage + o_val) : h->val;
    double* cost_nat = permute ? reinterpret_cast<double*>(stage + o_cost) : h->cost;
    const int64_t* rp64 = rp_dev ? row_ptr : reinterpret_cast<const int64_t*>(stage + o_rp64);
    StageBlock vb;  // pinned landing place of the verdicts
    const size_t vbytes = static_cast<size_t>(vblocks) * 3 * sizeof(int64_t);
    hipError_t e = on_dev && (vbytes > kStageBlockBytes || !stage_take(&vb)) ? hipErrorOutOfMemory : hipSuccess;
    if (e == hipSuccess && !rp_dev)
      e = copy_in(stage + o_rp64, row_ptr, (rows + 1) * sizeof(int64_t), h->stream);
    if (e == hipSuccess) e = launch_narrow_offsets(h->stream, rp64, rp_nat, rows + 1);
    if (e == hipSuccess) e = copy_in(col_nat, col, nnz * sizeof(int32_t), h->stream);
    if (e == hipSuccess) e = copy_in(val_nat, val, nnz * sizeof(double), h->stream);
    if (e == hipSuccess) e = copy_in(cost_nat, cost, rows * sizeof(double), h->stream);
    if (e == hipSuccess && on_dev) {
      auto* vd = reinterpret_cast<int64_t*>(stage);
      e = launch_validate(h->stream, S, rows, rp_nat, col_nat, val_nat, cost_nat, vd, vblocks);
      if (e == hipSuccess) e = hipMemcpyAsync(vb.p, vd, vbytes, hipMemcpyDeviceToHost, h->stream);
    }
    // moving rows is safe before the verdict: row_ptr was checked on the host
    if (e == hipSuccess && permute)
      e = launch_permute_rows(h->stream, S, A, rp_nat, col_nat, val_nat, cost_nat, h->row_ptr, h->col,
                              h->val, h->cost);
    if (stage) {
      const hipError_t ef = staging_free(stage, h->stream);  // after the kernels, in stream order
      if (e == hipSuccess) e = ef;
    }
    const hipError_t es = hipStreamSynchronize(h->stream);  // nothing in flight reads host memory
    if (e == hipSuccess) e = es;
    std::vector<int64_t> verdict(vbytes / sizeof(int64_t));
    if (e == hipSuccess && on_dev) std::memcpy(verdict.data(), vb.p, vbytes);
    stage_give(vb);
    CHK(e);
    if (on_dev) {
      int64_t cost_row = -1, entry_row = -1;
      int why = 0;
      for (int b = 0; b < vblocks; ++b) {
        const int64_t* q = &verdict[static_cast<size_t>(b) * 3];
        if (q[0] >= 0 && (cost_row < 0 || q[0] < cost_row)) cost_row = q[0];
        if (q[1] >= 0 && (entry_row < 0 || q[1] < entry_row)) {
          entry_row = q[1];
          why = static_cast<int>(q[2]);
        }
      }
      if (cost_row >= 0 || entry_row >= 0) return bail(entry_failure(cost_row, entry_row, why));
    }
  }
  h->maximize = o.objective == MDP_MAXIMIZE_REWARD;
  if (h->maximize) CHK(launch_negate(h->stream, h->cost, rows));  // rewards -> costs
  h->ctl_host = ctl_slot_take();
  if (!h->ctl_host) CHK(hipErrorOutOfMemory);
  {
    hipError_t e = hipSuccess;
    {
      std::shared_lock<std::shared_mutex> g(alloc_lock());
      e = hipEventCreateWithFlags(&h->ctl_event, hipEventDisableTiming);
    }
    CHK(e);
  }
  std::memset(h->ctl_host, 0, sizeof(Ctl));
  CHK(hipMemsetAsync(h->ctl, 0, sizeof(Ctl), h->stream));
  if (o.low_precision & MDP_BUILD_FP32) {
    mdp_status st = ensure_lowp(h, kF32);
    if (st < 0) return bail(st);
  }
  if (o.low_precision & MDP_BUILD_FP16) {
    mdp_status st = ensure_lowp(h, kF16);
    if (st < 0) return bail(st);
  }
  {
    // column-blocked copy for the float64 sweep: forced, or automatic when v
    // spans several L2s and most columns lie outside the row's own slice
    const int64_t slice_states = kColSliceBytes / static_cast<int64_t>(sizeof(double));
    const bool tiles_fit = static_cast<int64_t>(sweep_tile_states(A)) * A <= 4 * kBlock;
    int blocks = 0;
    if (o.col_blocks > 0) {
      blocks = o.col_blocks;
      if (!tiles_fit) return bail(fail(MDP_E_NOTSUP, "col_blocks needs A <= 1024"));
    } else if (o.col_blocks < 0 && tiles_fit && S >= kColBlockMinStates) {
      blocks = static_cast<int>(std::min<int64_t>(kMaxColBlocks, (S + slice_states - 1) / slice_states));
    }
    if (blocks > 0) {
      bool built = false;
      double far = 0.0;
      CHK(build_colblocks(h, blocks, o.col_blocks > 0, &built, &far));
      if (o.col_blocks > 0 && !built)
        return bail(fail(MDP_E_NOTSUP, "col_blocks: a row holds more than 255 entries of one column "
                                       "slice, or its columns are not in increasing slice order"));
    }
    // without a blocked copy, short rows: the sweep streams each tile's rows
    // (on the 4M-state maze, 4.2 entries per row: 336 against 547 us per
    // synced sweep; on the 1M-state workload, 16 per row, it would be slower)
    h->flat_sweep = o.col_blocks < 0 && h->cb_blocks == 0 && tiles_fit && S >= kPolicyCopyMinStates &&
                    h->nnz <= kPolicyCopyMaxRowMean * h->rows;
  }
  CHK(hipStreamSynchronize(h->stream));
#undef CHK
  *out = h;
  return MDP_OK;
}

mdp_status mdp_create_from_rows(int64_t S, int32_t A, int32_t k_max, mdp_rows_fn fn, void* user,
                                double gamma, const mdp_create_opts* opt, mdp_t* out) {
  clear_error();
  if (!out) return fail(MDP_E_INVAL, "out is NULL");
  *out = nullptr;
  if (!fn) return fail(MDP_E_INVAL, "row function is NULL");
  if (S < 1 || A < 1) return fail(MDP_E_INVAL, "S and A must be at least 1");
  if (k_max < 1) return fail(MDP_E_INVAL, "k_max must be at least 1");
  MDP_TRY(check_size_limits(S, A, -1));
  const int64_t rows = S * A;
  const unsigned nt = std::max(1u, std::min(16u, std::thread::hardware_concurrency()));
  // ranges of about 2^20 padded entries, handed out to the threads in turn
  const int64_t chunk = std::max<int64_t>(1, (int64_t{1} << 20) / (static_cast<int64_t>(A) * k_max));
  const int64_t n_chunks = (S + chunk - 1) / chunk;
  std::vector<int32_t> pcol, len(rows);
  std::vector<double> pval, cost(rows);
  try {
    pcol.resize(static_cast<size_t>(rows) * k_max);
    pval.resize(static_cast<size_t>(rows) * k_max);
  } catch (const std::bad_alloc&) {
    return fail(MDP_E_NOMEM, "host memory for the padded rows");
  }
  std::atomic<int64_t> next{0};
  std::atomic<int> failed{0};
  auto fill = [&]() {
    for (;;) {
      const int64_t c = next.fetch_add(1);
      if (c >= n_chunks || failed.load()) return;
      const int64_t s0 = c * chunk, s1 = std::min(S, s0 + chunk), r0 = s0 * A;
      if (fn(user, s0, s1, k_max, pcol.data() + r0 * k_max, pval.data() + r0 * k_max, len.data() + r0,
             cost.data() + r0) != 0)
        failed.store(1);
    }
  };
  {
    std::vector<std::thread> ts;
    for (unsigned t = 0; t < nt; ++t) ts.emplace_back(fill);
    for (auto& t : ts) t.join();
  }
  if (failed.load()) return fail(MDP_E_INVAL, "the row function reported a failure");
  std::vector<int64_t> rp(rows + 1);
  rp[0] = 0;
  for (int64_t r = 0; r < rows; ++r) {
    if (len[r] < 0 || len[r] > k_max)
      return fail(MDP_E_INVAL, "row " + std::to_string(r) + " has " + std::to_string(len[r]) +
                                   " entries (k_max " + std::to_string(k_max) + ")");
    rp[r + 1] = rp[r] + len[r];
  }
  const int64_t nnz = rp[rows];
  MDP_TRY(check_size_limits(S, A, nnz));
  std::vector<int32_t> col;
  std::vector<double> val;
  try {
    col.resize(nnz);
    val.resize(nnz);
  } catch (const std::bad_alloc&) {
    return fail(MDP_E_NOMEM, "host memory for the packed rows");
  }
  {
    std::vector<std::thread> ts;
    for (unsigned t = 0; t < nt; ++t)
      ts.emplace_back([&, t]() {
        for (int64_t r = t; r < rows; r += nt) {
          std::memcpy(col.data() + rp[r], pcol.data() + r * k_max, len[r] * sizeof(int32_t));
          std::memcpy(val.data() + rp[r], pval.data() + r * k_max, len[r] * sizeof(double));
        }
      });
    for (auto& t : ts) t.join();
  }
  std::vector<int32_t>().swap(pcol);
  std::vector<double>().swap(pval);
  return mdp_create(S, A, rp.data(), col.data(), val.data(), cost.data(), gamma, opt, out);
}

mdp_status mdp_info(mdp_t h, int64_t* S, int32_t* A, int64_t* nnz, int32_t* lanes,
                    int64_t* device_bytes) {
  clear_error();
  if (!h) return fail(MDP_E_INVAL, "NULL handle");
  if (S) *S = h->S;
  if (A) *A = h->A;
  if (nnz) *nnz = h->nnz;
  if (lanes) *lanes = h->lanes;
  if (device_bytes) *device_bytes = h->device_bytes;
  return MDP_OK;
}

mdp_status mdp_bellman(mdp_t h, const double* v, double* Tv, int32_t* policy, double* res_inf) {
  clear_error();
  if (!h) return fail(MDP_E_INVAL, "NULL handle");
  if (!v) return fail(MDP_E_INVAL, "v is NULL");
  BusyGuard g(h);
  if (!g.ok) return fail(MDP_E_STATE, "handle is busy");
  const size_t vb = h->S * sizeof(double), pb = h->S * sizeof(int32_t);
  const double* vin = v;
  if (!is_device_ptr(v) || v == Tv || h->maximize) {
    MDP_TRY(load_vec(h, v, h->io));  // negated into cost terms when the handle maximises
    vin = h->io;
  }
  double* tv_dev = (Tv && is_device_ptr(Tv)) ? Tv : h->Tv;
  int32_t* pi_dev = (policy && is_device_ptr(policy)) ? policy : h->pi;
  MDP_HIP(launch_bellman(h, kF64, vin, tv_dev, pi_dev, nullptr, false, kRedPlain, 0, 0.0, 0.0));
  if (Tv) {
    if (h->maximize) MDP_HIP(launch_negate(h->stream, tv_dev, h->S));
    MDP_TRY(store(h, Tv, tv_dev, vb));
  }
  if (policy) MDP_TRY(store(h, policy, pi_dev, pb));
  MDP_TRY(sync_ctl(h));
  const double res = h->ctl_host->res_max;
  if (res_inf) *res_inf = res;
  if (!std::isfinite(res)) return fail(MDP_E_NUMERIC, "non-finite Bellman residual");
  return MDP_OK;
}

mdp_status mdp_policy_apply(mdp_t h, const int32_t* policy, const double* x, double* y,
                            int32_t mode) {
  clear_error();
  if (!h) return fail(MDP_E_INVAL, "NULL handle");
  if (!x || !y) return fail(MDP_E_INVAL, "x and y must be non-NULL");
  if (mode != 0 && mode != 1) return fail(MDP_E_INVAL, "mode must be 0 or 1");
  BusyGuard g(h);
  if (!g.ok) return fail(MDP_E_STATE, "handle is busy");
  MDP_TRY(load_policy(h, policy, h->pi_io));
  const size_t vb = h->S * sizeof(double);
  const double* xin = x;
  if (!is_device_ptr(x) || x == y || h->maximize) {
    MDP_TRY(load_vec(h, x, h->io));
    xin = h->io;
  }
  double* ydev = is_device_ptr(y) ? y : h->Tv;
  MDP_HIP(launch_apply(h, mode == 0 ? kApplyOp : kApplyT, h->pi_io, xin, ydev, false, kRedNone, 0,
                       0.0, 0.0));
  if (h->maximize) MDP_HIP(launch_negate(h->stream, ydev, h->S));
  MDP_TRY(store(h, y, ydev, vb));
  MDP_HIP(hipStreamSynchronize(h->stream));
  return MDP_OK;
}

mdp_status mdp_policy_eval(mdp_t h, const int32_t* policy, const double* v0, double* v,
                           const mdp_eval_opts* opt, mdp_stats* stats) {
  clear_error();
  const double t0 = now_ms();
  if (!h) return fail(MDP_E_INVAL, "NULL handle");
  if (!v) return fail(MDP_E_INVAL, "v is NULL");
  if (!stats_ok(stats)) return fail(MDP_E_INVAL, "mdp_stats.struct_size too small");
  mdp_eval_opts o;
  mdp_default_eval_opts(&o);
  if (opt) {
    if (opt->struct_size < sizeof(mdp_eval_opts)) return fail(MDP_E_INVAL, "mdp_eval_opts.struct_size too small");
    o = *opt;
  }
  if (o.inner < MDP_INNER_GMRES || o.inner > MDP_INNER_TFQMR) return fail(MDP_E_INVAL, "unknown inner solver");
  if ((o.inner == MDP_INNER_BICGSTAB || o.inner == MDP_INNER_TFQMR) && o.precision != MDP_FP64)
    return fail(MDP_E_NOTSUP, "BiCGSTAB and TFQMR run in float64 only");
  if (o.restart < 1 || o.restart > kMaxRestart) return fail(MDP_E_INVAL, "restart must lie in [1,64]");
  if (o.precision < MDP_FP64 || o.precision > MDP_MIXED_FP16) return fail(MDP_E_INVAL, "unknown precision");
  if (o.inner == MDP_INNER_RICHARDSON && o.precision != MDP_FP64)
    return fail(MDP_E_NOTSUP, "Richardson runs in float64 only");
  if (!(o.rtol >= 0.0) || o.max_iter < 0) return fail(MDP_E_INVAL, "bad tolerance or iteration cap");
  if (o.precond_degree < 0 || o.precond_degree > kMaxPrecondDegree)
    return fail(MDP_E_INVAL, "precond_degree must lie in [0,16]");
  const int deg = std::max(1, o.precond_degree);
  if (deg > 1 && o.inner != MDP_INNER_GMRES)
    return fail(MDP_E_NOTSUP, "the polynomial preconditioner serves GMRES only");
  if (o.gs_passes < 0 || o.gs_passes > 2) return fail(MDP_E_INVAL, "gs_passes must be 0, 1 or 2");
  const bool gs2 = o.gs_passes == 2;
  if (gs2 && o.inner != MDP_INNER_GMRES) return fail(MDP_E_NOTSUP, "gs_passes = 2 serves GMRES only");
  BusyGuard g(h);
  if (!g.ok) return fail(MDP_E_STATE, "handle is busy");
  stats_begin(stats);
  const int sync_every = o.sync_every > 0 ? o.sync_every : 4;
  MDP_TRY(load_policy(h, policy, h->pi));
  MDP_TRY(load_vec(h, v0, h->v));
  MDP_HIP(launch_ctl_reset(h, 0.0));
  InnerResult ir;
  double* result = h->v;
  double rel = 0.0;
  if (o.inner == MDP_INNER_BICGSTAB || o.inner == MDP_INNER_TFQMR) {
    MDP_TRY(ensure_basis(h, kF64, std::max(o.restart, 7)));
    MDP_HIP(launch_apply(h, kApplyRes, h->pi, h->v, h->U64, false, kRedGmresStart, 1, o.rtol, 0.0));
    ir.applies += 1;
    MDP_TRY(bicgstab_inner(h, h->pi, h->v, o.max_iter, sync_every, &ir, o.inner == MDP_INNER_TFQMR,
                           o.policy_copy));
    rel = h->ctl_host->beta0 > 0 ? h->ctl_host->res_est / h->ctl_host->beta0 : 0.0;
  } else if (o.inner == MDP_INNER_GMRES) {
    const Prec prec = prec_of(o.precision);
    MDP_TRY(ensure_basis(h, prec == kF64 ? kF64 : kF32, o.restart + (deg > 1 ? 3 : 0)));
    if (prec != kF64) MDP_TRY(ensure_lowp(h, prec));
    void* slot0 = prec == kF64 ? static_cast<void*>(h->U64) : static_cast<void*>(h->U32);
    MDP_HIP(launch_apply(h, kApplyRes, h->pi, h->v, slot0, prec != kF64, kRedGmresStart, 1, o.rtol,
                         floor_of(prec)));
    ir.applies += 1;
    MDP_TRY(gmres_inner(h, prec, h->pi, h->v, o.restart, o.max_iter, sync_every, o.rtol, &ir, deg, gs2,
                        o.policy_copy));
    MDP_TRY(sync_ctl(h));
    rel = h->ctl_host->beta0 > 0 ? h->ctl_host->res_est / h->ctl_host->beta0 : 0.0;
    if (ir.converged && prec != kF64)
      rel = h->ctl_host->beta0 > 0 ? h->ctl_host->beta / h->ctl_host->beta0 : 0.0;
  } else {
    // first step sets the tolerance rtol * max|x1 - x0|
    MDP_HIP(launch_apply(h, kApplyT, h->pi, h->v, h->x2, false, kRedRichardson, 1, o.rtol, 0.0));
    if (o.max_iter >= 1) {
      MDP_TRY(richardson_inner(h, h->pi, h->v, h->x2, std::max<int64_t>(1, o.max_iter), sync_every,
                               &ir, &result));
    }
    rel = ir.converged ? 0.0 : 1.0;
  }
  MDP_TRY(store_values(h, v, result));
  MDP_HIP(hipStreamSynchronize(h->stream));
  if (stats) {
    stats->inner_iters = ir.steps;
    stats->policy_applies = ir.applies;
    stats->refinements = ir.refinements;
    stats->orth_loss = ir.orth_loss;
    stats->residual = rel;
    stats->bytes = ir.bytes;
    stats->time_ms = now_ms() - t0;
  }
  return ir.converged ? MDP_OK : MDP_W_MAXITER;
}

mdp_status mdp_solve(mdp_t h, const double* v0, double* v, int32_t* policy,
                     const mdp_solve_opts* opt, mdp_stats* stats) {
  clear_error();
  const double t0 = now_ms();
  if (!h) return fail(MDP_E_INVAL, "NULL handle");
  if (!v || !policy) return fail(MDP_E_INVAL, "v and policy must be non-NULL");
  if (!stats_ok(stats)) return fail(MDP_E_INVAL, "mdp_stats.struct_size too small");
  mdp_solve_opts o;
  mdp_default_solve_opts(&o);
  if (opt) {
    if (opt->struct_size < sizeof(mdp_solve_opts)) return fail(MDP_E_INVAL, "mdp_solve_opts.struct_size too small");
    o = *opt;
  }
  if (o.inner < MDP_INNER_GMRES || o.inner > MDP_INNER_TFQMR) return fail(MDP_E_INVAL, "unknown inner solver");
  if ((o.inner == MDP_INNER_BICGSTAB || o.inner == MDP_INNER_TFQMR) && o.precision != MDP_FP64)
    return fail(MDP_E_NOTSUP, "BiCGSTAB and TFQMR run in float64 only");
  if (o.restart < 1 || o.restart > kMaxRestart) return fail(MDP_E_INVAL, "restart must lie in [1,64]");
  if (o.precision < MDP_FP64 || o.precision > MDP_MIXED_FP16) return fail(MDP_E_INVAL, "unknown precision");
  if (o.inner == MDP_INNER_RICHARDSON && o.precision != MDP_FP64)
    return fail(MDP_E_NOTSUP, "Richardson runs in float64 only");
  if (!(o.alpha > 0.0 && o.alpha < 1.0)) return fail(MDP_E_INVAL, "alpha must lie in (0,1)");
  if (!(o.atol > 0.0) || o.max_outer < 0 || o.max_inner < 1) return fail(MDP_E_INVAL, "bad tolerance or caps");
  if (o.precond_degree < 0 || o.precond_degree > kMaxPrecondDegree)
    return fail(MDP_E_INVAL, "precond_degree must lie in [0,16]");
  const int deg = std::max(1, o.precond_degree);
  if (deg > 1 && o.inner != MDP_INNER_GMRES)
    return fail(MDP_E_NOTSUP, "the polynomial preconditioner serves GMRES only");
  if (o.gs_passes < 0 || o.gs_passes > 2) return fail(MDP_E_INVAL, "gs_passes must be 0, 1 or 2");
  const bool gs2 = o.gs_passes == 2;
  if (gs2 && o.inner != MDP_INNER_GMRES) return fail(MDP_E_NOTSUP, "gs_passes = 2 serves GMRES only");
  BusyGuard g(h);
  if (!g.ok) return fail(MDP_E_STATE, "handle is busy");
  stats_begin(stats);
  const int sync_every = o.sync_every > 0 ? o.sync_every : 4;
  const Prec iprec = prec_of(o.precision);
  const bool gm = o.inner == MDP_INNER_GMRES;
  const bool bi = o.inner == MDP_INNER_BICGSTAB || o.inner == MDP_INNER_TFQMR;
  if (gm) MDP_TRY(ensure_basis(h, iprec == kF64 ? kF64 : kF32, o.restart + (deg > 1 ? 3 : 0)));
  if (bi) MDP_TRY(ensure_basis(h, kF64, std::max(o.restart, 7)));
  if (iprec != kF64) MDP_TRY(ensure_lowp(h, iprec));
  MDP_TRY(load_vec(h, v0, h->v));
  MDP_HIP(launch_ctl_reset(h, 0.0));

  double alpha = o.alpha;
  double prev_res = std::numeric_limits<double>::infinity();
  double res = prev_res, tv_max = 0.0;
  int64_t k = 0, sweeps = 0, inner = 0, applies = 0, refinements = 0;
  double bytes = 0.0, orth_loss = 0.0;
  bool converged = false;
  // mixed precision: low-precision sweeps until the residual is small relative to |v|;
  // with a column-blocked copy the float64 sweep is the faster one and is used throughout
  bool lowp_sweep = iprec != kF64 && h->cb_blocks == 0;
  double prev_lowp_res = std::numeric_limits<double>::infinity();
  for (;;) {
    const Prec sp = lowp_sweep ? iprec : kF64;
    const void* vin = h->v;
    if (sp != kF64) {
      MDP_HIP(launch_cast_f32(h->stream, h->v, h->v32, h->S));
      vin = h->v32;
    }
    const bool r0f32 = iprec != kF64;
    // GMRES and BiCGSTAB start from r0 = T v - v, which the sweep writes into basis slot 0
    const bool keep_r0 = gm || bi;
    void* r0 = keep_r0 ? (iprec == kF64 ? static_cast<void*>(h->U64) : static_cast<void*>(h->U32)) : nullptr;
    double* tv_out = keep_r0 ? nullptr : h->x2;
    MDP_HIP(launch_bellman(h, sp, vin, tv_out, h->pi, r0, r0f32, keep_r0 ? kRedGmresStart : kRedPlain, 1,
                           alpha, floor_of(iprec)));
    ++sweeps;
    bytes += bytes_sweep(h, bval_of(sp), sp == kF64 ? 8 : 4, keep_r0, r0f32 ? 4 : 8);
    MDP_TRY(sync_ctl(h));
    res = h->ctl_host->res_max;
    tv_max = h->ctl_host->aux_max;
    if (!std::isfinite(res)) return fail(MDP_E_NUMERIC, "non-finite Bellman residual");
    if (lowp_sweep) {
      // The low-precision sweep stops being informative once its residual
      // nears the rounding level of the reduced-precision P (unit roundoff u_P
      // times |v|) or stops shrinking; from then on (and for the final stop
      // test) sweeps run in float64.  The sweep is redone at once in float64.
      const double uP = sp == kF16 ? 4.9e-4 : 6.0e-8;
      if (res <= std::max(1e-5, 16.0 * uP) * tv_max || res <= 10.0 * o.atol ||
          res > 0.5 * prev_lowp_res) {
        lowp_sweep = false;
        continue;
      }
      prev_lowp_res = res;
    }
    if (stats && stats->history && stats->history_len < stats->history_cap)
      stats->history[stats->history_len++] = res;
    const bool cert_ok = o.rtol_cert <= 0.0 || res <= o.rtol_cert * (1.0 - h->gamma) * tv_max;
    if (!lowp_sweep && res <= o.atol && cert_ok) {
      converged = true;
      break;
    }
    if (k >= o.max_outer) break;
    if (res > prev_res) alpha = std::max(alpha * 0.5, 1e-12);  // iPI is not globally monotone
    prev_res = res;
    InnerResult ir;
    if (gm) {
      MDP_TRY(gmres_inner(h, iprec, h->pi, h->v, o.restart, o.max_inner, sync_every, alpha, &ir, deg, gs2,
                          o.policy_copy));
    } else if (bi) {
      MDP_TRY(bicgstab_inner(h, h->pi, h->v, o.max_inner, sync_every, &ir, o.inner == MDP_INNER_TFQMR,
                             o.policy_copy));
    } else {
      // x1 = T v_k is already in x2; continue T_pi from there
      double* last = h->x2;
      ir.steps = 1;
      ir.applies = 0;
      if (o.max_inner > 1) {
        // the iterate x1 = T v_k sits in buffer 1 (x2); one step is done
        MDP_HIP(launch_rich_begin(h, alpha * res, 1, 1));
        MDP_TRY(richardson_inner(h, h->pi, h->v, h->x2, o.max_inner, sync_every, &ir, &last));
      }
      if (last != h->v) std::swap(h->v, h->x2);
    }
    inner += ir.steps;
    applies += ir.applies;
    refinements += ir.refinements;
    bytes += ir.bytes;
    orth_loss = std::max(orth_loss, ir.orth_loss);
    ++k;
  }
  MDP_TRY(store_values(h, v, h->v));
  MDP_TRY(store(h, policy, h->pi, h->S * sizeof(int32_t)));
  MDP_HIP(hipStreamSynchronize(h->stream));
  if (stats) {
    stats->outer_iters = k;
    stats->inner_iters = inner;
    stats->bellman_sweeps = sweeps;
    stats->policy_applies = applies;
    stats->refinements = refinements;
    stats->orth_loss = orth_loss;
    stats->residual = res;
    stats->bytes = bytes;
    stats->time_ms = now_ms() - t0;
  }
  return converged ? MDP_OK : MDP_W_MAXITER;
}

mdp_status mdp_solve_batch(mdp_t* handles, int32_t n, const double* const* v0, double* const* v,
                           int32_t* const* policy, const mdp_solve_opts* opt, mdp_stats* stats) {
  clear_error();
  const double t0 = now_ms();
  if (!handles || n < 1 || !v || !policy) return fail(MDP_E_INVAL, "bad batch arguments");
  mdp_solve_opts o;
  mdp_default_solve_opts(&o);
  if (opt) {
    if (opt->struct_size < sizeof(mdp_solve_opts)) return fail(MDP_E_INVAL, "mdp_solve_opts.struct_size too small");
    o = *opt;
  }
  if (o.inner != MDP_INNER_GMRES) return fail(MDP_E_NOTSUP, "batched solves use GMRES");
  if (o.precond_degree > 1) return fail(MDP_E_NOTSUP, "batched solves run without a preconditioner");
  if (o.gs_passes > 1) return fail(MDP_E_NOTSUP, "batched solves use one Gram-Schmidt pass");
  if (o.launch < MDP_LAUNCH_AUTO || o.launch > MDP_LAUNCH_DIRECT) return fail(MDP_E_INVAL, "unknown launch mode");
  if (o.restart < 1 || o.restart > kMaxRestart) return fail(MDP_E_INVAL, "restart must lie in [1,64]");
  if (o.precision < MDP_FP64 || o.precision > MDP_MIXED_FP16) return fail(MDP_E_INVAL, "unknown precision");
  if (!(o.alpha > 0.0 && o.alpha < 1.0)) return fail(MDP_E_INVAL, "alpha must lie in (0,1)");
  if (!(o.atol > 0.0) || o.max_outer < 0 || o.max_inner < 1) return fail(MDP_E_INVAL, "bad tolerance or caps");
  for (int i = 0; i < n; ++i) {
    if (!handles[i] || !v[i] || !policy[i]) return fail(MDP_E_INVAL, "NULL handle or output in batch");
    if (handles[i]->device != handles[0]->device) return fail(MDP_E_INVAL, "batch spans devices");
    for (int j = 0; j < i; ++j)
      if (handles[j] == handles[i]) return fail(MDP_E_INVAL, "handle listed twice in batch");
    if (stats && !stats_ok(stats + i)) return fail(MDP_E_INVAL, "mdp_stats.struct_size too small");
  }
  std::vector<std::unique_ptr<BusyGuard>> guards;
  for (int i = 0; i < n; ++i) {
    guards.emplace_back(new BusyGuard(handles[i]));
    if (!guards.back()->ok) return fail(MDP_E_STATE, "handle in batch is busy");
  }
  const Prec prec = prec_of(o.precision);
  std::vector<BatchItem> items(n);
  for (int i = 0; i < n; ++i) {
    mdp_handle* h = handles[i];
    if (stats) stats_begin(stats + i);
    MDP_TRY(ensure_basis(h, prec == kF64 ? kF64 : kF32, o.restart));
    if (prec != kF64) MDP_TRY(ensure_lowp(h, prec));
    MDP_TRY(load_vec(h, v0 ? v0[i] : nullptr, h->v));
    MDP_HIP(launch_ctl_reset(h, 0.0));
    MDP_HIP(hipStreamSynchronize(h->stream));
    BatchItem& it = items[i];
    it.h = h;
    it.alpha = o.alpha;
    it.prev_res = std::numeric_limits<double>::infinity();
    it.prev_lowp_res = std::numeric_limits<double>::infinity();
    it.lowp_sweep = prec != kF64;
  }
  EngineLease lease(handles[0]->device);
  if (!lease.eng) return fail(MDP_E_NOMEM, "batched engine allocation failed");
  BatchEngine& eng = *lease.eng;
  eng.stream = handles[0]->stream;
  eng.prec = prec;
  eng.use_graphs = o.launch != MDP_LAUNCH_DIRECT;
  eng.items.clear();
  MDP_TRY(eng.reserve(n));
  for (auto& it : items) eng.items.push_back(&it);
  for (;;) {
    bool left = false;
    for (auto& it : items) left = left || it.state != BatchItem::kDone;
    if (!left) break;
    MDP_TRY(eng.round(o));
  }
  mdp_status worst = MDP_OK;
  for (int i = 0; i < n; ++i) {
    BatchItem& it = items[i];
    mdp_handle* h = it.h;
    if (h->maximize) MDP_HIP(launch_negate(eng.stream, h->v, h->S));
    MDP_HIP(copy_out(v[i], h->v, h->S * sizeof(double), eng.stream));
    MDP_HIP(copy_out(policy[i], h->pi, h->S * sizeof(int32_t), eng.stream));
    if (it.status < 0 && worst >= 0) {
      worst = it.status;
      fail(it.status, "batch item " + std::to_string(i) + " failed with a non-finite residual");
    } else if (it.status == MDP_W_MAXITER && worst == MDP_OK) {
      worst = MDP_W_MAXITER;
    }
    if (stats) {
      mdp_stats* st = stats + i;
      st->outer_iters = it.k;
      st->inner_iters = it.inner;
      st->bellman_sweeps = it.sweeps;
      st->policy_applies = it.applies;
      st->refinements = it.refinements;
      st->residual = it.res;
      st->bytes = it.bytes;
      for (double r : it.history)
        if (st->history && st->history_len < st->history_cap) st->history[st->history_len++] = r;
    }
  }
  MDP_HIP(hipStreamSynchronize(eng.stream));
  const double dt = now_ms() - t0;
  if (stats)
    for (int i = 0; i < n; ++i) stats[i].time_ms = dt;
  return worst;
}

mdp_status mdp_profile_sampled(mdp_t h, int32_t enable, int32_t every) {
  clear_error();
  if (!h) return fail(MDP_E_INVAL, "NULL handle");
  if (every < 1) return fail(MDP_E_INVAL, "every must be at least 1");
  BusyGuard g(h);
  if (!g.ok) return fail(MDP_E_STATE, "handle is busy");
  prof_resolve(h);
  if (enable) {
    for (int k = 0; k < MDP_NUM_KERNEL_KINDS; ++k) {
      h->prof_launches[k] = 0;
      h->prof_ms[k] = 0.0;
      h->prof_bytes[k] = 0.0;
      h->prof_seen[k] = 0;
    }
  }
  h->prof_mask = enable < 0 ? (1 << MDP_NUM_KERNEL_KINDS) - 1 : enable;
  h->prof_every = every;
  return MDP_OK;
}

mdp_status mdp_profile(mdp_t h, int32_t enable) { return mdp_profile_sampled(h, enable, 1); }

mdp_status mdp_profile_read(mdp_t h, mdp_kernel_profile* out) {
  clear_error();
  if (!h || !out) return fail(MDP_E_INVAL, "NULL argument");
  if (out->struct_size < sizeof(mdp_kernel_profile)) return fail(MDP_E_INVAL, "mdp_kernel_profile.struct_size too small");
  BusyGuard g(h);
  if (!g.ok) return fail(MDP_E_STATE, "handle is busy");
  prof_resolve(h);
  for (int k = 0; k < MDP_NUM_KERNEL_KINDS; ++k) {
    out->launches[k] = h->prof_launches[k];
    out->ms[k] = h->prof_ms[k];
    out->bytes[k] = h->prof_bytes[k];
  }
  return MDP_OK;
}

mdp_status mdp_autotune(mdp_t h, int32_t* lanes) {
  clear_error();
  if (!h) return fail(MDP_E_INVAL, "NULL handle");
  BusyGuard g(h);
  if (!g.ok) return fail(MDP_E_STATE, "handle is busy");
  hipEvent_t e0, e1;
  MDP_HIP(hipEventCreate(&e0));
  MDP_HIP(hipEventCreate(&e1));
  MDP_HIP(hipMemsetAsync(h->io, 0, h->S * sizeof(double), h->stream));
  MDP_HIP(hipMemsetAsync(h->pi_io, 0, h->S * sizeof(int32_t), h->stream));
  const int prof_was = h->prof_mask;
  h->prof_mask = 0;
  // cost of a width: one sweep plus four policy products (a solve runs
  // several Arnoldi steps per sweep)
  auto time_width = [&](int L, float* out) -> mdp_status {
    h->lanes = L;
    for (int w = 0; w < 2; ++w) {
      MDP_HIP(launch_bellman(h, kF64, h->io, h->Tv, h->pi, nullptr, false, kRedNone, 0, 0, 0));
      MDP_HIP(launch_apply(h, kApplyOp, h->pi_io, h->io, h->x2, false, kRedNone, 0, 0, 0));
    }
    float ms_s = 0, ms_a = 0;
    MDP_HIP(hipEventRecord(e0, h->stream));
    for (int r = 0; r < 3; ++r)
      MDP_HIP(launch_bellman(h, kF64, h->io, h->Tv, h->pi, nullptr, false, kRedNone, 0, 0, 0));
    MDP_HIP(hipEventRecord(e1, h->stream));
    MDP_HIP(hipEventSynchronize(e1));
    MDP_HIP(hipEventElapsedTime(&ms_s, e0, e1));
    MDP_HIP(hipEventRecord(e0, h->stream));
    for (int r = 0; r < 3; ++r)
      MDP_HIP(launch_apply(h, kApplyOp, h->pi_io, h->io, h->x2, false, kRedNone, 0, 0, 0));
    MDP_HIP(hipEventRecord(e1, h->stream));
    MDP_HIP(hipEventSynchronize(e1));
    MDP_HIP(hipEventElapsedTime(&ms_a, e0, e1));
    *out = ms_s + 4.0f * ms_a;
    return MDP_OK;
  };
  // Timings taken while other work shares the GPU (a server tunes under
  // load) only ever come out too long, so every width is timed in three
  // rounds and keeps its shortest time; the width the row length suggests
  // stays unless another one beats it by more than 5%.
  const int dflt = default_lanes(static_cast<double>(h->nnz) / h->rows);
  float t_min[7];
  for (float& t : t_min) t = std::numeric_limits<float>::infinity();
  mdp_status st = MDP_OK;
  for (int round = 0; round < 3 && st == MDP_OK; ++round)
    for (int k = 0, L = 2; L <= 64 && st == MDP_OK; ++k, L <<= 1) {
      float ms = 0;
      st = time_width(L, &ms);
      if (st == MDP_OK && ms < t_min[k]) t_min[k] = ms;
    }
  int best = dflt;
  float best_ms = std::numeric_limits<float>::infinity();
  for (int k = 0, L = 2; L <= 64; ++k, L <<= 1)
    if (L == dflt) best_ms = t_min[k] / 1.05f;
  for (int k = 0, L = 2; L <= 64; ++k, L <<= 1)
    if (t_min[k] < best_ms) {
      best_ms = t_min[k];
      best = L;
    }
  h->lanes = best;
  h->prof_mask = prof_was;
  (void)hipEventDestroy(e0);
  (void)hipEventDestroy(e1);
  if (st < 0) return st;
  tune_store(h, best);
  if (lanes) *lanes = best;
  return MDP_OK;
}

}  // extern "C"
