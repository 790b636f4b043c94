// Internal declarations shared by the host driver and the HIP kernels.
#pragma once

#include <hip/hip_runtime.h>
#include <hip/hip_fp16.h>

#include <atomic>
#include <map>
#include <mutex>
#include <shared_mutex>
#include <unordered_map>
#include <vector>
#include <cstdint>
#include <string>

#include "mdp.h"

namespace mdp {

constexpr int kBlock = 256;       // threads per workgroup (4 wavefronts of 64)
constexpr int kWave = 64;         // CDNA wavefront width
constexpr int kNumXcd = 8;        // MI355X: 8 accelerator complex dies, one L2 each
constexpr int kMaxRestart = 64;   // largest GMRES restart length
constexpr int kMaxPrecondDegree = 16;  // most terms of the polynomial preconditioner
#ifndef MDP_APPLY_TILE
#define MDP_APPLY_TILE 512
#endif
#ifndef MDP_UNROLL
#define MDP_UNROLL 4
#endif
#ifndef MDP_SWEEP_ROWS
#define MDP_SWEEP_ROWS 1024
#endif
constexpr int kApplyTile = MDP_APPLY_TILE;  // states per workgroup in the P_pi products
constexpr int kUpdTile = 512;     // states per workgroup in the Arnoldi update

// Device-resident control block of the inner solvers.  Kernels read and
// write it so that the host only synchronises once per batch of steps.
struct Ctl {
  // --- header: the part the host copies back --------------------------------
  double res_max;      // last reduced max |d|
  double sumsq;        // last reduced sum d^2
  double beta;         // 2-norm of the residual that started the current cycle
  double tol;          // absolute stop threshold of the inner solve
  double res_est;      // GMRES residual estimate |g_{j+1}|
  double beta0;        // 2-norm of the first residual of the inner solve
  double tol_cycle;    // stop threshold of the current GMRES cycle (>= tol)
  double aux_max;      // last reduced max |Tv| (Bellman sweeps)
  double orth_loss;    // CGS2: largest ||second-pass coefficients|| / ||w|| of the cycles so far
  int32_t j;           // Arnoldi columns completed in the current cycle
  int32_t done;        // nonzero: kernels of the current batch exit at once
  int32_t converged;   // 1: tolerance met
  int32_t breakdown;   // 1: exact Krylov breakdown
  int32_t bad_policy;  // count of policy entries outside [0, A)
  int32_t steps;       // inner steps executed (device count)
  int32_t rich_cur;    // Richardson: index (0/1) of the buffer holding the iterate
  int32_t pad0;
  // --- Krylov state (device only) -------------------------------------------
  double scale[kMaxRestart + 1];               // 1/||w|| of each stored basis vector
  double hc[kMaxRestart + 1];                  // h_i * scale_i for the update
  double g[kMaxRestart + 1];                   // rotated right-hand side
  double cs[kMaxRestart], sn[kMaxRestart];     // Givens rotations
  double H[(kMaxRestart + 1) * kMaxRestart];   // Hessenberg / R, column-major
  double y[kMaxRestart];                       // least-squares solution
  double h2sq[kMaxRestart + 1];                // CGS2: squares of the second-pass coefficients
  // BiCGSTAB / TFQMR scalars (device only)
  double bi_rho, bi_alpha, bi_omega, bi_beta;
  double tf_theta, tf_eta, tf_tau, tf_half;  // TFQMR: theta, eta, tau, half-steps done
  int32_t tf_stop, pad1;                     // TFQMR: the bound met at the last half-step
};
constexpr size_t kCtlHeaderBytes = offsetof(Ctl, scale);

// A device arena (arena.cpp): one device allocation carved into handle
// arrays by the library, so that code admitting and retiring many handles
// never calls the HIP allocator.  alloc returns nullptr when no free range
// fits; free returns a range once the work queued on `st` so far has finished
// (at once for st == nullptr).  Thread-safe.
class DeviceArena {
 public:
  static DeviceArena* create(int dev, size_t bytes);  // nullptr when the memory is not there
  ~DeviceArena();
  void* alloc(size_t bytes);
  void free(void* p, hipStream_t st);
  bool owns(const void* p) const;
  size_t size() const { return size_; }
  int device() const { return dev_; }
  size_t in_use();

 private:
  DeviceArena() = default;
  struct Pending {
    size_t off;
    hipEvent_t ev;
  };
  int dev_ = 0;
  char* base_ = nullptr;
  size_t size_ = 0, in_use_ = 0;
  std::mutex mu_;
  std::map<size_t, size_t> free_;             // offset -> length, coalesced
  std::unordered_map<size_t, size_t> used_;   // offset -> length
  std::vector<Pending> pending_;              // freed, waiting for their streams
  std::vector<hipEvent_t> spare_;
  void release_locked(size_t off);
  void reap_locked();
};
// The arena holding p, if any.
DeviceArena* arena_of(const void* p);
// While an ArenaScope lives, handles created on this thread (and the staging
// of their creation) take their memory from its arena.
class ArenaScope {
 public:
  explicit ArenaScope(DeviceArena* a);
  ~ArenaScope();

 private:
  DeviceArena* prev_;
};
DeviceArena* current_arena();

struct Partials {
  double* buf;       // device scratch for per-workgroup partial results
  size_t cap;        // doubles
};

}  // namespace mdp

struct mdp_handle {
  int device = 0;
  hipStream_t stream = nullptr;
  bool own_stream = false;
  std::atomic<int> busy{0};

  int64_t S = 0;
  int32_t A = 0;
  int64_t rows = 0, nnz = 0;
  double gamma = 0;
  int32_t lanes = 16;
  int32_t kfix = 0;  // every row holds kfix entries (0: rows differ)
  bool maximize = false;  // costs hold rewards: stored negated, value vectors negated at the ABI

  // CSR on the device (int32 row offsets: nnz < 2^31)
  int32_t* row_ptr = nullptr;
  int32_t* col = nullptr;
  double* val = nullptr;
  double* cost = nullptr;
  char* arena = nullptr;        // one allocation holding row_ptr, col, val, cost, the S-vectors,
                                // the partials and the control block
  float* cv32 = nullptr;        // float32 copy, packed per row: the row's int32 columns, then its
                                // float32 values (2*nnz words; entry e of the row [st, en) has its
                                // column at word st + e and its value at word en + e)
  __half* val16 = nullptr;      // float16 copy
  double* corr16 = nullptr;     // per-row correction 1 - sum fp16(p)
  float* cost32 = nullptr;      // float32 costs

  // Column-blocked copy of P for the float64 sweep (cb_blocks == 0: none).
  // Columns are cut into cb_blocks slices of cb_slice states; the entries of
  // slice b are stored together, tile by tile and row by row inside a tile,
  // so that one pass over slice b gathers only from an L2-sized piece of v.
  int32_t cb_blocks = 0;
  int32_t cb_slice = 0;
  int32_t* cb_col = nullptr;    // nnz
  double* cb_val = nullptr;     // nnz
  uint16_t* cb_rel = nullptr;   // cb_blocks x rows: row start inside its (slice, tile) segment
  int32_t* cb_off = nullptr;    // cb_blocks x (sweep tiles + 1): first entry of (slice, tile)
  double* cb_acc = nullptr;     // cb_xcd: cb_blocks x rows slice parts; else rows: row sums so far
  bool cb_xcd = false;          // all slices in one launch, one slice per XCD
  bool flat_sweep = false;      // float64 sweeps stream each tile's rows (short rows, no blocked copy)

  // float64 vectors
  double* v = nullptr;       // current value iterate
  double* Tv = nullptr;      // Bellman sweep output
  double* x2 = nullptr;      // spare (Richardson ping-pong, residual)
  double* io = nullptr;      // staging for caller vectors
  int32_t* pi = nullptr;     // current policy
  int32_t* pi_io = nullptr;  // staging for caller policies
  // float32 vectors for the mixed path
  float* v32 = nullptr;
  float* x32a = nullptr;
  float* x32b = nullptr;

  // GMRES basis, (m+1) x ldu, in float64 and float32
  double* U64 = nullptr;
  float* U32 = nullptr;
  int32_t basis_m64 = 0, basis_m32 = 0;
  int64_t ldu = 0;

  mdp::Partials part{};
  mdp::Ctl* ctl = nullptr;        // device
  mdp::Ctl* ctl_host = nullptr;   // pinned host mirror of the header
  hipEvent_t ctl_event = nullptr; // marks the header copy of a snapshot

  int64_t device_bytes = 0;

  // XCD-partitioned copy of P_pi for the float64 Arnoldi products
  // (xcdprod.hip): pp_state 0 not set up, 1 set up, -1 not possible here.
  // pi_gen counts the launches that may write a policy; the copy is current
  // for pp_pi while pp_gen == pi_gen.
  int pp_state = 0;
  bool pp_ready = false;  // the products of the running evaluation use the copy
  int pp_blocks = 0, pp_slice = 0, pp_ntiles = 0;
  int64_t pp_cap = 0;
  int* pp_col = nullptr;
  double* pp_val = nullptr;
  uint16_t* pp_rel = nullptr;   // pp_blocks x S: state start inside its tile's segment
  int2* pp_seg = nullptr;       // pp_blocks x pp_ntiles: (first entry, length) of a segment
  double* pp_part = nullptr;    // pp_blocks x S: slice parts of a product
  int* pp_fill = nullptr;       // entries placed so far while the copy is formed, and a changed flag
  int* pp_snap = nullptr;       // the policy of the last formation (S entries)
  const int32_t* pp_pi = nullptr;
  int64_t pp_gen = -1, pi_gen = 0;

  mdp::DeviceArena* dev_arena = nullptr;  // where its arrays come from (nullptr: the pool)
  bool destroying = false;                // its stream is idle: frees return at once

  // profiler: one event pair per launch while enabled
  struct ProfRec {
    int kind;
    int tag;  // Arnoldi step index, or -1
    hipEvent_t a, b;
    double bytes;
  };
  int prof_mask = 0;  // bit k: record kernel class k
  int prof_every = 1;                                // record one launch in prof_every per class
  int64_t prof_seen[MDP_NUM_KERNEL_KINDS] = {};      // launches of each class since enabling
  std::vector<ProfRec> prof_pending;
  std::vector<hipEvent_t> prof_pool;
  int64_t prof_launches[MDP_NUM_KERNEL_KINDS] = {};
  double prof_ms[MDP_NUM_KERNEL_KINDS] = {};
  double prof_bytes[MDP_NUM_KERNEL_KINDS] = {};
};

namespace mdp {

// ---- error reporting (thread-local message) --------------------------------
mdp_status fail(mdp_status st, const std::string& msg);
void clear_error();

#define MDP_HIP(call)                                                              \
  do {                                                                             \
    hipError_t e_ = (call);                                                        \
    if (e_ != hipSuccess)                                                          \
      return ::mdp::fail(e_ == hipErrorOutOfMemory ? MDP_E_NOMEM : MDP_E_DEVICE,   \
                         std::string(#call) + ": " + hipGetErrorString(e_));       \
  } while (0)

#define MDP_TRY(expr)                     \
  do {                                    \
    mdp_status s_ = (expr);               \
    if (s_ < 0) return s_;                \
  } while (0)

// ---- kernel launchers (kernels.hip) -----------------------------------------
// All launchers enqueue on h->stream and return hipSuccess or the launch error.

enum ApplyMode { kApplyOp = 0, kApplyT = 1, kApplyRes = 2 };
enum Prec { kF64 = 0, kF32 = 1, kF16 = 2 };
enum ReduceMode { kRedNone = -1, kRedPlain = 0, kRedGmresStart = 1, kRedRichardson = 2 };

// Rows of the Bellman sweep handled by one workgroup (whole states).
constexpr int kSweepRows = MDP_SWEEP_ROWS;
// Column-blocked sweep: slices of at most 3.25 MB of the float64 vector, so
// that a slice and the streamed entries passing through share one XCD's 4 MB
// L2.  On the 4M-state workload (32 MB of v) a sweep takes 10.75 ms in 10
// slices, against 10.9 ms in 11, 11.2 ms in 9 and in 12, and earlier
// measurements of 12.0 ms in 8 slices of 4 MB and 12.6 ms in 16 of 2 MB:
// fewer passes read and write the running sums fewer times, until the slice
// crowds the streams out of the L2.  Built automatically from 2^21 states
// (16 MB of v) up.
constexpr int64_t kColSliceBytes = int64_t{13} << 18;
// Largest buffer of slice parts (cb_blocks x rows float64) for which the
// blocked sweep runs all slices in one launch, each XCD on its own slice,
// instead of one pass per slice.  0: never (on the 4M-state workload the
// one-launch sweep over 8 slices of 4 MB took 12.2 ms, the 12 passes 11.6 ms);
// MDP_CB_PARTS_MAX_BYTES in the environment replaces it.
constexpr int64_t kCbXcdMaxBytes = 0;
constexpr int64_t kColBlockMinStates = int64_t{1} << 21;
constexpr int kMaxColBlocks = 64;
__host__ __device__ inline int sweep_tile_states(int A) { return A >= kSweepRows ? 1 : kSweepRows / A; }

// Row order of P on the device.  States are grouped in sweep tiles of
// T = sweep_tile_states(A) states; a tile's rows are contiguous and, inside
// the tile, action-major: (s, a) is row t0*A + a*n + (s - t0), where t0 is the
// tile's first state and n its number of states.  A policy that picks the
// same action for neighbouring states then selects neighbouring rows, so the
// policy products read fewer partly used lines; the sweep still streams every
// row once.
__host__ __device__ inline int64_t row_of(int64_t s, int a, int A, int64_t S) {
  const int T = sweep_tile_states(A);
  const int64_t t0 = (s / T) * T;
  const int64_t n = (S - t0) < T ? (S - t0) : T;
  return t0 * A + a * n + (s - t0);
}
// The state of a stored row.
__host__ __device__ inline int64_t state_of_row(int64_t r, int A, int64_t S) {
  const int T = sweep_tile_states(A);
  const int64_t t0 = (r / (static_cast<int64_t>(T) * A)) * T;
  const int64_t n = (S - t0) < T ? (S - t0) : T;
  return t0 + (r - t0 * A) % n;
}

// Allocation and release of device memory, pinned host memory, streams and
// events go through these wrappers (api.cpp), which hold the library's
// allocation lock in shared mode.  Graph capture in the batched solver holds
// it exclusively: such calls from another thread (hipFree waits for the whole
// device) would break a capture in progress.
std::shared_mutex& alloc_lock();
// Handle memory (api.cpp): from the handle's arena when it has one (and the
// arena has room), else from the library's per-device stream-ordered pool,
// allocated and freed on the handle's stream; an allocation is usable from any
// stream once handle_alloc returns.  A free is ordered after the work queued on
// the handle's stream, so work on other streams that touches the memory must
// be finished first.
hipError_t handle_alloc(mdp_handle* h, void** p, size_t bytes);
void handle_free(mdp_handle* h, void* p);
hipError_t device_pool(int dev, hipMemPool_t* out);
hipError_t lib_malloc(void** p, size_t bytes);
void lib_free(void* p);
hipError_t lib_host_malloc(void** p, size_t bytes);
void lib_host_free(void* p);

// Copies between the device and host memory (api.cpp).  Memory that HIP
// knows (device memory, pinned or registered host memory) is copied directly
// and asynchronously.  Plain pageable host memory is never handed to the
// runtime: it goes through pinned blocks of the library, in pieces whose host
// side overlaps the transfer of the previous piece, and the call returns once
// the copy is complete, so every transfer the library issues is a DMA between
// the device and memory the runtime knows.
bool host_pageable(const void* p);
hipError_t copy_in(void* dst, const void* src, size_t bytes, hipStream_t st);
hipError_t copy_out(void* dst, const void* src, size_t bytes, hipStream_t st);
// Pinned host blocks of kStageBlockBytes, with an event each, kept until the
// process ends: stage_take lends one (false when none can be had), stage_give
// takes it back once nothing in flight uses it.
constexpr size_t kStageBlockBytes = size_t{4} << 20;
struct StageBlock {
  char* p = nullptr;
  hipEvent_t ev = nullptr;
};
bool stage_take(StageBlock* b);
void stage_give(const StageBlock& b);
// XCD-partitioned P_pi products (xcdprod.hip).  pp_prepare forms the copy
// for policy pi when it is not current and sets h->pp_ready when the Arnoldi
// products can use it; launch_pp_arnoldi_apply is then the Arnoldi product of
// step j on the float64 or float32 basis (input U_j, or xin), with the plain
// product's outputs except that the dot partials come in *nb_dots tiles (the
// unsliced copy's product and dots run in one launch over its own tiles).  The copy keeps float64 values; a float32 basis is
// gathered in float32 and the slice parts summed in float64.
hipError_t pp_prepare(mdp_handle* h, const int32_t* pi);
// Frees the copy's arrays (queued on the handle's stream).
void pp_release(mdp_handle* h);
// Handles without a column-blocked copy get the contiguous copy when they
// hold at least kPolicyCopyMinStates states (below, forming it and its host
// check cost more than they save) and at most kPolicyCopyMaxRowMean entries
// per row on average.  On the 4M-state maze (4.2 entries per row) its product
// takes 163 us against 254 us through row_ptr; with 16 entries per row (the
// 1M-state workload) the row_ptr kernel, 16 lanes per row, is faster (81
// against 91 us).
constexpr int64_t kPolicyCopyMinStates = int64_t{1} << 17;
constexpr int64_t kPolicyCopyMaxRowMean = 8;
hipError_t launch_pp_arnoldi_apply(mdp_handle* h, bool basis_f32, int j, const void* xin, double* partials,
                                   int nb, int* nb_dots);
// One Horner step y = b + gamma P_pi x of the polynomial preconditioner on
// the copy (float64 or float32 vectors); ctl may be NULL.  y must be neither
// x nor b (on the unsliced copy one launch gathers x while it writes y).
hipError_t launch_pp_horner(mdp_handle* h, bool f32, const void* x, const void* b, void* y, const Ctl* ctl);
// The float64 product y = x - gamma P_pi x of BiCGSTAB and TFQMR on the
// copy (y must not be x); exits at once once ctl->done is set.
hipError_t launch_pp_op(mdp_handle* h, const double* x, double* y);
// The float64 residual g_pi - (x - gamma P_pi x) of a GMRES restart on the
// copy, into y (float64 or float32) with the per-tile (max, sum of squares)
// partials of the row_ptr kernel (nb tiles of kApplyTile states).
hipError_t launch_pp_residual(mdp_handle* h, const double* x, void* y, bool y_f32, double4* partials, int nb);

// dst[i] = src[i] for i < n, 64-bit row offsets narrowed to the stored 32-bit
// ones (values checked on the host beforehand) (vecops.hip).
hipError_t launch_narrow_offsets(hipStream_t st, const int64_t* src, int32_t* dst, int64_t n);

// Copy natural-order rows (s*A + a) into the stored order and write the
// stored row offsets rp_new[0..S*A] (vecops.hip).
hipError_t launch_permute_rows(hipStream_t st, int64_t S, int A, const int32_t* rp_old,
                               const int32_t* col_old, const double* val_old,
                               const double* cost_old, int32_t* rp_new, int32_t* col_new,
                               double* val_new, double* cost_new);
size_t partials_doubles(int64_t S, int A, int m);

// Host helpers shared by the single and the batched drivers (api.cpp).
bool is_device_ptr(const void* p);
// Sizes the kernels can index: A <= 4096, S*A < 2^31 - 1, S < 2^29 (gathers
// form 32-bit byte offsets into float64 vectors) and nnz <= kMaxNnz (row loops
// step an int32 entry index past a row's end by up to a wavefront).  nnz < 0:
// not known yet.  MDP_E_NOTSUP with a message otherwise.
constexpr int64_t kMaxStates = (int64_t{1} << 29) - 1;
constexpr int64_t kMaxNnz = (int64_t{1} << 31) - 4096;
mdp_status check_size_limits(int64_t S, int32_t A, int64_t nnz);
// Default lanes per CSR row for a mean row length (api.cpp).
int default_lanes(double mean_row);
// Validation (api.cpp): row_ptr structure; entries and costs on the host;
// both.  entry_failure turns a verdict into the shared message.
mdp_status validate_row_ptr(int64_t S, int32_t A, const int64_t* rp);
mdp_status validate_entries_host(int64_t S, int32_t A, const int64_t* rp, const int32_t* col,
                                 const double* val, const double* cost);
mdp_status entry_failure(int64_t cost_row, int64_t entry_row, int why);
// Entry checks on the device (vecops.hip): workgroup b writes out[3b..3b+2] =
// lowest row with a non-finite cost, lowest row with a bad entry or row sum,
// and that row's reason (1 column, 2 probability, 3 sum); -1 for none.
int validate_blocks(int64_t rows);
hipError_t launch_validate(hipStream_t st, int64_t S, int64_t rows, const int32_t* rp, const int32_t* col,
                           const double* val, const double* cost, int64_t* out, int blocks);
mdp_status validate_host(int64_t S, int32_t A, const int64_t* rp, const int32_t* col,
                         const double* val, const double* cost);
mdp_status sync_ctl(mdp_handle* h);
// Enqueue a copy of the control header into the host mirror, and wait for it.
mdp_status ctl_snapshot(mdp_handle* h);
mdp_status ctl_wait(mdp_handle* h);
mdp_status ensure_basis(mdp_handle* h, Prec prec, int m);
mdp_status ensure_lowp(mdp_handle* h, Prec prec);
Prec prec_of(int p);
int bval_of(Prec p);
double floor_of(Prec p);

// Algorithmic bytes of one launch (P_pi row count estimated by the mean row length).
double bytes_sweep(const mdp_handle* h, int bval, int bv, bool r0, int br);
double bytes_apply(const mdp_handle* h, int bval, int bx, int by);
double bytes_arnoldi_apply(const mdp_handle* h, int bval, int bb, int j);
double bytes_arnoldi_update(const mdp_handle* h, int bb, int j);

// Autotuner cache (tune.cpp): class key, stored lane width (0: none), store.
std::string tune_key(const mdp_handle* h);
int tune_lookup(const mdp_handle* h);
void tune_store(const mdp_handle* h, int lanes);
// The server tunes each new class once per process: tune_claim is true for the
// first caller of a class, which tunes and then calls tune_release; later
// callers of the class wait in tune_wait until the width is stored.
bool tune_claim(const mdp_handle* h);
void tune_release(const mdp_handle* h);
void tune_wait(const mdp_handle* h);

// Profiler hooks: bracket one launch with events when its class is selected.
void prof_begin(mdp_handle* h, int kind, hipEvent_t* a);
void prof_end(mdp_handle* h, int kind, hipEvent_t a, double bytes, int tag);
void prof_resolve(mdp_handle* h);
// Drop pending records from index `from` on whose tag is >= min_tag (Arnoldi
// steps enqueued past the end of a cycle exit at once and did no work).
void prof_discard_steps(mdp_handle* h, size_t from, int min_tag);

// K1 fused Bellman sweep on v (double* for kF64, float* otherwise) with the P
// copy of `prec`.  Writes Tv (may be null), pi (may be null) and r0 = Tv - v
// (may be null; float when r0_f32).  Then reduces max|Tv-v|, sum (Tv-v)^2 and
// max|Tv| into ctl with the given ReduceMode (kRedGmresStart starts a GMRES
// cycle from r0; first_cycle fixes the inner tolerance alpha*||r0||_2).
// Column-blocked float64 sweep (colblock.hip): build the blocked copy with
// `blocks` slices (returns false in *built when the rows do not allow it) and
// run a sweep over it with the arguments of launch_bellman.
// x <- -x on the stream (vecops.hip).
hipError_t launch_negate(hipStream_t st, double* x, int64_t n);

hipError_t build_colblocks(mdp_handle* h, int blocks, bool require, bool* built, double* far_frac);
hipError_t launch_bellman_cb(mdp_handle* h, const double* v, double* Tv, int32_t* pi, void* r0,
                             bool r0_f32, double4* part, int nb);
// The float64 sweep streamed tile by tile over the CSR rows (colblock.hip),
// for handles with h->flat_sweep.
hipError_t launch_bellman_flat(mdp_handle* h, const double* v, double* Tv, int32_t* pi, void* r0, bool r0_f32,
                               double4* part, int nb);

hipError_t launch_bellman(mdp_handle* h, Prec prec, const void* v, double* Tv, int32_t* pi,
                          void* r0, bool r0_f32, int red_mode, int first_cycle, double alpha,
                          double floor_rel);

// K2/K3/K10 float64 policy products (see ApplyMode); y is float when y_f32.
hipError_t launch_apply(mdp_handle* h, int mode, const int32_t* pi, const double* x, void* y,
                        bool y_f32, int red_mode, int first_cycle, double alpha,
                        double floor_rel);

// Richardson step on the ping-pong pair, early-exiting on ctl->done.
hipError_t launch_richardson_step(mdp_handle* h, const int32_t* pi, double* buf0, double* buf1);
// BiCGSTAB (krylov.hip) on (I - gamma P_pi) x = g_pi in float64.  The
// residual r0 sits in basis slot 0 and ctl holds its norm and the tolerance
// (kRedGmresStart); init sets up the shadow residual and the first direction,
// step enqueues one iteration (two products).  Slots 0..5 of the float64
// basis hold r, r^, p, v, s, t.
hipError_t launch_bicgstab_init(mdp_handle* h);
hipError_t launch_bicgstab_step(mdp_handle* h, const int32_t* pi, double* x);
// TFQMR (krylov.hip), same conventions; slots 0..7 hold r^, w, y1, y2, v, d,
// A y2, A y1.
hipError_t launch_tfqmr_init(mdp_handle* h, const int32_t* pi);
hipError_t launch_tfqmr_step(mdp_handle* h, const int32_t* pi, double* x);

// One Arnoldi step j (product + Gram-Schmidt + norm + Givens), early-exiting.
// deg > 1: right polynomial preconditioning, the product runs on
// M^-1 U_j = sum_{i<deg} (gamma P_pi)^i U_j (deg - 1 Horner steps in basis
// slots m + 1, m + 2; the basis must hold m + 4 slots).
// gs2: classical Gram-Schmidt with one re-orthogonalisation pass (CGS2): the
// updated vector's dots with the basis are taken again, added into the
// Hessenberg column and subtracted once more; ctl->orth_loss keeps the largest
// relative size of that second correction.
hipError_t launch_arnoldi_step(mdp_handle* h, Prec prec, const int32_t* pi, int j, int m, int deg = 1,
                               bool gs2 = false);
// End of a cycle with polynomial preconditioning: x += M^-1 (V y) (slots
// m + 1 .. m + 3).
hipError_t launch_precond_update_x(mdp_handle* h, Prec prec, const int32_t* pi, double* x, int m, int deg);

// x += V y over the completed columns of the current cycle.
hipError_t launch_gmres_update_x(mdp_handle* h, Prec prec, double* x);

hipError_t launch_check_policy(mdp_handle* h, const int32_t* pi);
hipError_t launch_ctl_reset(mdp_handle* h, double tol);
// Richardson start: tolerance, index of the buffer holding the iterate, steps done.
hipError_t launch_rich_begin(mdp_handle* h, double tol, int cur, int steps);
hipError_t launch_build_lowp(mdp_handle* h, int which);
hipError_t launch_cast_f32(hipStream_t st, const double* src, float* dst, int64_t n);
hipError_t launch_i64_to_i32(hipStream_t st, const int64_t* src, int32_t* dst, int64_t n);

}  // namespace mdp
