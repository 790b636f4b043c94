/*
 * mdp.h -- C ABI of the MI355X inexact-policy-iteration library.
 *
 * Problem (the paper's "Summary" and "Problem Setting and Solution Methods"
 * sections): an infinite-horizon discounted MDP with finite state space
 * {0..S-1}, finite action space {0..A-1}, stage costs g(s,a), discount
 * gamma in [0,1) and transition probabilities P[(s,a), s'].  The solver
 * minimises the expected discounted cumulative cost (or, on request,
 * maximises the expected discounted cumulative reward).  It uses inexact
 * policy iteration: a greedy improvement step (one Bellman sweep) alternates
 * with an approximate policy evaluation whose level of inexactness and inner
 * solver (restarted GMRES, Richardson, BiCGSTAB or TFQMR) the caller selects.
 *
 * Layout of an MDP handed to mdp_create ("Implementation" section: an MDP is
 * created from offline data):
 *   - rows r = s*A + a (state-major), S*A rows in total (this is the input
 *     order only: the library copies rows into an order of its own);
 *   - row_ptr: int64[S*A+1], CSR row offsets, row_ptr[0] = 0, nondecreasing,
 *     every row non-empty, row_ptr[S*A] = nnz;
 *   - col: int32[nnz], column (successor state) indices in [0,S);
 *   - val: double[nnz], probabilities, >= 0 and finite, each row summing to 1
 *     within 1e-12*max(1, row length);
 *   - cost: double[S*A], finite stage costs g(s,a), same row order.
 *
 * Pointers: every array argument may be host memory or device memory of the
 * handle's GPU; the library tells them apart with hipPointerGetAttributes.
 * Inputs are copied (the caller keeps ownership and may free them when the
 * call returns); outputs are caller-allocated.
 *
 * Errors: every call returns an mdp_status.  No call aborts or throws.  A
 * negative status leaves the outputs unspecified; mdp_last_error() returns a
 * thread-local message describing the last failure on this thread.
 *
 * Threads: a handle serves one call at a time; a call made while another is
 * running on the same handle returns MDP_E_STATE.
 */
#ifndef MDP_H
#define MDP_H

#include <stddef.h>
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

typedef struct mdp_handle* mdp_t;

typedef enum {
  MDP_OK = 0,
  MDP_W_MAXITER = 1,   /* iteration cap reached; outputs hold the last iterate */
  MDP_E_INVAL = -1,    /* invalid argument or invalid MDP data */
  MDP_E_NOMEM = -2,    /* device or host allocation failed */
  MDP_E_DEVICE = -3,   /* a HIP runtime call failed (also: no GPU present) */
  MDP_E_NUMERIC = -4,  /* NaN or Inf met in a residual */
  MDP_E_STATE = -5,    /* handle busy with another call */
  MDP_E_NOTSUP = -6    /* valid request the library does not support */
} mdp_status;

/* Arithmetic of the sweeps and of the inner solver. */
enum {
  MDP_FP64 = 0,        /* everything in float64 */
  MDP_MIXED_FP32 = 1,  /* P and vectors in float32 for inner sweeps/GMRES; float64 residuals and refinement */
  MDP_MIXED_FP16 = 2   /* as MIXED_FP32 but P held in float16 with a float64 per-row sum correction */
};

/* Objective of mdp_create_opts.objective. */
enum { MDP_MINIMIZE_COST = 0, MDP_MAXIMIZE_REWARD = 1 };

/* Inner solver of the approximate policy evaluation (the paper leaves the
 * choice of iterative solver for the linear system of policy evaluation open,
 * section "Problem Setting and Solution Methods"): restarted GMRES, the
 * Richardson / T_pi iteration, BiCGSTAB (van der Vorst 1992) or TFQMR (Freund
 * 1993; stops on its residual bound tau * sqrt(m + 1)). */
enum { MDP_INNER_GMRES = 0, MDP_INNER_RICHARDSON = 1, MDP_INNER_BICGSTAB = 2, MDP_INNER_TFQMR = 3 };

/* mdp_create_opts.validate.  row_ptr is checked on the host in every mode, before
 * any kernel reads a row.  MDP_VALIDATE_NONE leaves the entries and costs
 * unchecked; MDP_VALIDATE_HOST checks them on host threads (copying device inputs
 * to the host first); MDP_VALIDATE_DEVICE checks them in a kernel over the
 * uploaded copy, which spares the host a pass over the data.  The two checking
 * modes reject the same inputs with the same messages: both form a row's sum in
 * one fixed order (eight interleaved partial sums, each in entry order,
 * combined as ((p0+p4)+(p2+p6)) + ((p1+p5)+(p3+p7))). */
enum { MDP_VALIDATE_NONE = 0, MDP_VALIDATE_HOST = 1, MDP_VALIDATE_DEVICE = 2 };

/* Bits of mdp_create_opts.low_precision: which reduced-precision copies of P to build. */
enum { MDP_BUILD_FP32 = 1, MDP_BUILD_FP16 = 2 };

typedef struct {
  size_t struct_size;     /* sizeof(mdp_create_opts) */
  void* stream;           /* hipStream_t to run on; NULL: the handle creates its own stream */
  int32_t device;         /* HIP device ordinal; -1: the current device */
  int32_t validate;       /* MDP_VALIDATE_* (default MDP_VALIDATE_HOST): check the MDP data */
  int32_t low_precision;  /* MDP_BUILD_* bits (also built on first use by a mixed solve); the
                             float32 copy is packed per row, the float16 copy carries a float64
                             per-row correction */
  int32_t lanes_per_row;  /* 0: from the autotuner's cache, else from the mean row length;
                             otherwise a power of two in [2, 64] */
  int32_t col_blocks;     /* column-blocked copy of P for the float64 sweep: -1 (default)
                             builds one when S >= 2^21 and at least half of the entries lie
                             outside their row's column slice (slices of 3.25 MB of v); without
                             one, handles of at least 2^17 states with at most 8 entries per row
                             on average stream each tile's rows as one segment in the float64
                             sweep (no copy); 0: never either, every sweep gathers row by row;
                             n >= 1: always the blocked copy, with n slices (MDP_E_NOTSUP if a
                             row holds more than 255 entries of one slice, its columns are
                             not in increasing slice order, or A > 1024).  The blocked and
                             streamed sweeps take a row's sum as one fma chain (per slice), so
                             their rounding differs from the row-by-row sweep's within the
                             usual bound. */
  int32_t objective;      /* MDP_MINIMIZE_COST (default): minimise expected discounted cost, as
                             in the paper's problem statement; MDP_MAXIMIZE_REWARD: `cost`
                             holds rewards and every value vector passed in or out (v0, v,
                             Tv, x, y) is in reward terms.  Internally the rewards are stored
                             negated, so the two give bitwise the same arithmetic.  Batched
                             solves accept such handles; the server does not build them. */
} mdp_create_opts;

typedef struct {
  size_t struct_size;     /* sizeof(mdp_eval_opts) */
  int32_t inner;          /* MDP_INNER_GMRES, _RICHARDSON, _BICGSTAB or _TFQMR (BiCGSTAB and
                             TFQMR: float64 only, two products per iteration) */
  int32_t restart;        /* GMRES restart length m, 1..64 (default 30) */
  int32_t precision;      /* MDP_FP64, MDP_MIXED_FP32 or MDP_MIXED_FP16 */
  int32_t sync_every;     /* inner steps enqueued between host checks; 0: default */
  double rtol;            /* stop when ||r|| <= rtol*||r0|| (GMRES, BiCGSTAB: 2-norm of the
                             residual; Richardson: max-norm of successive differences) */
  int64_t max_iter;       /* cap on inner steps (default 10000) */
  int32_t precond_degree; /* GMRES only: 0 or 1 (default) no preconditioner; d in [2,16]: right
                             polynomial preconditioner M^-1 = sum_{i<d} (gamma P_pi)^i, the
                             first d terms of the Neumann series of (I - gamma P_pi)^-1, applied
                             matrix-free (d - 1 extra products with P_pi per Arnoldi step).
                             GMRES then works on (I - gamma P_pi) M^-1 = I - (gamma P_pi)^d
                             and still minimises the true residual.  MDP_E_NOTSUP with the
                             other inner solvers, batched solves and the server. */
  int32_t gs_passes;      /* GMRES Gram-Schmidt passes per Arnoldi step: 0 or 1 (default)
                             classical Gram-Schmidt (CGS), one pass over the basis; 2: CGS2,
                             which takes the dots of the orthogonalised vector once more and
                             subtracts them again, and reports the relative size of that
                             second correction (mdp_stats.orth_loss), the loss of orthogonality
                             a single pass would have left.  2 is MDP_E_NOTSUP with the other
                             inner solvers, batched solves and the server. */
  int32_t policy_copy;    /* GMRES (float64 or mixed float32), BiCGSTAB and TFQMR: -1 (default)
                             runs the inner solve's products on a copy of P_pi formed once per
                             policy (about S * 16 + nnz(P_pi) * 12 bytes more device memory), on
                             handles with a column-blocked copy (see mdp_create_opts.col_blocks)
                             cut into column slices, one per XCD, and on other handles of at
                             least 2^17 states with at most 8 entries per row on average stored
                             contiguously; 0 gathers the selected rows through row_ptr (as every
                             other product does: sweeps, Richardson, mdp_policy_apply).  The two
                             differ only in the rounding of each row's sum. */
} mdp_eval_opts;

typedef struct {
  size_t struct_size;     /* sizeof(mdp_solve_opts) */
  int32_t inner;          /* inner solver, as in mdp_eval_opts */
  int32_t restart;        /* GMRES restart length (default 30) */
  int32_t precision;      /* MDP_FP64, MDP_MIXED_FP32 or MDP_MIXED_FP16 */
  int32_t sync_every;     /* as in mdp_eval_opts */
  double alpha;           /* inner forcing term: inner stop at alpha * ||r0|| (default 1e-4) */
  double atol;            /* outer stop: ||T v - v||_inf <= atol (default 1e-8) */
  double rtol_cert;       /* if > 0, also require ||T v - v||_inf <= rtol_cert*(1-gamma)*||T v||_inf */
  int64_t max_outer;      /* cap on Bellman sweeps (default 1000) */
  int64_t max_inner;      /* cap on inner steps per evaluation (default 10000) */
  int32_t launch;         /* batched solves and the server: how a GMRES cycle's Arnoldi steps
                             reach the GPU.  MDP_LAUNCH_GRAPHS replays HIP graphs captured once
                             per configuration, with fixed persistent grids; MDP_LAUNCH_DIRECT
                             launches each kernel with a grid sized to the round's work.
                             MDP_LAUNCH_AUTO (the default) means graphs for mdp_solve_batch and
                             direct launches for the server, whose batches change with every
                             arrival.  Both give bitwise the same results.  mdp_solve ignores
                             it. */
  int32_t precond_degree; /* as in mdp_eval_opts (the paper leaves the inner solver, and so its
                             preconditioning, to the caller: "Problem Setting and Solution
                             Methods") */
  int32_t gs_passes;      /* as in mdp_eval_opts */
  int32_t policy_copy;    /* as in mdp_eval_opts (batched solves and the server ignore it) */
} mdp_solve_opts;

enum { MDP_LAUNCH_AUTO = 0, MDP_LAUNCH_GRAPHS = 1, MDP_LAUNCH_DIRECT = 2 };

typedef struct {
  size_t struct_size;     /* sizeof(mdp_stats) */
  int64_t outer_iters;    /* policy improvement steps (Bellman sweeps minus one) */
  int64_t inner_iters;    /* inner steps (Arnoldi or Richardson steps), summed */
  int64_t bellman_sweeps; /* Bellman sweeps of any precision */
  int64_t policy_applies; /* products with P_pi of any precision */
  int64_t refinements;    /* float64 residual refinements (mixed precision only) */
  double residual;        /* last ||T v - v||_inf (solve) or relative inner residual (eval) */
  double time_ms;         /* wall time of the call */
  double bytes;           /* algorithmic bytes moved by the call's kernels */
  double* history;        /* optional caller array receiving ||T v_k - v_k||_inf per sweep */
  int64_t history_cap;    /* its capacity */
  int64_t history_len;    /* entries written */
  double orth_loss;       /* gs_passes = 2: largest ||second-pass coefficients|| / ||w|| over the
                             Arnoldi steps of the call (0 otherwise) */
} mdp_stats;

/* Fill option structs with defaults. */
void mdp_default_create_opts(mdp_create_opts* o);
void mdp_default_eval_opts(mdp_eval_opts* o);
void mdp_default_solve_opts(mdp_solve_opts* o);

/* Create a handle from offline data (the paper's "Implementation" section
 * builds an MDP from offline data or from online simulation): copy the MDP
 * (layout above) to the device, optionally validate it, and build the
 * requested reduced-precision copies of P.  opt may be NULL (defaults).
 * Size limits (MDP_E_NOTSUP beyond them, checked before any array is read
 * past row_ptr[S*A]): A <= 4096, S*A < 2^31 - 1, S < 2^29 (the kernels form
 * 32-bit byte offsets into float64 vectors) and nnz <= 2^31 - 4096.  On
 * success *out owns all device memory of the MDP. */
mdp_status mdp_create(int64_t S, int32_t A, const int64_t* row_ptr, const int32_t* col,
                      const double* val, const double* cost, double gamma,
                      const mdp_create_opts* opt, mdp_t* out);

/* Rows of an MDP produced on demand, e.g. by a simulator (the paper builds
 * MDPs from offline data or from online simulation, section
 * "Implementation").  The function fills the rows of states [s_begin, s_end):
 * row i = (s - s_begin) * A + a holds len[i] <= k_max entries in
 * col[i * k_max + j], val[i * k_max + j] (j < len[i], columns increasing) and
 * the cost (or, with MDP_MAXIMIZE_REWARD, the reward) cost[i].  It returns 0,
 * or nonzero to abort the creation.  It is called from several host threads
 * at once, on disjoint state ranges. */
typedef int32_t (*mdp_rows_fn)(void* user, int64_t s_begin, int64_t s_end, int32_t k_max,
                               int32_t* col, double* val, int32_t* len, double* cost);

/* Create a handle from a row function: host threads (up to 16) call fn on
 * ranges of states, the rows are packed into CSR, validated as by mdp_create
 * when opt->validate is set, and copied to the device.  Host memory peaks at
 * about (S*A*k_max + nnz) * 12 bytes (the padded rows and the packed CSR).
 * MDP_E_INVAL when fn returns nonzero or a row is longer than k_max; other
 * errors as mdp_create. */
mdp_status mdp_create_from_rows(int64_t S, int32_t A, int32_t k_max, mdp_rows_fn fn, void* user,
                                double gamma, const mdp_create_opts* opt, mdp_t* out);

/* Rows of an MDP produced on the device by the caller's own kernel, e.g. a
 * simulator running one thread per state (the paper builds MDPs from online
 * simulation as well as from offline data, both in parallel, section
 * "Implementation").  The kernel takes this struct by value as its only
 * argument, extern "C" __global__ void k(mdp_device_rows_args a), and is
 * launched with 256 threads per workgroup and ceil((s_end - s_begin) / 256)
 * workgroups on a 1-D grid; thread blockIdx.x * 256 + threadIdx.x fills state
 * s = s_begin + that index when s < s_end.  For row i = (s - s_begin) * A + a
 * it writes len[i] in [1, k_max], col[i * k_max + j] (columns in [0, S),
 * increasing) and val[i * k_max + j] for j < len[i], and cost[i] (or, with
 * MDP_MAXIMIZE_REWARD, the reward).  All four arrays are device staging
 * owned by the library. */
typedef struct {
  int64_t S;
  int32_t A;
  int32_t k_max;
  int64_t s_begin, s_end;
  int32_t* col;
  double* val;
  int32_t* len;
  double* cost;
  const void* user;  /* the caller's pointer, passed through unchanged */
} mdp_device_rows_args;

/* Create a handle from a row kernel (a hipFunction_t, e.g. from
 * mdp_load_kernel or hipModuleGetFunction) on the device of opt (or the
 * current one): the library launches it into device staging of S*A*k_max
 * slots (at most 2^34), checks every length, turns the rows into CSR on the
 * device (a scan of the lengths, then a compaction) and builds the handle from
 * those device arrays as mdp_create does.  No row is formed on the host.
 * Validation follows opt->validate; with opt NULL it runs on the device.
 * MDP_E_INVAL when a length lies outside [1, k_max] or the launch fails; other
 * errors as mdp_create.  Staging is freed before the call returns. */
mdp_status mdp_create_from_device_rows(int64_t S, int32_t A, int32_t k_max, void* kernel,
                                       const void* user, double gamma, const mdp_create_opts* opt,
                                       mdp_t* out);

/* Load a code object (hipcc --genco, gfx950) and look up the kernel `name`
 * in it, for mdp_create_from_device_rows.  The module stays loaded until the
 * process ends.  MDP_E_INVAL when the file or the kernel is missing. */
mdp_status mdp_load_kernel(const char* code_object_path, const char* name, void** kernel);

/* One fused Bellman sweep in float64: the greedy (policy improvement) step of
 * policy iteration, section "Problem Setting and Solution Methods", applied to
 * the minimisation of discounted cost stated in the "Summary":
 *   Tv[s] = min_a g(s,a) + gamma * sum_j P[(s,a),j] v[j],
 *   policy[s] = the lowest action attaining the minimum,
 *   *res_inf = max_s |Tv[s] - v[s]|.
 * v: double[S].  Tv (double[S]), policy (int32[S]) and res_inf may be NULL. */
mdp_status mdp_bellman(mdp_t h, const double* v, double* Tv, int32_t* policy, double* res_inf);

/* For callers that cannot allocate device memory (code under HIP graph
 * capture, tight serving loops, harnesses that forbid hipMalloc): the sweep of
 * mdp_bellman on the caller's own device arrays, with no handle and no
 * allocation.  The per-workgroup partials go to a fixed device array of the
 * library (2 MiB per GPU, held until the process ends).
 *   row_ptr int64[S*A+1], col int32[nnz], val double[nnz], cost double[S*A]:
 *     the MDP in the input layout of mdp_create (rows r = s*A + a), NOT
 *     validated here (validate it once with mdp_create or on the host);
 *   v double[S]; Tv double[S], policy int32[S] and res_inf double[1] may each
 *     be NULL; Tv must not alias v;
 *   lanes_per_row: 0 (from the mean row length) or a power of two in [2,64];
 *     with the width of a handle (mdp_info) the results are bitwise those of
 *     mdp_bellman on that handle;
 *   stream: hipStream_t (NULL: the null stream).
 * Every pointer must be device memory of the current device (else
 * MDP_E_INVAL).  The call only enqueues work on the stream and returns; the
 * outputs are ready when the stream reaches that point.  It calls no
 * allocator.  Limits: S*A rows in at most 65536 sweep tiles (about 2^26 rows,
 * MDP_E_NOTSUP beyond) and the size limits of mdp_create.  All calls on one
 * GPU share the partials array: calls that overlap in time on one GPU (two
 * streams, two threads) race and must be serialised by the caller. */
mdp_status mdp_bellman_noalloc(int64_t S, int32_t A, int64_t nnz, const int64_t* row_ptr,
                               const int32_t* col, const double* val, const double* cost,
                               double gamma, const double* v, double* Tv, int32_t* policy,
                               double* res_inf, int32_t lanes_per_row, void* stream);

/* Product with the transition matrix of a policy, gathering rows s*A+policy[s]
 * of P without forming P_pi: the operator of the linear system that policy
 * evaluation solves (section "Problem Setting and Solution Methods"):
 *   mode 0: y = x - gamma * P_pi x         ((I - gamma P_pi) x)
 *   mode 1: y = g_pi + gamma * P_pi x      (T_pi x)
 * policy: int32[S] with entries in [0,A) (else MDP_E_INVAL); x, y: double[S]. */
mdp_status mdp_policy_apply(mdp_t h, const int32_t* policy, const double* x, double* y,
                            int32_t mode);

/* Approximate policy evaluation (section "Problem Setting and Solution
 * Methods": the inexact evaluation step of iPI, with a caller-chosen inner
 * iterative solver and level of inexactness): solve (I - gamma P_pi) v = g_pi
 * starting from v0 (NULL: zero) with the inner solver and tolerance of opt
 * (NULL: defaults).
 * v: double[S] output.  stats may be NULL.  Returns MDP_W_MAXITER when the
 * tolerance was not met within max_iter steps. */
mdp_status mdp_policy_eval(mdp_t h, const int32_t* policy, const double* v0, double* v,
                           const mdp_eval_opts* opt, mdp_stats* stats);

/* Inexact policy iteration (section "Problem Setting and Solution Methods":
 * greedy steps alternating with approximate evaluations; value iteration and
 * modified policy iteration are the special cases of Richardson inner solves
 * with one or a fixed number of steps) from v0 (NULL: zero).  Stops at the first sweep
 * with ||T v_k - v_k||_inf <= atol (and the certified relative test if
 * rtol_cert > 0); returns v = v_k and policy = the greedy policy of v_k.
 * Returns MDP_W_MAXITER with the last iterate after max_outer sweeps. */
mdp_status mdp_solve(mdp_t h, const double* v0, double* v, int32_t* policy,
                     const mdp_solve_opts* opt, mdp_stats* stats);

/* Batched inexact policy iteration (an extension: the paper defines no
 * batched or served solve; each MDP follows mdp_solve): solve n MDPs (handles
 * on one device) together.  Each round advances every unfinished MDP by one phase (a Bellman
 * sweep, or one GMRES cycle with its restart) in persistent kernels that walk
 * a table of (MDP, tile) work items; the cycle's Arnoldi steps are replayed
 * from captured HIP graphs (see mdp_solve_opts.launch).  The engine and its
 * graphs are kept per device between calls, so only the first call of a
 * configuration captures.  Every MDP gets bitwise the same v, policy and
 * statistics as mdp_solve would give it alone (same kernels bodies, tiling,
 * reduction order and decisions).  v0 may be NULL (all zero) or hold n
 * pointers (each NULL or double[S_i]); v[i] (double[S_i]) and policy[i]
 * (int32[S_i]) receive the results; stats may be NULL or point to n structs.
 * GMRES only (MDP_E_NOTSUP for Richardson).  Runs on handles[0]'s stream. */
mdp_status mdp_solve_batch(mdp_t* handles, int32_t n, const double* const* v0, double* const* v,
                           int32_t* const* policy, const mdp_solve_opts* opt, mdp_stats* stats);

/* ---- serving: continuous batching of solve requests ----------------------
 * An extension the paper does not define: requests are solved as by
 * mdp_solve_batch.  A server owns worker threads on one GPU.  Submitted MDPs wait in a queue;
 * the server admits them in order while the estimated device footprint of the resident
 * set stays within hbm_budget_bytes and at most max_batch are resident (when the
 * request at the head does not fit, later ones that fit may pass it, up to 64
 * times, after which it waits for room), keeps
 * admitted MDPs and their iterates resident, and advances all of them with
 * the batched engine (see mdp_solve_batch), one round at a time.  Requests
 * that arrive while others run join at the next round; finished ones leave,
 * freeing their memory.  A request's v and policy are bitwise those of
 * mdp_solve on the same MDP with the server's solve options. */
typedef struct mdp_server* mdp_server_t;

typedef struct {
  size_t struct_size;        /* sizeof(mdp_server_opts) */
  void* stream;              /* hipStream_t for the worker; NULL: its own */
  int64_t hbm_budget_bytes;  /* admission limit on resident device bytes (default 64 GiB).  The
                                server reserves the budget plus a quarter (for the staging of
                                admissions in flight) as one device allocation when it starts,
                                less when the device has less free memory, and places admitted
                                MDPs in it, so that admitting and retiring never call the HIP
                                allocator; what does not fit there comes from the library's
                                device pool */
  int32_t device;            /* HIP device; -1: the current device */
  int32_t max_batch;         /* most MDPs resident at once (default 256) */
  int32_t admit_threads;     /* threads copying new MDPs to the device (default 4: while one
                                waits for its upload, the others queue theirs) */
  int32_t retire_threads;    /* threads copying results out and freeing (default 4) */
  mdp_solve_opts solve;      /* GMRES only; default precision MDP_MIXED_FP32 */
  int32_t autotune;          /* 1: the first request of a class with no remembered lane width
                                (see mdp_autotune) is timed at admission and its width stored,
                                once per class and process; later requests of the class start
                                from it.  0 (default): widths come from the cache or the mean
                                row length only.  Results stay those of mdp_solve on a handle
                                created with the same width. */
  int64_t split_nnz;         /* size classes: requests of at most split_nnz nonzeros are advanced
                                by one worker, larger ones by a second worker on its own stream,
                                so that a small request's rounds do not wait for a large
                                request's GMRES cycles (default 2^24; 0: one worker for all).
                                Results do not depend on the class. */
  const char* trace_path;    /* non-NULL: the server times each admission (handle created, lane
                                width known, end; with the bytes in use in the server's
                                allocation and the free device bytes at its start), each round (sweep phase end,
                                MDPs advanced, swept and finished) and each retirement, in ms
                                since its creation, and writes them to this file, one JSON
                                object a line, when it is destroyed (default NULL: no trace) */
} mdp_server_opts;

typedef struct {
  size_t struct_size;        /* sizeof(mdp_request_stats) */
  double submit_ms;          /* server clock (ms since creation) at submission */
  double admit_ms;           /* ... when the MDP became resident */
  double finish_ms;          /* ... when its result was ready */
  int64_t outer_iters, inner_iters, bellman_sweeps;
  double residual;           /* final ||T v - v||_inf */
  double bytes;              /* algorithmic bytes of its kernels */
} mdp_request_stats;

void mdp_default_server_opts(mdp_server_opts* o);
mdp_status mdp_server_create(const mdp_server_opts* opt, mdp_server_t* out);
/* Queue a solve.  The MDP (host arrays, layout as for mdp_create) is copied
 * and validated-by-shape at submission; *request_id identifies it.
 * MDP_E_NOMEM if its footprint alone exceeds the budget. */
mdp_status mdp_server_submit(mdp_server_t s, int64_t S, int32_t A, const int64_t* row_ptr,
                             const int32_t* col, const double* val, const double* cost,
                             double gamma, int64_t* request_id);
/* As mdp_server_submit, without the copy: the arrays are read (and
 * validated) when the request is admitted, so the caller keeps them valid and
 * unchanged until mdp_server_wait returns for this request.  An invalid MDP
 * then fails at mdp_server_wait with MDP_E_INVAL. */
mdp_status mdp_server_submit_borrowed(mdp_server_t s, int64_t S, int32_t A,
                                      const int64_t* row_ptr, const int32_t* col,
                                      const double* val, const double* cost, double gamma,
                                      int64_t* request_id);
/* *done = 1 once the request's result is ready. */
mdp_status mdp_server_poll(mdp_server_t s, int64_t request_id, int32_t* done);
/* Block until the request is done, copy v (double[S]) and policy (int32[S])
 * to host memory (either may be NULL), fill stats (may be NULL) and forget
 * the request.  Returns the request's solve status. */
mdp_status mdp_server_wait(mdp_server_t s, int64_t request_id, double* v, int32_t* policy,
                           mdp_request_stats* stats);
/* Queue length, resident count and bytes, rounds run so far (any may be NULL). */
mdp_status mdp_server_info(mdp_server_t s, int64_t* queued, int64_t* resident,
                           int64_t* resident_bytes, int64_t* rounds);
/* Finish the resident requests, drop queued ones, stop the worker, free all. */
mdp_status mdp_server_destroy(mdp_server_t s);

/* Sizes and placement of a handle (any pointer may be NULL). */
mdp_status mdp_info(mdp_t h, int64_t* S, int32_t* A, int64_t* nnz, int32_t* lanes_per_row,
                    int64_t* device_bytes);

/* Choose lanes_per_row for this handle by timing candidate widths on the
 * device (one sweep plus four policy products per width, each width timed in
 * three rounds and kept at its shortest time, since work sharing the GPU only
 * lengthens a timing; the width that covers the mean row length is kept
 * unless another is more than 5% faster); writes the chosen
 * width to *lanes (may be NULL) and remembers it for the handle's class (GPU
 * architecture, action count and mean row length, each rounded up to a power
 * of two, and the nonzero count within a factor of 16) in $MDP_TUNE_CACHE (default $HOME/.cache/mdp_mi355x_tune.json).
 * mdp_create with lanes_per_row = 0 starts from a remembered width. */
mdp_status mdp_autotune(mdp_t h, int32_t* lanes);

/* Kernel classes reported by the profiler. */
enum {
  MDP_K_BELLMAN = 0,         /* fused Bellman sweep */
  MDP_K_ARNOLDI_APPLY = 1,   /* P_pi product fused with the Gram-Schmidt dot products */
  MDP_K_ARNOLDI_UPDATE = 2,  /* Gram-Schmidt update and norm */
  MDP_K_POLICY_APPLY = 3,    /* P_pi products: operator, T_pi (Richardson), residual */
  MDP_K_GMRES_UPDATE_X = 4,  /* x += V y at the end of a GMRES cycle */
  MDP_K_REDUCE = 5,          /* single-workgroup reductions, Givens rotations */
  MDP_K_OTHER = 6,           /* casts, conversions, checks */
  MDP_NUM_KERNEL_KINDS = 7
};

typedef struct {
  size_t struct_size;                        /* sizeof(mdp_kernel_profile) */
  int64_t launches[MDP_NUM_KERNEL_KINDS];    /* kernel launches per class */
  double ms[MDP_NUM_KERNEL_KINDS];           /* summed kernel durations (HIP events on the handle's stream) */
  double bytes[MDP_NUM_KERNEL_KINDS];        /* summed algorithmic bytes of those launches */
} mdp_kernel_profile;

/* Start (counters cleared) or stop recording a HIP event pair around kernel
 * launches of the handle: enable < 0 records every class, enable > 0 is a
 * bit mask (bit k records class k), 0 stops.  Arnoldi steps enqueued past
 * the end of a GMRES cycle exit at once and are not counted. */
mdp_status mdp_profile(mdp_t h, int32_t enable);

/* As mdp_profile, but only the first of every `every` launches (>= 1) of each
 * class gets its event pair, so that a timed run pays for few of the
 * event records (each costs a few microseconds of idle GPU time). */
mdp_status mdp_profile_sampled(mdp_t h, int32_t enable, int32_t every);

/* Wait for the recorded launches and return the accumulated counters. */
mdp_status mdp_profile_read(mdp_t h, mdp_kernel_profile* out);

/* Release a handle and all of its device memory.  NULL is accepted. */
mdp_status mdp_destroy(mdp_t h);

/* Message for the last failure on the calling thread ("" if none). */
const char* mdp_last_error(void);

/* Library version string. */
const char* mdp_version(void);

#ifdef __cplusplus
}
#endif

#endif /* MDP_H */
