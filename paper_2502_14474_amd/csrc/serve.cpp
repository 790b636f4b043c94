// Serving loop: continuous batching of MDP solve requests on one GPU.
//
// Submitted requests wait in a host queue.  A worker thread admits them while
// the estimated device footprint of the resident set stays within the HBM
// budget (and the resident count within max_batch), keeps each admitted MDP's
// CSR data and iterates resident, and advances all resident MDPs together one
// round at a time with the batch engine.  Requests that arrive while others
// are on the GPU join at the next round boundary; finished ones are copied
// out, their memory released, and their slots reused.  Because the batch
// engine is batch-invariant, a request's result does not depend on what else
// was resident.
#include <algorithm>
#include <chrono>
#include <condition_variable>
#include <cstring>
#include <cstdio>
#include <deque>
#include <limits>
#include <map>
#include <memory>
#include <mutex>
#include <shared_mutex>
#include <string>
#include <thread>
#include <vector>

#include "batch.h"
#include "internal.h"

namespace mdp {

struct Request {
  int64_t id = 0;
  int64_t S = 0;
  int32_t A = 0;
  double gamma = 0;
  std::vector<int64_t> row_ptr;
  std::vector<int32_t> col;
  std::vector<double> val, cost;
  // borrowed submission: caller arrays, read at admission
  const int64_t* b_row_ptr = nullptr;
  const int32_t* b_col = nullptr;
  const double* b_val = nullptr;
  const double* b_cost = nullptr;
  bool borrowed = false;
  int64_t footprint = 0;
  int lane = 0;  // the worker (size class) that advances it
  int passed = 0;  // times a later request was admitted ahead of it
  // results
  std::vector<double> v;
  std::vector<int32_t> pi;
  mdp_request_stats st{};
  bool done = false;
  mdp_status status = MDP_OK;
  std::string error;
  // while resident
  mdp_handle* h = nullptr;
  BatchItem item;
};

static double clock_ms() {
  using namespace std::chrono;
  return duration<double, std::milli>(steady_clock::now().time_since_epoch()).count();
}

// One timed event of the server's trace: an admission (t[0] start, t[1]
// handle created, t[2] lane width known, t[3] end; n[0] nonzeros, n[1]
// states, n[2] lane width, n[3] bytes in use in the server's arena (without
// one: held by the device pool) and n[4] free device bytes at the start), a
// round (t[0] start, t[1] sweep phase done,
// t[3] end; n[0] MDPs advanced, n[1] of them swept, n[2] finished) or a
// retirement (t[0] start, t[1] results on the host, t[3] end).  Times are
// milliseconds since the server's creation.
struct TraceEvent {
  char kind = 0;  // 'a', 'r' or 'x'
  int lane = 0;
  int64_t id = 0;
  double t[4] = {0, 0, 0, 0};
  int64_t n[5] = {0, 0, 0, 0, 0};
};

// Device bytes a request will hold while resident (CSR, costs, vectors,
// GMRES basis, reduced-precision copies, partials).
static int64_t footprint_of(int64_t S, int32_t A, int64_t nnz, const mdp_solve_opts& o) {
  const int64_t rows = S * A;
  const int64_t ldu = (S + 255) / 256 * 256;
  const bool mixed = o.precision != MDP_FP64;
  int64_t b = nnz * 12 + (rows + 1) * 4 + rows * 8;          // CSR + costs
  b += S * (8 * 4 + 4 * 2);                                   // v, Tv, x2, io, pi, pi_io
  b += static_cast<int64_t>(o.restart + 1) * ldu * (mixed ? 4 : 8);
  if (o.precision == MDP_MIXED_FP32) b += nnz * 8 + S * 4;  // packed columns + float32 values
  if (o.precision == MDP_MIXED_FP16) b += nnz * 2 + rows * 8 + S * 4;
  b += static_cast<int64_t>(partials_doubles(S, A, kMaxRestart)) * 8 + sizeof(Ctl);
  return b;
}

}  // namespace mdp

// One worker of the server: its own batch engine, stream and resident set.
// Workers serve size classes (small and large requests), so a small request
// never waits for a large one's GMRES cycle inside a round.
struct ServerLane {
  hipStream_t stream = nullptr;
  bool own_stream = false;
  mdp::BatchEngine eng;
  std::vector<mdp::Request*> ready;     // admitted, joining at the next round
  std::vector<mdp::Request*> resident;  // advanced by the rounds
  std::thread thread;
  int64_t rounds = 0;
  int index = 0;
};

struct mdp_server {
  mdp_server_opts opts{};
  int device = 0;
  std::mutex mu;
  std::condition_variable cv_admit, cv_work, cv_reap, cv_done;
  std::deque<mdp::Request*> queue;     // submitted, not yet admitted
  std::vector<std::unique_ptr<ServerLane>> lanes;
  std::deque<mdp::Request*> retiring;  // finished, results being copied out
  std::map<int64_t, std::unique_ptr<mdp::Request>> all;
  int64_t next_id = 1;
  int64_t held_bytes = 0;              // footprint of admitting + resident + retiring
  int admitting = 0;
  bool stop = false;
  int workers_left = 0;
  double t0 = 0;
  std::vector<std::thread> admitters, reapers;
  int reapers_left = 0;
  mdp::DeviceArena* arena = nullptr;  // where admitted MDPs live (nullptr: the device pool)
  bool tracing = false;
  std::string trace_path;
  std::mutex trace_mu;
  std::vector<mdp::TraceEvent> trace;
  double now() const { return mdp::clock_ms() - t0; }
  void record(const mdp::TraceEvent& e) {
    std::lock_guard<std::mutex> g(trace_mu);
    trace.push_back(e);
  }
  void write_trace();

  void admit_loop();
  void work_loop(ServerLane* ln);
  void reap_loop();
  mdp_status admit_one(mdp::Request* r);
  void retire(mdp::Request* r);
  int in_flight() const {
    int n = admitting;
    for (const auto& l : lanes) n += static_cast<int>(l->ready.size() + l->resident.size());
    return n;
  }
};

using namespace mdp;

// Admission runs beside the rounds: device allocations and host-to-device
// copies of a new MDP happen on its own stream while the worker keeps the
// resident set busy.  A request is admitted while the held footprint
// (admitting + resident + retiring) stays within the budget, or when nothing
// is held at all.
void mdp_server::admit_loop() {
  (void)hipSetDevice(device);
  ArenaScope in_arena(arena);
  std::unique_lock<std::mutex> lk(mu);
  // The queue is served in order, except that while the request at its head
  // does not fit the budget, later requests that fit may pass it, at most
  // kMaxPasses times (then the head waits for room): a large request does not
  // hold up the small ones behind it, and is not starved by them either.
  constexpr int kMaxPasses = 64;
  auto pick = [&]() -> std::deque<Request*>::iterator {
    if (queue.empty() || in_flight() >= opts.max_batch) return queue.end();
    auto fits = [&](const Request* r) { return held_bytes == 0 || held_bytes + r->footprint <= opts.hbm_budget_bytes; };
    if (fits(queue.front())) return queue.begin();
    if (queue.front()->passed >= kMaxPasses) return queue.end();
    for (auto it = std::next(queue.begin()); it != queue.end(); ++it)
      if (fits(*it)) return it;
    return queue.end();
  };
  for (;;) {
    std::deque<Request*>::iterator it;
    cv_admit.wait(lk, [&]() { return stop || (it = pick()) != queue.end(); });
    if (stop) return;
    Request* r = *it;
    if (it != queue.begin()) ++queue.front()->passed;
    queue.erase(it);
    held_bytes += r->footprint;
    ++admitting;
    lk.unlock();
    const mdp_status st = admit_one(r);
    lk.lock();
    --admitting;
    if (st < 0) {
      held_bytes -= r->footprint;
      r->status = st;
      r->error = mdp_last_error();
      r->done = true;
      r->st.finish_ms = clock_ms() - t0;
      cv_done.notify_all();
      cv_admit.notify_all();
      continue;
    }
    lanes[r->lane]->ready.push_back(r);
    cv_work.notify_all();
  }
}

void mdp_server::work_loop(ServerLane* ln) {
  (void)hipSetDevice(device);
  std::unique_lock<std::mutex> lk(mu);
  for (;;) {
    cv_work.wait(lk, [&]() { return !ln->ready.empty() || !ln->resident.empty() || (stop && admitting == 0); });
    for (Request* r : ln->ready) ln->resident.push_back(r);
    ln->ready.clear();
    if (ln->resident.empty()) {
      if (stop && admitting == 0) break;
      continue;
    }
    // one round over this worker's resident set
    ln->eng.items.clear();
    for (Request* r : ln->resident) ln->eng.items.push_back(&r->item);
    TraceEvent ev;
    if (tracing) {
      ev.kind = 'r';
      ev.lane = ln->index;
      ev.id = ln->rounds;
      ev.n[0] = static_cast<int64_t>(ln->resident.size());
      ev.t[0] = now();
    }
    lk.unlock();
    const mdp_status st = ln->eng.round(opts.solve);
    lk.lock();
    ++ln->rounds;
    if (st < 0) {
      // the message goes into each request under the lock, so that the
      // reapers (which run unlocked) only read what was handed to them
      const std::string msg = mdp_last_error();
      for (Request* r : ln->resident) {
        r->item.status = st;
        r->item.state = BatchItem::kDone;
        r->error = msg;
      }
    }
    std::vector<Request*> keep;
    for (Request* r : ln->resident) {
      if (r->item.state == BatchItem::kDone) retiring.push_back(r);
      else keep.push_back(r);
    }
    if (tracing) {
      ev.t[1] = ln->eng.last_sweep_end_ms - t0;
      ev.t[3] = now();
      ev.n[1] = ln->eng.last_swept;
      ev.n[2] = static_cast<int64_t>(ln->resident.size() - keep.size());
      record(ev);
    }
    ln->resident.swap(keep);
    cv_reap.notify_all();
  }
  --workers_left;
  cv_reap.notify_all();
}

// Retirement copies results out and frees device memory off the round loop.
void mdp_server::reap_loop() {
  (void)hipSetDevice(device);
  std::unique_lock<std::mutex> lk(mu);
  for (;;) {
    cv_reap.wait(lk, [&]() { return !retiring.empty() || workers_left == 0; });
    if (retiring.empty() && workers_left == 0) {
      --reapers_left;
      return;
    }
    Request* r = retiring.front();
    retiring.pop_front();
    lk.unlock();
    retire(r);
    lk.lock();
    held_bytes -= r->footprint;
    r->done = true;
    cv_done.notify_all();
    cv_admit.notify_all();
  }
}

mdp_status mdp_server::admit_one(Request* r) {
  TraceEvent ev;
  ev.kind = 'a';
  ev.lane = r->lane;
  ev.id = r->id;
  ev.t[0] = now();
  if (tracing) {
    hipMemPool_t pool = nullptr;
    uint64_t held = 0;
    size_t fr = 0, tot = 0;
    if (arena)
      ev.n[3] = static_cast<int64_t>(arena->in_use());
    else if (device_pool(device, &pool) == hipSuccess &&
             hipMemPoolGetAttribute(pool, hipMemPoolAttrReservedMemCurrent, &held) == hipSuccess)
      ev.n[3] = static_cast<int64_t>(held);
    if (hipMemGetInfo(&fr, &tot) == hipSuccess) ev.n[4] = static_cast<int64_t>(fr);
    (void)hipGetLastError();
  }
  mdp_create_opts co;
  mdp_default_create_opts(&co);
  co.stream = nullptr;  // the handle's own stream: admission overlaps the rounds
  co.device = device;
  // copied requests were validated at submission; lent arrays are checked
  // here, on the device, over the uploaded copy
  co.validate = r->borrowed ? MDP_VALIDATE_DEVICE : MDP_VALIDATE_NONE;
  mdp_handle* h = nullptr;
  const int64_t* rp = r->borrowed ? r->b_row_ptr : r->row_ptr.data();
  const int32_t* cl = r->borrowed ? r->b_col : r->col.data();
  const double* vl = r->borrowed ? r->b_val : r->val.data();
  const double* cs = r->borrowed ? r->b_cost : r->cost.data();
  MDP_TRY(mdp_create(r->S, r->A, rp, cl, vl, cs, r->gamma, &co, &h));
  r->h = h;
  ev.t[1] = now();
  ev.n[0] = h->nnz;
  ev.n[1] = h->S;
  // a class seen for the first time: time its lane widths once, on this MDP;
  // requests of the class admitted meanwhile wait for the stored width, so
  // that every request of a class runs with the same width
  if (opts.autotune && tune_lookup(h) == 0) {
    if (tune_claim(h)) {
      const mdp_status ts = mdp_autotune(h, nullptr);
      tune_release(h);
      if (ts < 0) {
        mdp_destroy(h);
        r->h = nullptr;
        return ts;
      }
    } else {
      tune_wait(h);
      if (const int L = tune_lookup(h)) h->lanes = L;
    }
  }
  ev.t[2] = now();
  ev.n[2] = h->lanes;
  const Prec prec = prec_of(opts.solve.precision);
  mdp_status st = ensure_basis(h, prec == kF64 ? kF64 : kF32, opts.solve.restart);
  if (st >= 0 && prec != kF64) st = ensure_lowp(h, prec);
  if (st < 0) {
    mdp_destroy(h);
    r->h = nullptr;
    return st;
  }
  hipError_t e = hipMemsetAsync(h->v, 0, h->S * sizeof(double), h->stream);
  if (e == hipSuccess) e = launch_ctl_reset(h, 0.0);
  if (e == hipSuccess) e = hipStreamSynchronize(h->stream);
  if (e != hipSuccess) {
    mdp_destroy(h);
    r->h = nullptr;
    return fail(MDP_E_DEVICE, std::string("admission: ") + hipGetErrorString(e));
  }
  // host copies are no longer needed once the MDP is resident
  std::vector<int64_t>().swap(r->row_ptr);
  std::vector<int32_t>().swap(r->col);
  std::vector<double>().swap(r->val);
  std::vector<double>().swap(r->cost);
  BatchItem& it = r->item;
  it = BatchItem();
  it.h = h;
  it.alpha = opts.solve.alpha;
  it.prev_res = std::numeric_limits<double>::infinity();
  it.prev_lowp_res = std::numeric_limits<double>::infinity();
  it.lowp_sweep = prec != kF64;
  r->st.admit_ms = clock_ms() - t0;
  if (tracing) {
    ev.t[3] = r->st.admit_ms;
    record(ev);
  }
  return MDP_OK;
}

void mdp_server::retire(Request* r) {
  TraceEvent ev;
  ev.kind = 'x';
  ev.lane = r->lane;
  ev.id = r->id;
  ev.t[0] = now();
  mdp_handle* h = r->h;
  const BatchItem& it = r->item;
  r->v.resize(h->S);
  r->pi.resize(h->S);
  // the worker synchronised its stream before handing the request over
  hipError_t e = copy_out(r->v.data(), h->v, h->S * sizeof(double), h->stream);
  if (e == hipSuccess) e = copy_out(r->pi.data(), h->pi, h->S * sizeof(int32_t), h->stream);
  if (e == hipSuccess) e = hipStreamSynchronize(h->stream);
  r->st.finish_ms = clock_ms() - t0;  // results are on the host
  r->status = e != hipSuccess ? MDP_E_DEVICE : it.status;
  if (e != hipSuccess) r->error = hipGetErrorString(e);
  else if (it.status < 0 && r->error.empty()) r->error = "non-finite residual";
  r->st.outer_iters = it.k;
  r->st.inner_iters = it.inner;
  r->st.bellman_sweeps = it.sweeps;
  r->st.residual = it.res;
  r->st.bytes = it.bytes;
  ev.t[1] = r->st.finish_ms;
  mdp_destroy(h);
  r->h = nullptr;
  if (tracing) {
    ev.t[3] = now();
    record(ev);
  }
}

void mdp_server::write_trace() {
  FILE* f = std::fopen(trace_path.c_str(), "w");
  if (!f) return;
  for (const TraceEvent& e : trace)
    std::fprintf(f,
                 "{\"kind\": \"%c\", \"lane\": %d, \"id\": %lld, \"t\": [%.3f, %.3f, %.3f, %.3f], "
                 "\"n\": [%lld, %lld, %lld, %lld, %lld]}\n",
                 e.kind, e.lane, static_cast<long long>(e.id), e.t[0], e.t[1], e.t[2], e.t[3],
                 static_cast<long long>(e.n[0]), static_cast<long long>(e.n[1]), static_cast<long long>(e.n[2]),
                 static_cast<long long>(e.n[3]), static_cast<long long>(e.n[4]));
  std::fclose(f);
}

extern "C" {

void mdp_default_server_opts(mdp_server_opts* o) {
  if (!o) return;
  std::memset(o, 0, sizeof(*o));
  o->struct_size = sizeof(*o);
  o->device = -1;
  o->stream = nullptr;
  o->hbm_budget_bytes = int64_t{64} << 30;
  o->max_batch = 256;
  o->admit_threads = 4;
  o->retire_threads = 4;
  o->split_nnz = int64_t{1} << 24;
  mdp_default_solve_opts(&o->solve);
  o->solve.precision = MDP_MIXED_FP32;
}

mdp_status mdp_server_create(const mdp_server_opts* opt, mdp_server_t* out) {
  clear_error();
  if (!out) return fail(MDP_E_INVAL, "out is NULL");
  *out = nullptr;
  mdp_server_opts o;
  mdp_default_server_opts(&o);
  if (opt) {
    if (opt->struct_size < sizeof(mdp_server_opts)) return fail(MDP_E_INVAL, "mdp_server_opts.struct_size too small");
    o = *opt;
  }
  if (o.split_nnz < 0) return fail(MDP_E_INVAL, "split_nnz must be >= 0");
  if (o.max_batch < 1 || o.max_batch > 65536 || o.hbm_budget_bytes <= 0 ||
      o.admit_threads < 1 || o.admit_threads > 64 || o.retire_threads < 1 || o.retire_threads > 64)
    return fail(MDP_E_INVAL, "bad server limits");
  if (o.solve.inner != MDP_INNER_GMRES) return fail(MDP_E_NOTSUP, "the server uses GMRES");
  if (o.solve.launch < MDP_LAUNCH_AUTO || o.solve.launch > MDP_LAUNCH_DIRECT)
    return fail(MDP_E_INVAL, "unknown launch mode");
  if (o.solve.restart < 1 || o.solve.restart > kMaxRestart) return fail(MDP_E_INVAL, "restart must lie in [1,64]");
  if (o.solve.precond_degree > 1) return fail(MDP_E_NOTSUP, "the server runs without a preconditioner");
  if (o.solve.gs_passes > 1) return fail(MDP_E_NOTSUP, "the server uses one Gram-Schmidt pass");
  if (o.solve.precision < MDP_FP64 || o.solve.precision > MDP_MIXED_FP16) return fail(MDP_E_INVAL, "unknown precision");
  if (!(o.solve.alpha > 0.0 && o.solve.alpha < 1.0) || !(o.solve.atol > 0.0))
    return fail(MDP_E_INVAL, "bad tolerances");
  auto* s = new mdp_server();
  s->opts = o;
  s->opts.trace_path = nullptr;  // the caller's string is copied, not kept
  if (o.trace_path) {
    s->tracing = true;
    s->trace_path = o.trace_path;
  }
  if (o.device >= 0) {
    if (hipSetDevice(o.device) != hipSuccess) {
      delete s;
      return fail(MDP_E_DEVICE, "hipSetDevice failed");
    }
  }
  if (hipGetDevice(&s->device) != hipSuccess) {
    delete s;
    return fail(MDP_E_DEVICE, "no HIP device");
  }
  // one worker per size class: requests of at most split_nnz nonzeros on the
  // first, larger ones on the second (split_nnz = 0: a single worker)
  const int nlanes = o.split_nnz > 0 ? 2 : 1;
  mdp_status st = MDP_OK;
  for (int w = 0; w < nlanes && st >= 0; ++w) {
    auto ln = std::make_unique<ServerLane>();
    ln->index = w;
    if (w == 0 && o.stream) {
      ln->stream = static_cast<hipStream_t>(o.stream);
    } else {
      hipError_t e = hipSuccess;
      {
        std::shared_lock<std::shared_mutex> g(alloc_lock());
        e = hipStreamCreateWithFlags(&ln->stream, hipStreamNonBlocking);
      }
      if (e != hipSuccess) {
        st = fail(MDP_E_DEVICE, "stream creation failed");
        break;
      }
      ln->own_stream = true;
    }
    ln->eng.stream = ln->stream;
    ln->eng.prec = prec_of(o.solve.precision);
    // a server's batches change with every arrival, so new graph keys (and
    // captures, which hold the allocation lock against admissions) keep
    // coming: it launches directly unless graphs are asked for
    ln->eng.use_graphs = o.solve.launch == MDP_LAUNCH_GRAPHS;
    st = ln->eng.reserve(o.max_batch);
    s->lanes.push_back(std::move(ln));
  }
  // the budget, and room for the staging of admissions in flight, as one
  // device allocation that admitted MDPs are placed in: admitting and
  // retiring then never call the HIP allocator.  Without the memory for it
  // the server takes its handles from the device pool instead.
  if (st >= 0) {
    size_t fr = 0, tot = 0;
    const size_t want = static_cast<size_t>(o.hbm_budget_bytes) + static_cast<size_t>(o.hbm_budget_bytes) / 4;
    if (hipMemGetInfo(&fr, &tot) == hipSuccess) {
      const size_t margin = size_t{4} << 30;
      const size_t can = fr > margin ? fr - margin : 0;
      s->arena = DeviceArena::create(s->device, std::min(want, can));
    }
    (void)hipGetLastError();
  }
  if (st < 0) {
    for (auto& ln : s->lanes) {
      ln->eng.release();
      if (ln->own_stream) {
        std::shared_lock<std::shared_mutex> g(alloc_lock());
        (void)hipStreamDestroy(ln->stream);
      }
    }
    delete s;
    return st;
  }
  s->t0 = clock_ms();
  for (int i = 0; i < o.admit_threads; ++i) s->admitters.emplace_back([s]() { s->admit_loop(); });
  s->workers_left = static_cast<int>(s->lanes.size());
  for (auto& ln : s->lanes) {
    ServerLane* l = ln.get();
    l->thread = std::thread([s, l]() { s->work_loop(l); });
  }
  s->reapers_left = o.retire_threads;
  for (int i = 0; i < o.retire_threads; ++i) s->reapers.emplace_back([s]() { s->reap_loop(); });
  *out = s;
  return MDP_OK;
}

static mdp_status submit_common(mdp_server_t s, int64_t S, int32_t A, const int64_t* row_ptr,
                                const int32_t* col, const double* val, const double* cost,
                                double gamma, int64_t* request_id, bool borrow) {
  clear_error();
  if (!s || !request_id) return fail(MDP_E_INVAL, "NULL argument");
  if (S < 1 || A < 1 || !row_ptr || !col || !val || !cost) return fail(MDP_E_INVAL, "bad MDP");
  if (!(gamma >= 0.0 && gamma < 1.0)) return fail(MDP_E_INVAL, "gamma must lie in [0,1)");
  MDP_TRY(check_size_limits(S, A, -1));
  const int64_t rows = S * A;
  const int64_t nnz = row_ptr[rows];
  if (nnz < rows) return fail(MDP_E_INVAL, "bad row_ptr");
  MDP_TRY(check_size_limits(S, A, nnz));
  auto r = std::make_unique<Request>();
  r->S = S;
  r->A = A;
  r->gamma = gamma;
  r->footprint = footprint_of(S, A, nnz, s->opts.solve);
  r->lane = (s->lanes.size() > 1 && nnz > s->opts.split_nnz) ? 1 : 0;
  if (r->footprint > s->opts.hbm_budget_bytes)
    return fail(MDP_E_NOMEM, "request footprint exceeds the server's HBM budget");
  if (borrow) {
    r->borrowed = true;
    r->b_row_ptr = row_ptr;
    r->b_col = col;
    r->b_val = val;
    r->b_cost = cost;
  } else {
    MDP_TRY(validate_host(S, A, row_ptr, col, val, cost));
    r->row_ptr.assign(row_ptr, row_ptr + rows + 1);
    r->col.assign(col, col + nnz);
    r->val.assign(val, val + nnz);
    r->cost.assign(cost, cost + rows);
  }
  Request* raw = r.get();
  std::lock_guard<std::mutex> g(s->mu);
  raw->id = s->next_id++;
  raw->st.struct_size = sizeof(mdp_request_stats);
  raw->st.submit_ms = clock_ms() - s->t0;
  s->all[raw->id] = std::move(r);
  s->queue.push_back(raw);
  *request_id = raw->id;
  s->cv_admit.notify_all();
  return MDP_OK;
}

mdp_status mdp_server_submit(mdp_server_t s, int64_t S, int32_t A, const int64_t* row_ptr,
                             const int32_t* col, const double* val, const double* cost,
                             double gamma, int64_t* request_id) {
  return submit_common(s, S, A, row_ptr, col, val, cost, gamma, request_id, false);
}

mdp_status mdp_server_submit_borrowed(mdp_server_t s, int64_t S, int32_t A,
                                      const int64_t* row_ptr, const int32_t* col,
                                      const double* val, const double* cost, double gamma,
                                      int64_t* request_id) {
  return submit_common(s, S, A, row_ptr, col, val, cost, gamma, request_id, true);
}

mdp_status mdp_server_poll(mdp_server_t s, int64_t id, int32_t* done) {
  clear_error();
  if (!s || !done) return fail(MDP_E_INVAL, "NULL argument");
  std::lock_guard<std::mutex> g(s->mu);
  auto it = s->all.find(id);
  if (it == s->all.end()) return fail(MDP_E_INVAL, "unknown request id");
  *done = it->second->done ? 1 : 0;
  return MDP_OK;
}

mdp_status mdp_server_wait(mdp_server_t s, int64_t id, double* v, int32_t* policy,
                           mdp_request_stats* stats) {
  clear_error();
  if (!s) return fail(MDP_E_INVAL, "NULL server");
  if (stats && stats->struct_size < sizeof(mdp_request_stats))
    return fail(MDP_E_INVAL, "mdp_request_stats.struct_size too small");
  std::unique_ptr<Request> r;
  {
    std::unique_lock<std::mutex> lk(s->mu);
    auto it = s->all.find(id);
    if (it == s->all.end()) return fail(MDP_E_INVAL, "unknown request id");
    Request* raw = it->second.get();
    s->cv_done.wait(lk, [&]() { return raw->done; });
    r = std::move(it->second);
    s->all.erase(it);
  }
  if (r->status < 0) return fail(r->status, "request failed: " + r->error);
  if (v) std::memcpy(v, r->v.data(), r->v.size() * sizeof(double));
  if (policy) std::memcpy(policy, r->pi.data(), r->pi.size() * sizeof(int32_t));
  if (stats) *stats = r->st;
  return r->status;
}

mdp_status mdp_server_info(mdp_server_t s, int64_t* queued, int64_t* resident,
                           int64_t* resident_bytes, int64_t* rounds) {
  clear_error();
  if (!s) return fail(MDP_E_INVAL, "NULL server");
  std::lock_guard<std::mutex> g(s->mu);
  if (queued) *queued = static_cast<int64_t>(s->queue.size());
  int64_t res = 0, rnd = 0;
  for (const auto& ln : s->lanes) {
    res += static_cast<int64_t>(ln->resident.size() + ln->ready.size());
    rnd += ln->rounds;
  }
  if (resident) *resident = res;
  if (resident_bytes) *resident_bytes = s->held_bytes;
  if (rounds) *rounds = rnd;
  return MDP_OK;
}

mdp_status mdp_server_destroy(mdp_server_t s) {
  if (!s) return MDP_OK;
  {
    std::lock_guard<std::mutex> g(s->mu);
    s->stop = true;
    // requests still queued are dropped; admitted ones finish
    for (Request* r : s->queue) {
      r->status = MDP_E_STATE;
      r->error = "server destroyed";
      r->done = true;
    }
    s->queue.clear();
    s->cv_admit.notify_all();
    s->cv_work.notify_all();
    s->cv_done.notify_all();
  }
  for (auto& t : s->admitters) t.join();
  {
    std::lock_guard<std::mutex> g(s->mu);
    s->cv_work.notify_all();
  }
  for (auto& ln : s->lanes)
    if (ln->thread.joinable()) ln->thread.join();
  for (auto& t : s->reapers) t.join();
  for (auto& kv : s->all)
    if (kv.second->h) mdp_destroy(kv.second->h);
  for (auto& ln : s->lanes) {
    ln->eng.release();
    if (ln->own_stream && ln->stream) {
      std::shared_lock<std::shared_mutex> g(alloc_lock());
      (void)hipStreamDestroy(ln->stream);
    }
  }
  delete s->arena;
  if (s->tracing) s->write_trace();
  delete s;
  return MDP_OK;
}

}  // extern "C"
