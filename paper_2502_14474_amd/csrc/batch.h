// Batched inexact policy iteration: device descriptors, work lists and the
// host engine that advances many resident MDPs round by round.
#pragma once

#include <map>
#include <shared_mutex>
#include <tuple>
#include <vector>

#include "internal.h"

namespace mdp {

// One MDP of a batch as the batched kernels see it (device copy).
struct BDesc {
  int64_t S;
  int A;
  int basis_f32;  // basis and r0 stored in float32 (mixed precision)
  int kfix;       // common row length, or 0
  double gamma;
  const int* row_ptr;
  const int* col;
  const double* val;
  const float* cv32;  // packed float32 copy (see mdp_handle::cv32)
  const __half* val16;
  const double* corr16;
  const double* cost;
  double* v;  // outer iterate and inner GMRES iterate
  float* v32;
  int* pi;
  double* U64;
  float* U32;
  int64_t ldu;
  double* part;
  Ctl* ctl;
  double alpha;
  double floor_rel;
  int nb_sweep, nb_apply, nb_upd;  // tiles of this MDP per kernel kind
};

// Work list: listed descriptor indices and the prefix sums of their tiles,
// laid out as [n, cap, item[cap], tstart[cap + 1]].
struct WorkList {
  int n;
  int cap;
  int data[1];
  __host__ __device__ int it(int k) const { return data[k]; }
  __host__ __device__ const int* ts() const { return data + cap; }
  __host__ __device__ int* items() { return data; }
  __host__ __device__ int* tss() { return data + cap; }
  static size_t bytes(int cap) { return sizeof(int) * ((2 + 2 * cap + 1 + 63) / 64 * 64); }
};

// Per-MDP host state of the batched solve.
struct BatchItem {
  enum State { kSweep = 0, kGmres = 1, kDone = 2 };
  mdp_handle* h = nullptr;
  int state = kSweep;
  mdp_status status = MDP_OK;
  double alpha = 1e-4;
  double prev_res = 0.0, res = 0.0;
  bool lowp_sweep = false;
  double prev_lowp_res = 0.0;
  int64_t k = 0, sweeps = 0, inner = 0, applies = 0, refinements = 0, eval_steps = 0;
  double bytes = 0.0;
  std::vector<double> history;
  void finish_eval();
};

struct GraphKey {
  int prec;
  std::vector<int> lanes;
  int m, se;
  int g_apply, g_upd, g_small;  // the captured grids (powers of two, capped)
  bool operator<(const GraphKey& o) const {
    return std::tie(prec, lanes, m, se, g_apply, g_upd, g_small) <
           std::tie(o.prec, o.lanes, o.m, o.se, o.g_apply, o.g_upd, o.g_small);
  }
};
struct ChunkGraphs {
  std::vector<hipGraphExec_t> exec;
};

class BatchEngine {
 public:
  static constexpr int kMaxClasses = 6;  // lane widths 2..64
  // sweep groups are (lane width, sweep precision): up to 3 * kMaxClasses
  enum {
    kListSweep0 = 0,
    kListApply0 = 3 * kMaxClasses,
    kListAll = 4 * kMaxClasses,
    kListGm,
    kListGmUpd,
    kListCast,
    kNumLists
  };
  hipStream_t stream = nullptr;
  Prec prec = kF64;
  bool use_graphs = true;
  std::vector<BatchItem*> items;
  // the last round: how many items it swept, and when (steady-clock ms) its
  // sweep phase ended
  int last_swept = 0;
  double last_sweep_end_ms = 0;

  ~BatchEngine();
  mdp_status reserve(int n);
  mdp_status round(const mdp_solve_opts& o);
  void release();

 private:
  int cap = 0;
  BDesc* descs_d = nullptr;
  BDesc* descs_h = nullptr;  // pinned, so uploads never queue behind pageable copies
  void* lists_d = nullptr;
  void* lists_h = nullptr;
  Ctl* hdr_d = nullptr;
  Ctl* hdr_h = nullptr;
  std::map<GraphKey, ChunkGraphs> graphs;

  WorkList* list_d(int slot) const;
  WorkList* list_h(int slot) const;
  void fill_desc(int i);
  int build_list(int slot, const std::vector<int>& idx, int kind);
  mdp_status upload(int nitems, int nlists);
  mdp_status headers(int slot, int n);
  hipError_t enqueue_steps(const std::vector<int>& lanes, int j0, int j1, int m, const GraphKey* fixed,
                           int tiles_apply_max, int tiles_upd, int n_items);
  mdp_status sweep_phase(const mdp_solve_opts& o, std::vector<int>& need);
  mdp_status cycle_phase(const mdp_solve_opts& o, std::vector<int>& gm);
};

// A batched engine leased from the library's per-device cache (api.cpp).
struct EngineLease {
  explicit EngineLease(int dev);
  ~EngineLease();
  EngineLease(const EngineLease&) = delete;
  EngineLease& operator=(const EngineLease&) = delete;
  int dev;
  BatchEngine* eng = nullptr;
};

}  // namespace mdp
