// MDP construction on the device from the caller's own row kernel (the
// paper's construction from online simulation, run in parallel): the caller's
// kernel fills padded rows straight into device staging, the library turns
// them into CSR on the device and builds the handle from the device arrays,
// so no row is generated on the host or copied over PCIe.
#include <hipcub/hipcub.hpp>

#include <algorithm>
#include <cstring>
#include <mutex>
#include <string>
#include <vector>

#include "device.h"

namespace mdp {

namespace {

// len[r] must lie in [1, k_max]: *bad (all ones before) receives the lowest
// offending row, and the lengths widen to int64 for the scan.
__global__ __launch_bounds__(kBlock) void k_rows_lengths(const int32_t* __restrict__ len, int64_t rows, int k_max,
                                                         int64_t* __restrict__ len64,
                                                         unsigned long long* __restrict__ bad) {
  for (int64_t r = static_cast<int64_t>(blockIdx.x) * kBlock + threadIdx.x; r < rows;
       r += static_cast<int64_t>(gridDim.x) * kBlock) {
    const int n = len[r];
    const bool ok = n >= 1 && n <= k_max;
    len64[r] = ok ? n : 0;
    if (!ok) atomicMin(bad, static_cast<unsigned long long>(r));
  }
}

// Row r's first len[r] slots move to [row_ptr[r], row_ptr[r+1]) of the CSR
// arrays; groups of 8 lanes per row.
__global__ __launch_bounds__(kBlock) void k_rows_compact(int64_t rows, int k_max, const int64_t* __restrict__ rp,
                                                         const int32_t* __restrict__ pcol,
                                                         const double* __restrict__ pval,
                                                         int32_t* __restrict__ col, double* __restrict__ val) {
  constexpr int G = 8;
  const int l = threadIdx.x % G;
  for (int64_t r = (static_cast<int64_t>(blockIdx.x) * kBlock + threadIdx.x) / G; r < rows;
       r += static_cast<int64_t>(gridDim.x) * (kBlock / G)) {
    const int64_t st = rp[r], n = rp[r + 1] - st;
    const int64_t src = r * k_max;
    for (int64_t e = l; e < n; e += G) {
      col[st + e] = pcol[src + e];
      val[st + e] = pval[src + e];
    }
  }
}

std::mutex g_mod_mu;
std::vector<hipModule_t> g_modules;  // loaded code objects, kept until the process ends

struct DevBuf {
  void* p = nullptr;
  ~DevBuf() { lib_free(p); }
  hipError_t alloc(size_t b) { return lib_malloc(&p, b > 0 ? b : 1); }
};

}  // namespace

}  // namespace mdp

extern "C" mdp_status mdp_load_kernel(const char* code_object_path, const char* name, void** kernel) {
  using namespace mdp;
  clear_error();
  if (!code_object_path || !name || !kernel) return fail(MDP_E_INVAL, "NULL argument");
  *kernel = nullptr;
  hipModule_t mod = nullptr;
  hipError_t e = hipModuleLoad(&mod, code_object_path);
  if (e != hipSuccess) {
    (void)hipGetLastError();
    return fail(MDP_E_INVAL, std::string("cannot load code object ") + code_object_path + ": " + hipGetErrorString(e));
  }
  hipFunction_t f = nullptr;
  e = hipModuleGetFunction(&f, mod, name);
  if (e != hipSuccess) {
    (void)hipGetLastError();
    (void)hipModuleUnload(mod);
    return fail(MDP_E_INVAL, std::string("no kernel ") + name + " in " + code_object_path);
  }
  {
    std::lock_guard<std::mutex> lk(g_mod_mu);
    g_modules.push_back(mod);
  }
  *kernel = reinterpret_cast<void*>(f);
  return MDP_OK;
}

extern "C" mdp_status mdp_create_from_device_rows(int64_t S, int32_t A, int32_t k_max, void* kernel,
                                                  const void* user, double gamma, const mdp_create_opts* opt,
                                                  mdp_t* out) {
  using namespace mdp;
  clear_error();
  if (!out) return fail(MDP_E_INVAL, "out is NULL");
  *out = nullptr;
  if (!kernel) return fail(MDP_E_INVAL, "kernel is NULL");
  if (S < 1 || A < 1) return fail(MDP_E_INVAL, "S and A must be at least 1");
  if (k_max < 1 || k_max > 4096) return fail(MDP_E_INVAL, "k_max must lie in [1,4096]");
  MDP_TRY(check_size_limits(S, A, -1));
  const int64_t rows = S * A;
  const int64_t slots = rows * static_cast<int64_t>(k_max);
  if (slots > (int64_t{1} << 34)) return fail(MDP_E_NOTSUP, "S*A*k_max above 2^34 slots of staging");
  if (opt && opt->struct_size < sizeof(mdp_create_opts))
    return fail(MDP_E_INVAL, "mdp_create_opts.struct_size too small");
  if (opt && opt->device >= 0) MDP_HIP(hipSetDevice(opt->device));
  hipStream_t st = opt && opt->stream ? static_cast<hipStream_t>(opt->stream) : nullptr;
  DevBuf pcol, pval, len, cost, len64, rp, col, val, bad, tmp;
  MDP_HIP(pcol.alloc(slots * sizeof(int32_t)));
  MDP_HIP(pval.alloc(slots * sizeof(double)));
  MDP_HIP(len.alloc(rows * sizeof(int32_t)));
  MDP_HIP(cost.alloc(rows * sizeof(double)));
  // the caller's kernel: one thread per state, 256 threads per workgroup
  mdp_device_rows_args a;
  std::memset(&a, 0, sizeof(a));
  a.S = S;
  a.A = A;
  a.k_max = k_max;
  a.s_begin = 0;
  a.s_end = S;
  a.col = static_cast<int32_t*>(pcol.p);
  a.val = static_cast<double*>(pval.p);
  a.len = static_cast<int32_t*>(len.p);
  a.cost = static_cast<double*>(cost.p);
  a.user = user;
  void* params[] = {&a};
  const int64_t grid = (S + kBlock - 1) / kBlock;
  if (grid > 0x7FFFFFFF) return fail(MDP_E_NOTSUP, "too many states for one launch");
  hipError_t e = hipModuleLaunchKernel(reinterpret_cast<hipFunction_t>(kernel), static_cast<unsigned>(grid), 1, 1,
                                       kBlock, 1, 1, 0, st, params, nullptr);
  if (e != hipSuccess) {
    (void)hipGetLastError();
    return fail(MDP_E_INVAL, std::string("row kernel launch failed: ") + hipGetErrorString(e));
  }
  // lengths: checked, widened, scanned into int64 row offsets
  MDP_HIP(len64.alloc(rows * sizeof(int64_t)));
  MDP_HIP(bad.alloc(sizeof(unsigned long long)));
  MDP_HIP(rp.alloc((rows + 1) * sizeof(int64_t)));
  const unsigned long long none = ~0ull;
  MDP_HIP(hipMemsetAsync(bad.p, 0xFF, sizeof(unsigned long long), st));
  const int g = static_cast<int>(std::min<int64_t>((rows + kBlock - 1) / kBlock, 8192));
  k_rows_lengths<<<g, kBlock, 0, st>>>(static_cast<const int32_t*>(len.p), rows, k_max,
                                       static_cast<int64_t*>(len64.p), static_cast<unsigned long long*>(bad.p));
  MDP_HIP(hipGetLastError());
  unsigned long long bad_h = 0;
  MDP_HIP(copy_out(&bad_h, bad.p, sizeof(bad_h), st));
  MDP_HIP(hipStreamSynchronize(st));
  if (bad_h != none)
    return fail(MDP_E_INVAL, "row kernel gave row " + std::to_string(bad_h) + " a length outside [1, k_max]");
  MDP_HIP(hipMemsetAsync(rp.p, 0, sizeof(int64_t), st));
  size_t tbytes = 0;
  auto* rp1 = static_cast<int64_t*>(rp.p) + 1;
  MDP_HIP(hipcub::DeviceScan::InclusiveSum(nullptr, tbytes, static_cast<const int64_t*>(len64.p), rp1,
                                           static_cast<int>(rows), st));
  MDP_HIP(tmp.alloc(tbytes));
  MDP_HIP(hipcub::DeviceScan::InclusiveSum(tmp.p, tbytes, static_cast<const int64_t*>(len64.p), rp1,
                                           static_cast<int>(rows), st));
  int64_t nnz = 0;
  MDP_HIP(copy_out(&nnz, rp1 + rows - 1, sizeof(nnz), st));
  MDP_HIP(hipStreamSynchronize(st));
  MDP_TRY(check_size_limits(S, A, nnz));
  MDP_HIP(col.alloc(nnz * sizeof(int32_t)));
  MDP_HIP(val.alloc(nnz * sizeof(double)));
  k_rows_compact<<<g, kBlock, 0, st>>>(rows, k_max, static_cast<const int64_t*>(rp.p),
                                       static_cast<const int32_t*>(pcol.p), static_cast<const double*>(pval.p),
                                       static_cast<int32_t*>(col.p), static_cast<double*>(val.p));
  MDP_HIP(hipGetLastError());
  MDP_HIP(hipStreamSynchronize(st));
  // the CSR is on the device: the handle is built from it as from any caller
  // device arrays, validated as opt->validate asks (without opt: on the
  // device, so that no entry crosses to the host)
  mdp_create_opts o;
  mdp_default_create_opts(&o);
  if (opt) o = *opt;
  else o.validate = MDP_VALIDATE_DEVICE;
  return mdp_create(S, A, static_cast<const int64_t*>(rp.p), static_cast<const int32_t*>(col.p),
                    static_cast<const double*>(val.p), static_cast<const double*>(cost.p), gamma, &o, out);
}
