// Gather-rate probe: throughput of uniformly random 8-byte gathers from
// tables of several sizes (one XCD's L2, the Infinity Cache, HBM).  A sparse
// product whose columns are uniform random over a large vector is bound by
// this rate rather than by its streamed bytes; the probe gives that ceiling.
// 96 * 2^20 gathers per launch (about the size of a product with P_pi on the 4M-state,
// 24-entry workload), four independent gathers in flight per thread, indices
// from the SplitMix64 output mix of the gather number, so that they are
// uniform and reproducible.
#include <hip/hip_runtime.h>
#include <cstdio>
#include <cstdint>
#include <vector>

#define CHK(x) do { hipError_t e_ = (x); if (e_ != hipSuccess) { printf("HIP error %s at %d\n", hipGetErrorString(e_), __LINE__); return 1; } } while (0)

__global__ void fill_idx(int* idx, int64_t n, uint32_t table, uint32_t seed) {
  for (int64_t i = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; i < n; i += (int64_t)gridDim.x * blockDim.x) {
    uint64_t z = (uint64_t)i * 0x9E3779B97F4A7C15ull + seed;
    z = (z ^ (z >> 30)) * 0xBF58476D1CE4E5B9ull;
    z = (z ^ (z >> 27)) * 0x94D049BB133111EBull;
    z ^= z >> 31;
    idx[i] = (int)(z % table);
  }
}

__global__ void fill_x(double* x, int64_t n) {
  for (int64_t i = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; i < n; i += (int64_t)gridDim.x * blockDim.x) x[i] = 1.0 + (double)(i & 7);
}

// every thread: U independent gathers in flight per iteration
template <int U>
__global__ __launch_bounds__(256) void gather(const int* __restrict__ idx, const double* __restrict__ x, int64_t n, double* out) {
  double s = 0.0;
  const int64_t stride = (int64_t)gridDim.x * blockDim.x;
  int64_t i = blockIdx.x * (int64_t)blockDim.x + threadIdx.x;
  for (; i + (U - 1) * stride < n; i += U * stride) {
    int c[U];
#pragma unroll
    for (int u = 0; u < U; ++u) c[u] = __builtin_nontemporal_load(idx + i + u * stride);
    double v[U];
#pragma unroll
    for (int u = 0; u < U; ++u) v[u] = x[c[u]];
#pragma unroll
    for (int u = 0; u < U; ++u) s += v[u];
  }
  for (; i < n; i += stride) s += x[idx[i]];
  out[blockIdx.x * (int64_t)blockDim.x + threadIdx.x] = s;
}

// The same gathers through a raw buffer resource with the cache-policy bits
// AUX of the load instruction (gfx950: bit 0 sc0, bit 1 nt, bit 4 sc1): how
// the line granularity of the path a gather takes changes the rate.
template <int AUX>
__global__ __launch_bounds__(256) void gather_policy(const int* __restrict__ idx, const double* __restrict__ x,
                                                     int64_t nx, int64_t n, double* out) {
  const __amdgpu_buffer_rsrc_t r = __builtin_amdgcn_make_buffer_rsrc(
      const_cast<double*>(x), static_cast<short>(0), static_cast<int>(static_cast<uint32_t>(nx * 8)), 0x00020000);
  constexpr int U = 4;
  double s = 0.0;
  const int64_t stride = (int64_t)gridDim.x * blockDim.x;
  int64_t i = blockIdx.x * (int64_t)blockDim.x + threadIdx.x;
  for (; i + (U - 1) * stride < n; i += U * stride) {
    int c[U];
#pragma unroll
    for (int u = 0; u < U; ++u) c[u] = __builtin_nontemporal_load(idx + i + u * stride);
    double v[U];
#pragma unroll
    for (int u = 0; u < U; ++u)
      v[u] = __builtin_bit_cast(double, __builtin_amdgcn_raw_buffer_load_b64(
                                            r, static_cast<int>(static_cast<uint32_t>(c[u]) * 8u), 0, AUX));
#pragma unroll
    for (int u = 0; u < U; ++u) s += v[u];
  }
  for (; i < n; i += stride) s += x[idx[i]];
  out[blockIdx.x * (int64_t)blockDim.x + threadIdx.x] = s;
}

// Slice-aligned indices: element i is read by thread i % T of the grid-stride
// loop (T = grid * 256), i.e. by workgroup w = (i % T) / 256, and falls in
// slice f(w) of a table cut into nslices equal slices.  mode 0: f(w) = w % 8 +
// 8 * ((w / 8) % (nslices / 8)), so the workgroups dispatched to one XCD
// (w % 8) share that XCD's slices; mode 1: f(w) = (w / 8) % nslices, every
// XCD sees every slice.
__global__ void fill_idx_sliced(int* idx, int64_t n, int64_t T, int mode, uint32_t slice_len, int nslices,
                                uint32_t seed) {
  for (int64_t i = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; i < n; i += (int64_t)gridDim.x * blockDim.x) {
    const int64_t w = (i % T) / 256;
    uint64_t z = (uint64_t)i * 0x9E3779B97F4A7C15ull + seed;
    z = (z ^ (z >> 30)) * 0xBF58476D1CE4E5B9ull;
    z = (z ^ (z >> 27)) * 0x94D049BB133111EBull;
    z ^= z >> 31;
    const int sl = mode == 0 ? (int)(w % 8) + 8 * (int)((w / 8) % (nslices / 8)) : (int)((w / 8) % nslices);
    idx[i] = sl * (int)slice_len + (int)(z % slice_len);
  }
}

// The traffic of the blocked sweep and of the sliced policy product around
// each gather: a streamed 4-byte column and 8-byte value per entry, the
// product accumulated, and one 8-byte partial written per three entries.
__global__ __launch_bounds__(256) void gather_stream(const int* __restrict__ idx, const double* __restrict__ val,
                                                     const double* __restrict__ x, int64_t n,
                                                     double* __restrict__ part) {
  constexpr int U = 4;
  double s = 0.0;
  const int64_t stride = (int64_t)gridDim.x * blockDim.x;
  int64_t i = blockIdx.x * (int64_t)blockDim.x + threadIdx.x;
  for (; i + (U - 1) * stride < n; i += U * stride) {
    int c[U];
    double p[U];
#pragma unroll
    for (int u = 0; u < U; ++u) {
      c[u] = __builtin_nontemporal_load(idx + i + u * stride);
      p[u] = __builtin_nontemporal_load(val + i + u * stride);
    }
    double v[U];
#pragma unroll
    for (int u = 0; u < U; ++u) v[u] = x[c[u]];
#pragma unroll
    for (int u = 0; u < U; ++u) s = fma(p[u], v[u], s);
    if ((i / stride) % 3 == 0) part[i / 3] = s;
  }
  for (; i < n; i += stride) s = fma(val[i], x[idx[i]], s);
  part[(blockIdx.x * (int64_t)blockDim.x + threadIdx.x) / 3] = s;
}

// streaming read of the index array alone (the gather-free floor)
__global__ __launch_bounds__(256) void stream_idx(const int* __restrict__ idx, int64_t n, double* out) {
  double s = 0.0;
  for (int64_t i = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; i < n; i += (int64_t)gridDim.x * blockDim.x)
    s += (double)__builtin_nontemporal_load(idx + i);
  out[blockIdx.x * (int64_t)blockDim.x + threadIdx.x] = s;
}

int main() {
  const int64_t n = 96ll << 20;  // 96M gathers (the config-4 policy product)
  const int grid = 256 * 16;
  int* idx;
  double *x, *out;
  const int64_t max_table = 1ll << 27;  // 1 GiB of doubles
  CHK(hipMalloc(&idx, n * sizeof(int)));
  CHK(hipMalloc(&x, max_table * sizeof(double)));
  CHK(hipMalloc(&out, (int64_t)grid * 256 * sizeof(double)));
  fill_x<<<4096, 256>>>(x, max_table);
  CHK(hipGetLastError());
  hipEvent_t a, b;
  CHK(hipEventCreate(&a));
  CHK(hipEventCreate(&b));
  const int64_t tables[] = {1ll << 19, 1ll << 22, 1ll << 24, 1ll << 25, 1ll << 27};
  for (int64_t t : tables) {
    fill_idx<<<4096, 256>>>(idx, n, (uint32_t)t, 12345u);
    CHK(hipGetLastError());
    CHK(hipDeviceSynchronize());
    for (int rep = 0; rep < 2; ++rep) gather<4><<<grid, 256>>>(idx, x, n, out);
    CHK(hipEventRecord(a));
    const int reps = 10;
    for (int rep = 0; rep < reps; ++rep) gather<4><<<grid, 256>>>(idx, x, n, out);
    CHK(hipEventRecord(b));
    CHK(hipEventSynchronize(b));
    float ms;
    CHK(hipEventElapsedTime(&ms, a, b));
    ms /= reps;
    printf("table %8.1f MB: %.3f ms per %lld gathers -> %.1f G gathers/s (index stream %.2f TB/s)\n",
           t * 8.0 / 1e6, ms, (long long)n, n / (ms * 1e-3) / 1e9, n * 4.0 / (ms * 1e-3) / 1e12);
    fflush(stdout);
  }
  // cache-policy variants of the gathers on a 33.6 MB and a 1 GiB table
  const int64_t ptables[] = {1ll << 22, 1ll << 27};
  for (int64_t t : ptables) {
    fill_idx<<<4096, 256>>>(idx, n, (uint32_t)t, 12345u);
    CHK(hipGetLastError());
    CHK(hipDeviceSynchronize());
    auto run = [&](auto kern, const char* name) -> int {
      for (int rep = 0; rep < 2; ++rep) kern<<<grid, 256>>>(idx, x, t, n, out);
      CHK(hipEventRecord(a));
      for (int rep = 0; rep < 10; ++rep) kern<<<grid, 256>>>(idx, x, t, n, out);
      CHK(hipEventRecord(b));
      CHK(hipEventSynchronize(b));
      float ms;
      CHK(hipEventElapsedTime(&ms, a, b));
      ms /= 10;
      printf("table %8.1f MB, buffer load %-8s: %.3f ms -> %.1f G gathers/s\n", t * 8.0 / 1e6, name, ms,
             n / (ms * 1e-3) / 1e9);
      fflush(stdout);
      return 0;
    };
    if (run(gather_policy<0>, "default")) return 1;
    if (run(gather_policy<1>, "sc0")) return 1;
    if (run(gather_policy<2>, "nt")) return 1;
    if (run(gather_policy<3>, "sc0 nt")) return 1;
    if (run(gather_policy<16>, "sc1")) return 1;
    if (run(gather_policy<17>, "sc0 sc1")) return 1;
    if (run(gather_policy<18>, "sc1 nt")) return 1;
    if (run(gather_policy<19>, "all")) return 1;
  }
  // slices aligned with the XCDs, on a 33.6 MB table (a 4M-state float64
  // vector): plain gathers, then with the streamed entries and partials
  {
    const int64_t t = 1ll << 22;
    const int64_t T = (int64_t)grid * 256;
    double *val, *part;
    CHK(hipMalloc(&val, n * sizeof(double)));
    CHK(hipMalloc(&part, (n / 3 + 1) * sizeof(double)));
    fill_x<<<4096, 256>>>(val, n);
    CHK(hipGetLastError());
    struct Case { int mode, nslices; const char* name; };
    const Case cases[] = {{0, 8, "w%8 -> slice (8 x 4.2 MB)"},
                          {1, 8, "(w/8)%8 -> slice (8 x 4.2 MB)"},
                          {0, 16, "w%8 + 8*((w/8)%2) (16 x 2.1 MB)"},
                          {1, 16, "(w/8)%16 (16 x 2.1 MB)"}};
    for (const Case& c : cases) {
      fill_idx_sliced<<<4096, 256>>>(idx, n, T, c.mode, (uint32_t)(t / c.nslices), c.nslices, 12345u);
      CHK(hipGetLastError());
      CHK(hipDeviceSynchronize());
      float ms[2];
      for (int k = 0; k < 2; ++k) {
        for (int rep = 0; rep < 2; ++rep) {
          if (k == 0) gather<4><<<grid, 256>>>(idx, x, n, out);
          else gather_stream<<<grid, 256>>>(idx, val, x, n, part);
        }
        CHK(hipEventRecord(a));
        for (int rep = 0; rep < 10; ++rep) {
          if (k == 0) gather<4><<<grid, 256>>>(idx, x, n, out);
          else gather_stream<<<grid, 256>>>(idx, val, x, n, part);
        }
        CHK(hipEventRecord(b));
        CHK(hipEventSynchronize(b));
        CHK(hipEventElapsedTime(&ms[k], a, b));
        ms[k] /= 10;
      }
      printf("sliced table 33.6 MB, %-34s gathers %.1f G/s; with streamed entries and partials %.1f G/s\n",
             c.name, n / (ms[0] * 1e-3) / 1e9, n / (ms[1] * 1e-3) / 1e9);
      fflush(stdout);
    }
    // one slice for all workgroups (a pass of the blocked sweep): 2.75 MB and 3.25 MB of v
    for (const int64_t bytes : {11ll << 18, 13ll << 18}) {
      fill_idx<<<4096, 256>>>(idx, n, (uint32_t)(bytes / 8), 12345u);
      CHK(hipGetLastError());
      CHK(hipDeviceSynchronize());
      for (int rep = 0; rep < 2; ++rep) gather_stream<<<grid, 256>>>(idx, val, x, n, part);
      CHK(hipEventRecord(a));
      for (int rep = 0; rep < 10; ++rep) gather_stream<<<grid, 256>>>(idx, val, x, n, part);
      CHK(hipEventRecord(b));
      CHK(hipEventSynchronize(b));
      float ms1;
      CHK(hipEventElapsedTime(&ms1, a, b));
      ms1 /= 10;
      printf("one %.2f MB table for all workgroups, with streamed entries and partials: %.1f G/s\n",
             bytes / 1048576.0, n / (ms1 * 1e-3) / 1e9);
      fflush(stdout);
    }
    CHK(hipFree(val));
    CHK(hipFree(part));
  }
  CHK(hipEventRecord(a));
  for (int rep = 0; rep < 10; ++rep) stream_idx<<<grid, 256>>>(idx, n, out);
  CHK(hipEventRecord(b));
  CHK(hipEventSynchronize(b));
  float ms;
  CHK(hipEventElapsedTime(&ms, a, b));
  printf("index stream alone: %.3f ms -> %.2f TB/s\n", ms / 10, n * 4.0 / (ms / 10 * 1e-3) / 1e12);
  return 0;
}
