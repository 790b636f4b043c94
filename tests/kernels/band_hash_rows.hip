// Row kernel for the device-construction tests: a seeded MDP whose every
// number comes from SplitMix64 (Steele, Lea and Flood 2014, in the form Vigna
// publishes it), so that tests/kernels/band_hash_rows.py can rebuild the same
// arrays on the host with numpy.  Row r = s*A + a holds len = 1 + h(r,0) mod
// k_max entries: columns (s + 3j + h(r,1) mod 5) mod S for j < len, sorted
// increasing with their weights; weights ((h(r, 100+j) >> 11) * 2^-53) +
// 1/1024, divided by their sum taken in sorted order; cost (h(r, 999) >> 11) *
// 2^-53.  Here h(r, t) = splitmix64(seed ^ (r * 1000003 + t)) and the user
// pointer is the address of the 64-bit seed on the device.
#include <hip/hip_runtime.h>
#include <stdint.h>

#include "mdp.h"

__device__ __forceinline__ uint64_t splitmix64(uint64_t x) {
  uint64_t z = x + 0x9E3779B97F4A7C15ull;
  z = (z ^ (z >> 30)) * 0xBF58476D1CE4E5B9ull;
  z = (z ^ (z >> 27)) * 0x94D049BB133111EBull;
  return z ^ (z >> 31);
}

__device__ __forceinline__ uint64_t h(uint64_t seed, int64_t r, int t) {
  return splitmix64(seed ^ (static_cast<uint64_t>(r) * 1000003ull + static_cast<uint64_t>(t)));
}

extern "C" __global__ void band_hash_rows(mdp_device_rows_args a) {
  const int64_t s = a.s_begin + static_cast<int64_t>(blockIdx.x) * blockDim.x + threadIdx.x;
  if (s >= a.s_end) return;
  const uint64_t seed = *static_cast<const uint64_t*>(a.user);
  for (int act = 0; act < a.A; ++act) {
    const int64_t r = s * a.A + act;
    const int64_t i = (s - a.s_begin) * a.A + act;
    const int len = 1 + static_cast<int>(h(seed, r, 0) % static_cast<uint64_t>(a.k_max));
    const int shift = static_cast<int>(h(seed, r, 1) % 5ull);
    int c[64];
    double w[64];
    for (int j = 0; j < len; ++j) {
      c[j] = static_cast<int>((s + 3 * j + shift) % a.S);
      w[j] = static_cast<double>(h(seed, r, 100 + j) >> 11) * 0x1.0p-53 + 0x1.0p-10;
    }
    // insertion sort by column (columns are distinct while 3 * k_max + 5 <= S)
    for (int j = 1; j < len; ++j) {
      const int cj = c[j];
      const double wj = w[j];
      int k = j - 1;
      while (k >= 0 && c[k] > cj) {
        c[k + 1] = c[k];
        w[k + 1] = w[k];
        --k;
      }
      c[k + 1] = cj;
      w[k + 1] = wj;
    }
    double sum = 0.0;
    for (int j = 0; j < len; ++j) sum += w[j];
    for (int j = 0; j < len; ++j) {
      a.col[i * a.k_max + j] = c[j];
      a.val[i * a.k_max + j] = w[j] / sum;
    }
    a.len[i] = len;
    a.cost[i] = static_cast<double>(h(seed, r, 999) >> 11) * 0x1.0p-53;
  }
}
