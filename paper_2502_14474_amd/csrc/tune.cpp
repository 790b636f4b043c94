// Lanes-per-row autotuner: times candidate lane widths for a handle's MDP and
// remembers the best width per (GPU architecture, class) in a small JSON file,
// so that later handles of the same class start from the tuned width.
//
// Class key: "A<a>_k<k>_n<e>": a = the action count rounded up to a power of
// two, k = the mean row length rounded up to a power of two, 2^e <= nnz
// rounded up to a power of two < 2^(e+4) with e a multiple of 4 (the best
// width of a small, launch-bound MDP says little about a large one).  The cache file is
// $MDP_TUNE_CACHE, else $HOME/.cache/mdp_mi355x_tune.json; a missing or
// unreadable file is treated as empty.  The file is read once per process
// (again whenever the path changes) and rewritten, via a temporary and a
// rename, by every store; a store that cannot write the file keeps the width
// for this process only.  The file holds one flat object:
//   {"gfx950:A8_k16_n20": 16, ...}
#include <cstdio>
#include <cstdlib>
#include <fstream>
#include <limits>
#include <map>
#include <mutex>
#include <condition_variable>
#include <sstream>
#include <string>

#include <sys/stat.h>

#include "internal.h"

namespace mdp {

namespace {
std::mutex g_tune_mu;
// File contents as read on first use, updated by every store; the device
// architecture names, filled on first use per device.
std::string g_loaded_path;
bool g_loaded = false;
std::map<std::string, int> g_cache;
std::map<int, std::string> g_arch;

int pow2_ceil(double x) {
  int p = 1;
  while (p < x && p < (1 << 20)) p <<= 1;
  return p;
}

std::string cache_path() {
  if (const char* p = std::getenv("MDP_TUNE_CACHE")) return p;
  const char* home = std::getenv("HOME");
  return std::string(home ? home : "/tmp") + "/.cache/mdp_mi355x_tune.json";
}

std::map<std::string, int> read_cache() {
  std::map<std::string, int> m;
  std::ifstream f(cache_path());
  if (!f) return m;
  std::stringstream ss;
  ss << f.rdbuf();
  const std::string s = ss.str();
  size_t i = 0;
  while (true) {
    const size_t a = s.find('"', i);
    if (a == std::string::npos) break;
    const size_t b = s.find('"', a + 1);
    if (b == std::string::npos) break;
    const size_t c = s.find(':', b);
    if (c == std::string::npos) break;
    char* end = nullptr;
    const long v = std::strtol(s.c_str() + c + 1, &end, 10);
    if (end == s.c_str() + c + 1) break;
    m[s.substr(a + 1, b - a - 1)] = static_cast<int>(v);
    i = static_cast<size_t>(end - s.c_str());
  }
  return m;
}

void write_cache(const std::map<std::string, int>& m) {
  const std::string path = cache_path();
  const size_t slash = path.find_last_of('/');
  if (slash != std::string::npos && slash > 0) ::mkdir(path.substr(0, slash).c_str(), 0755);
  const std::string tmp = path + ".tmp";
  std::FILE* f = std::fopen(tmp.c_str(), "w");
  if (!f) return;
  std::fputs("{", f);
  bool first = true;
  for (const auto& kv : m) {
    std::fprintf(f, "%s\n \"%s\": %d", first ? "" : ",", kv.first.c_str(), kv.second);
    first = false;
  }
  std::fputs("\n}\n", f);
  std::fclose(f);
  std::rename(tmp.c_str(), path.c_str());
}

std::string arch_of(int device) {
  const auto it = g_arch.find(device);
  if (it != g_arch.end()) return it->second;
  hipDeviceProp_t p;
  if (hipGetDeviceProperties(&p, device) != hipSuccess) return "unknown";
  std::string a = p.gcnArchName;
  const size_t colon = a.find(':');
  if (colon != std::string::npos) a = a.substr(0, colon);
  g_arch[device] = a;
  return a;
}

const std::map<std::string, int>& cache() {
  const std::string path = cache_path();
  if (!g_loaded || path != g_loaded_path) {
    g_cache = read_cache();
    g_loaded_path = path;
    g_loaded = true;
  }
  return g_cache;
}

}  // namespace

static std::string key_locked(const mdp_handle* h) {
  const double k = static_cast<double>(h->nnz) / static_cast<double>(h->rows);
  int e = 0;
  while (e < 62 && (int64_t{1} << e) < h->nnz) ++e;
  return arch_of(h->device) + ":A" + std::to_string(pow2_ceil(h->A)) + "_k" +
         std::to_string(pow2_ceil(k)) + "_n" + std::to_string(e / 4 * 4);
}

std::string tune_key(const mdp_handle* h) {
  std::lock_guard<std::mutex> g(g_tune_mu);
  return key_locked(h);
}

int tune_lookup(const mdp_handle* h) {
  std::lock_guard<std::mutex> g(g_tune_mu);
  const auto& m = cache();
  const auto it = m.find(key_locked(h));
  if (it == m.end()) return 0;
  const int L = it->second;
  return (L >= 2 && L <= 64 && (L & (L - 1)) == 0) ? L : 0;
}

namespace {
std::map<std::string, bool> g_claims;  // class -> tuning finished (claimed classes only)
std::condition_variable g_claim_cv;
}  // namespace

bool tune_claim(const mdp_handle* h) {
  std::lock_guard<std::mutex> g(g_tune_mu);
  return g_claims.emplace(key_locked(h), false).second;
}

void tune_release(const mdp_handle* h) {
  {
    std::lock_guard<std::mutex> g(g_tune_mu);
    g_claims[key_locked(h)] = true;
  }
  g_claim_cv.notify_all();
}

void tune_wait(const mdp_handle* h) {
  std::unique_lock<std::mutex> g(g_tune_mu);
  const std::string k = key_locked(h);
  g_claim_cv.wait(g, [&]() {
    const auto it = g_claims.find(k);
    return it == g_claims.end() || it->second;
  });
}

void tune_store(const mdp_handle* h, int lanes) {
  std::lock_guard<std::mutex> g(g_tune_mu);
  cache();
  auto m = read_cache();  // keep entries other processes stored meanwhile
  m[key_locked(h)] = lanes;
  write_cache(m);
  g_cache = m;
  g_loaded_path = cache_path();
}

}  // namespace mdp
