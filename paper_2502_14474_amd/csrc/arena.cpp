// Device arenas: one device allocation made up front and carved into the
// arrays of many handles by the library itself.  A server makes one when it
// starts and admits its requests into it, so the serving loop never calls the
// HIP allocator.  (With the runtime's stream-ordered pool, which hands freed
// memory back after a synchronisation whatever its release threshold, the
// allocations and releases of admissions and retirements stalled every stream
// of the process for up to two seconds at a time, with the GPU idle.)
//
// Ranges are handed out best fit, 256-byte aligned, and coalesced when they
// come back.  A range freed against a stream returns once the work queued on
// that stream so far has finished (an event marks the point); one freed with
// no stream returns at once.
#include <algorithm>
#include <map>
#include <mutex>
#include <shared_mutex>
#include <unordered_map>
#include <vector>

#include "internal.h"

namespace mdp {

namespace {
constexpr size_t kArenaAlign = 256;

std::shared_mutex g_arenas_mu;
std::vector<DeviceArena*> g_arenas;  // live arenas, for arena_of
thread_local DeviceArena* t_current = nullptr;
}  // namespace

DeviceArena* DeviceArena::create(int dev, size_t bytes) {
  bytes = (bytes + kArenaAlign - 1) / kArenaAlign * kArenaAlign;
  if (bytes == 0) return nullptr;
  void* p = nullptr;
  if (lib_malloc(&p, bytes) != hipSuccess) {
    (void)hipGetLastError();
    return nullptr;
  }
  auto* a = new DeviceArena();
  a->dev_ = dev;
  a->base_ = static_cast<char*>(p);
  a->size_ = bytes;
  a->free_[0] = bytes;
  std::unique_lock<std::shared_mutex> g(g_arenas_mu);
  g_arenas.push_back(a);
  return a;
}

DeviceArena::~DeviceArena() {
  {
    std::unique_lock<std::shared_mutex> g(g_arenas_mu);
    g_arenas.erase(std::remove(g_arenas.begin(), g_arenas.end(), this), g_arenas.end());
  }
  {
    std::lock_guard<std::mutex> lk(mu_);
    for (Pending& q : pending_) {
      (void)hipEventSynchronize(q.ev);
      spare_.push_back(q.ev);
    }
    pending_.clear();
  }
  {
    std::shared_lock<std::shared_mutex> g(alloc_lock());
    for (hipEvent_t e : spare_) (void)hipEventDestroy(e);
  }
  lib_free(base_);
}

bool DeviceArena::owns(const void* p) const {
  const char* c = static_cast<const char*>(p);
  return c >= base_ && c < base_ + size_;
}

void DeviceArena::release_locked(size_t off) {
  auto u = used_.find(off);
  if (u == used_.end()) return;
  size_t len = u->second;
  used_.erase(u);
  in_use_ -= len;
  // coalesce with the free neighbours on both sides
  auto next = free_.lower_bound(off);
  if (next != free_.end() && off + len == next->first) {
    len += next->second;
    next = free_.erase(next);
  }
  if (next != free_.begin()) {
    auto prev = std::prev(next);
    if (prev->first + prev->second == off) {
      prev->second += len;
      return;
    }
  }
  free_[off] = len;
}

void DeviceArena::reap_locked() {
  size_t k = 0;
  for (Pending& q : pending_) {
    if (hipEventQuery(q.ev) == hipSuccess) {
      release_locked(q.off);
      spare_.push_back(q.ev);
    } else {
      pending_[k++] = q;
    }
  }
  pending_.resize(k);
  (void)hipGetLastError();  // hipErrorNotReady of the queries
}

void* DeviceArena::alloc(size_t bytes) {
  bytes = std::max<size_t>(kArenaAlign, (bytes + kArenaAlign - 1) / kArenaAlign * kArenaAlign);
  std::lock_guard<std::mutex> lk(mu_);
  reap_locked();
  auto best = free_.end();
  for (auto it = free_.begin(); it != free_.end(); ++it)
    if (it->second >= bytes && (best == free_.end() || it->second < best->second)) best = it;
  if (best == free_.end()) return nullptr;
  const size_t off = best->first, len = best->second;
  free_.erase(best);
  if (len > bytes) free_[off + bytes] = len - bytes;
  used_[off] = bytes;
  in_use_ += bytes;
  return base_ + off;
}

void DeviceArena::free(void* p, hipStream_t st) {
  const size_t off = static_cast<size_t>(static_cast<char*>(p) - base_);
  std::lock_guard<std::mutex> lk(mu_);
  if (!st) {
    release_locked(off);
    return;
  }
  hipEvent_t ev = nullptr;
  if (!spare_.empty()) {
    ev = spare_.back();
    spare_.pop_back();
  } else {
    std::shared_lock<std::shared_mutex> g(alloc_lock());
    if (hipEventCreateWithFlags(&ev, hipEventDisableTiming) != hipSuccess) ev = nullptr;
  }
  if (!ev || hipEventRecord(ev, st) != hipSuccess) {
    // no event to mark the point: wait for the stream instead
    (void)hipGetLastError();
    if (ev) spare_.push_back(ev);
    (void)hipStreamSynchronize(st);
    release_locked(off);
    return;
  }
  pending_.push_back({off, ev});
}

size_t DeviceArena::in_use() {
  std::lock_guard<std::mutex> lk(mu_);
  return in_use_;
}

DeviceArena* arena_of(const void* p) {
  if (!p) return nullptr;
  std::shared_lock<std::shared_mutex> g(g_arenas_mu);
  for (DeviceArena* a : g_arenas)
    if (a->owns(p)) return a;
  return nullptr;
}

ArenaScope::ArenaScope(DeviceArena* a) : prev_(t_current) { t_current = a; }
ArenaScope::~ArenaScope() { t_current = prev_; }
DeviceArena* current_arena() { return t_current; }

}  // namespace mdp
