// Caching device allocator of the library (see pool_alloc in the internal
// header).  Sizes are rounded to 256 bytes below 1 MiB and to eighths of a
// power of two above, and blocks are reused only at exactly their rounded
// size, so repeated plans of one shape hit the cache every time.
#include <mutex>
#include <unordered_map>

#include "phs_internal.h"

namespace phs {

namespace {

std::mutex g_mu;
std::unordered_map<size_t, std::vector<void *>> g_free;  // rounded size -> idle blocks
std::unordered_map<void *, size_t> g_size;               // every block the pool owns
std::unordered_map<void *, bool> g_idle;                 // blocks on a free list
thread_local std::vector<void *> t_pending;
thread_local int64_t t_net = 0;  // bytes this thread took from the pool minus those it returned
int64_t g_allocs = 0, g_mallocs = 0, g_bytes = 0, g_inuse = 0;

size_t round_size(size_t b) {
  if (b <= (size_t(1) << 20)) return (b + 255) & ~size_t(255);
  size_t top = 1;
  while (top < b) top <<= 1;
  const size_t step = top >> 3;
  return (b + step - 1) / step * step;
}

}  // namespace

void *pool_alloc(size_t bytes) {
  const size_t r = round_size(bytes);
  {
    std::lock_guard<std::mutex> lk(g_mu);
    auto it = g_free.find(r);
    if (it != g_free.end() && !it->second.empty()) {
      void *p = it->second.back();
      it->second.pop_back();
      g_idle.erase(p);
      ++g_allocs;
      g_inuse += (int64_t)r;
      t_net += (int64_t)r;
      return p;
    }
  }
  void *p = nullptr;
  hipError_t e = hipMalloc(&p, r);
  if (e != hipSuccess) {
    (void)hipGetLastError();
    pool_trim();
    e = hipMalloc(&p, r);
    if (e != hipSuccess) {
      (void)hipGetLastError();
      throw Error{PHS_ERR_OUT_OF_MEMORY, "hipMalloc of " + std::to_string(r) + " bytes failed"};
    }
  }
  std::lock_guard<std::mutex> lk(g_mu);
  g_size[p] = r;
  ++g_allocs;
  ++g_mallocs;
  g_bytes += (int64_t)r;
  g_inuse += (int64_t)r;
  t_net += (int64_t)r;
  return p;
}

void pool_free(void *p) {
  if (!p) return;
  // a block is parked once: a second free of the same pointer is ignored
  for (void *q : t_pending)
    if (q == p) return;
  {
    std::lock_guard<std::mutex> lk(g_mu);
    auto it = g_size.find(p);
    if (g_idle.count(p) || it == g_size.end()) return;
    t_net -= (int64_t)it->second;
  }
  t_pending.push_back(p);
}

int64_t pool_thread_net() { return t_net; }

void pool_mark_idle() {
  if (t_pending.empty()) return;
  (void)hipDeviceSynchronize();
  std::lock_guard<std::mutex> lk(g_mu);
  for (void *p : t_pending) {
    auto it = g_size.find(p);
    if (it != g_size.end() && !g_idle.count(p)) {
      g_free[it->second].push_back(p);
      g_idle[p] = true;
      g_inuse -= (int64_t)it->second;
    }
  }
  t_pending.clear();
}

void pool_trim() {
  (void)hipDeviceSynchronize();
  std::lock_guard<std::mutex> lk(g_mu);
  for (auto &kv : g_free)
    for (void *p : kv.second) {
      (void)hipFree(p);
      g_bytes -= (int64_t)g_size[p];
      g_size.erase(p);
      g_idle.erase(p);
    }
  g_free.clear();
}

void pool_stats(int64_t *allocs, int64_t *device_mallocs, int64_t *bytes_in_use,
                int64_t *bytes_held) {
  std::lock_guard<std::mutex> lk(g_mu);
  if (allocs) *allocs = g_allocs;
  if (device_mallocs) *device_mallocs = g_mallocs;
  if (bytes_in_use) *bytes_in_use = g_inuse;
  if (bytes_held) *bytes_held = g_bytes;
}

}  // namespace phs
