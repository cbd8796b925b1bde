// Caching device allocator.
//
// A tree owns a few hundred device buffers (sorted data, cell arrays, lists,
// expansions, solver workspaces).  Returning them to the driver and asking
// for them again on every build costs tens of microseconds per call, which
// adds up to a sizeable part of a build-solve-destroy cycle.  Freed blocks
// are therefore kept per device and handed out again for requests of a
// close size.
//
// A freed block may still be in use by kernels queued before the free, on
// any stream.  Such blocks first go to a pending list; the first request
// that would reuse one synchronises the device once and moves every pending
// block to the ready list.  A request that fails for lack of memory returns
// every cached block of its device to the driver and tries once more.
#include <hip/hip_runtime.h>

#include <cstdlib>
#include <map>
#include <mutex>
#include <unordered_map>
#include <vector>

#include "common.h"

namespace bemfmm {
namespace {

constexpr size_t ROUND = 512;  // sizes are rounded up to this many bytes

struct DevCache {
  std::multimap<size_t, void *> ready;    // size -> block, safe to reuse
  std::vector<std::pair<size_t, void *>> pending;  // freed, maybe still in use
  size_t cached_bytes = 0;                // ready + pending
  size_t limit = 0;                       // upper bound of cached_bytes
  bool limit_set = false;
};

struct Cache {
  std::mutex mu;
  std::unordered_map<void *, std::pair<int, size_t>> live;  // block -> (device, size)
  std::map<int, DevCache> dev;
};

// Bytes a device keeps cached at most: BEMFMM_CACHE_LIMIT_MB, else half of
// the device's memory.  A large tree (10^7 panels) holds about 100 GB, and
// returning blocks of that size to the driver can stall for a second, so the
// default keeps a whole tree's worth for the next build.
size_t cache_limit() {
  if (const char *e = getenv("BEMFMM_CACHE_LIMIT_MB")) return (size_t)atoll(e) << 20;
  size_t fr = 0, total = 0;
  if (hipMemGetInfo(&fr, &total) != hipSuccess) {
    (void)hipGetLastError();
    return (size_t)32768 << 20;
  }
  return total / 2;
}

Cache &cache() {
  static Cache *c = new Cache();  // never destroyed: blocks live until exit
  return *c;
}

void flush_device(DevCache &d) {
  if (!d.pending.empty()) (void)hipDeviceSynchronize();
  for (auto &kv : d.ready) (void)hipFree(kv.second);
  for (auto &kv : d.pending) (void)hipFree(kv.second);
  d.ready.clear();
  d.pending.clear();
  d.cached_bytes = 0;
}

}  // namespace

void *dev_alloc(size_t bytes) {
  if (bytes == 0) return nullptr;
  const size_t sz = (bytes + ROUND - 1) / ROUND * ROUND;
  int device = 0;
  HIP_OK(hipGetDevice(&device));
  Cache &c = cache();
  std::lock_guard<std::mutex> lk(c.mu);
  DevCache &d = c.dev[device];
  if (!d.limit_set) {
    d.limit = cache_limit();
    d.limit_set = true;
  }
  // best fit among blocks of at most 1/8 more than requested
  const size_t slack = sz / 8;
  auto take = [&](void) -> void * {
    auto it = d.ready.lower_bound(sz);
    if (it == d.ready.end() || it->first > sz + slack) return nullptr;
    void *p = it->second;
    const size_t bsz = it->first;
    d.ready.erase(it);
    d.cached_bytes -= bsz;
    c.live[p] = {device, bsz};
    return p;
  };
  if (void *p = take()) return p;
  if (!d.pending.empty()) {
    bool fits = false;
    for (auto &kv : d.pending) fits |= kv.first >= sz && kv.first <= sz + slack;
    if (fits) {
      HIP_OK(hipDeviceSynchronize());
      for (auto &kv : d.pending) d.ready.emplace(kv.first, kv.second);
      d.pending.clear();
      if (void *p = take()) return p;
    }
  }
  void *p = nullptr;
  hipError_t e = hipMalloc(&p, sz);
  if (e == hipErrorOutOfMemory) {
    (void)hipGetLastError();
    flush_device(d);
    e = hipMalloc(&p, sz);
  }
  if (e != hipSuccess) {
    (void)hipGetLastError();
    BF_THROW(e == hipErrorOutOfMemory ? BEMFMM_ENOMEM : BEMFMM_EDEVICE,
             std::string("device allocation of ") + std::to_string(bytes) + " bytes: " + hipGetErrorString(e));
  }
  c.live[p] = {device, sz};
  return p;
}

void dev_free(void *p) noexcept {
  if (!p) return;
  Cache &c = cache();
  std::lock_guard<std::mutex> lk(c.mu);
  auto it = c.live.find(p);
  if (it == c.live.end()) return;
  const int device = it->second.first;
  const size_t sz = it->second.second;
  c.live.erase(it);
  DevCache &d = c.dev[device];
  if (d.cached_bytes + sz > d.limit) {
    (void)hipFree(p);  // waits for the device like any hipFree
    return;
  }
  d.pending.emplace_back(sz, p);
  d.cached_bytes += sz;
}

void dev_cache_release() {
  Cache &c = cache();
  std::lock_guard<std::mutex> lk(c.mu);
  int cur = 0;
  (void)hipGetDevice(&cur);
  for (auto &kv : c.dev) {
    if (kv.second.ready.empty() && kv.second.pending.empty()) continue;
    (void)hipSetDevice(kv.first);
    flush_device(kv.second);
  }
  (void)hipSetDevice(cur);
}

}  // namespace bemfmm
