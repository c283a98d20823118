// alloc.hip -- the block cache behind DBuf (pool_alloc, pool_free,
// pool_trim): size classes of four per doubling, one free list per (device,
// class), released blocks pending until one device-wide wait makes them
// reusable.
#include <mutex>
#include <unordered_map>
#include <vector>

#include "dc_common.h"

namespace dc {

namespace {

// The smallest size m * 2^e >= bytes with m in 4..8 (8 * 2^e is 4 * 2^(e+1)).
size_t size_class(size_t bytes) {
  if (bytes <= 256) return 256;
  int e = 0;
  while ((size_t(8) << e) < bytes) ++e;  // 8 * 2^e >= bytes
  for (size_t m = 4; m <= 8; ++m)
    if ((m << e) >= bytes) return m << e;
  return size_t(8) << e;
}

struct Block {
  void* p;
  size_t bytes;
  int dev;
};

struct Cache {
  std::mutex mu;
  std::unordered_map<void*, int> live;  // device of every block handed out
  std::unordered_map<uint64_t, std::vector<void*>> free;  // (device, class) -> blocks
  std::vector<Block> pending;  // released, reusable after a device-wide wait
};

// never destroyed: DBufs with static storage release into it at exit
Cache& cache() {
  static Cache* c = new Cache();
  return *c;
}

uint64_t key_of(int dev, size_t bytes) { return (uint64_t(uint32_t(dev)) << 48) ^ bytes; }

// caller holds the lock
void settle_pending(Cache& c) {
  if (c.pending.empty()) return;
  int cur = 0;
  (void)hipGetDevice(&cur);
  bool waited_cur = false;
  for (const Block& b : c.pending) {  // every device that released a block waits once
    if (b.dev == cur) {
      if (!waited_cur) (void)hipDeviceSynchronize();
      waited_cur = true;
      continue;
    }
    bool seen = false;
    for (const Block& a : c.pending) {
      if (&a == &b) break;
      seen = seen || a.dev == b.dev;
    }
    if (seen) continue;
    (void)hipSetDevice(b.dev);
    (void)hipDeviceSynchronize();
    (void)hipSetDevice(cur);
  }
  for (const Block& b : c.pending) c.free[key_of(b.dev, b.bytes)].push_back(b.p);
  c.pending.clear();
}

}  // namespace

void* pool_alloc(size_t bytes, size_t* got) {
  const size_t cls = size_class(bytes);
  int dev = 0;
  DC_HIP(hipGetDevice(&dev));
  Cache& c = cache();
  std::lock_guard<std::mutex> lk(c.mu);
  settle_pending(c);
  auto it = c.free.find(key_of(dev, cls));
  void* p = nullptr;
  if (it != c.free.end() && !it->second.empty()) {
    p = it->second.back();
    it->second.pop_back();
  } else {
    hipError_t e = hipMalloc(&p, cls);
    if (e == hipErrorOutOfMemory || e == hipErrorMemoryAllocation) {
      (void)hipGetLastError();  // the cached blocks go first, then one more try
      (void)hipDeviceSynchronize();
      for (auto& kv : c.free)
        for (void* q : kv.second) {
          c.live.erase(q);
          (void)hipFree(q);
        }
      c.free.clear();
      e = hipMalloc(&p, cls);
    }
    if (e != hipSuccess)
      throw DeviceError(e, std::string("hipMalloc(") + std::to_string(cls) + ") -> " +
                               hipGetErrorString(e));
  }
  c.live[p] = dev;
  *got = cls;
  return p;
}

void pool_free(void* p, size_t bytes) noexcept {
  if (!p) return;
  Cache& c = cache();
  std::lock_guard<std::mutex> lk(c.mu);
  auto it = c.live.find(p);
  const int dev = it != c.live.end() ? it->second : 0;
  c.pending.push_back(Block{p, bytes, dev});
}

void pool_trim() noexcept {
  Cache& c = cache();
  std::lock_guard<std::mutex> lk(c.mu);
  settle_pending(c);
  for (auto& kv : c.free)
    for (void* q : kv.second) {
      c.live.erase(q);
      (void)hipFree(q);
    }
  c.free.clear();
}

}  // namespace dc
