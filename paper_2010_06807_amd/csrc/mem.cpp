#include "mem.hpp"

#include <cstdint>
#include <map>
#include <mutex>
#include <set>
#include <unordered_map>
#include <string>
#include <vector>

#include "common.hpp"

namespace spaqr {

namespace {
std::mutex g_mu;
std::set<int> g_ready;
std::vector<PinnedChunk> g_free;

// Device blocks freed by the library are kept for reuse instead of going
// back to the stream-ordered pool: returning a block there can block the
// host for milliseconds once many blocks are live.  A freed block is handed
// out again only on the stream it was freed on, so stream order keeps the
// reuse after every earlier use.
struct Block {
  void* p;
  hipStream_t s;
};
std::mutex g_dmu;
std::multimap<size_t, Block> g_cache;         // free blocks by size
std::unordered_map<void*, size_t> g_size;     // size of every live block
size_t g_cached = 0;                          // bytes in g_cache

size_t round_block(size_t b) {
  if (b <= (size_t(1) << 20)) return (b + 4095) & ~size_t(4095);
  return (b + (size_t(2) << 20) - 1) & ~((size_t(2) << 20) - 1);
}

// free blocks back to the pool (caller holds g_dmu); the memory is usable
// by every stream once the device has synchronized
void flush_cache() {
  for (auto& kv : g_cache) (void)hipFreeAsync(kv.second.p, kv.second.s);
  g_cache.clear();
  g_cached = 0;
  (void)hipDeviceSynchronize();
}
}  // namespace

void mem_setup(hipStream_t) {
  int dev = 0;
  if (hipGetDevice(&dev) != hipSuccess) return;
  std::lock_guard<std::mutex> lk(g_mu);
  if (g_ready.count(dev)) return;
  hipMemPool_t pool;
  if (hipDeviceGetDefaultMemPool(&pool, dev) == hipSuccess) {
    uint64_t thr = UINT64_MAX;
    (void)hipMemPoolSetAttribute(pool, hipMemPoolAttrReleaseThreshold, &thr);
  }
  g_ready.insert(dev);
}

void* dev_alloc(size_t bytes, hipStream_t s) {
  const size_t sz = round_block(bytes ? bytes : 256);
  std::lock_guard<std::mutex> lk(g_dmu);
  // best fit on the same stream, wasting at most a quarter of the block
  for (auto it = g_cache.lower_bound(sz); it != g_cache.end() && it->first - sz <= it->first / 4; ++it)
    if (it->second.s == s) {
      void* p = it->second.p;
      g_size[p] = it->first;
      g_cached -= it->first;
      g_cache.erase(it);
      return p;
    }
  void* p = nullptr;
  hipError_t e = hipMallocAsync(&p, sz, s);
  if ((e != hipSuccess || !p) && !g_cache.empty()) {
    (void)hipGetLastError();
    flush_cache();
    p = nullptr;
    e = hipMallocAsync(&p, sz, s);
  }
  if (e != hipSuccess || !p) {
    (void)hipGetLastError();
    throw Error(SPAQR_ENOMEM, "device allocation of " + std::to_string(sz) + " bytes failed");
  }
  g_size[p] = sz;
  return p;
}

void dev_free(void* p, hipStream_t s) {
  if (!p) return;
  std::lock_guard<std::mutex> lk(g_dmu);
  auto it = g_size.find(p);
  if (it == g_size.end()) {
    (void)hipFreeAsync(p, s);
    return;
  }
  g_cache.insert({it->second, Block{p, s}});
  g_cached += it->second;
  g_size.erase(it);
}

void mem_trim_if_large() {
  std::lock_guard<std::mutex> lk(g_dmu);
  size_t fr = 0, total = 0;
  if (g_cache.empty() || hipMemGetInfo(&fr, &total) != hipSuccess || g_cached <= total / 4) {
    (void)hipGetLastError();
    return;
  }
  flush_cache();
  int dev = 0;
  hipMemPool_t mp = nullptr;
  if (hipGetDevice(&dev) == hipSuccess && hipDeviceGetDefaultMemPool(&mp, dev) == hipSuccess && mp)
    (void)hipMemPoolTrimTo(mp, 0);
  (void)hipGetLastError();
}

void mem_release_all() {
  {
    std::lock_guard<std::mutex> lk(g_dmu);
    if (!g_cache.empty()) {
      (void)hipDeviceSynchronize();
      for (auto& kv : g_cache) (void)hipFree(kv.second.p);
      g_cache.clear();
      g_cached = 0;
    }
  }
  std::lock_guard<std::mutex> lk(g_mu);
  for (auto& c : g_free) (void)hipHostFree(c.p);
  g_free.clear();
}

PinnedChunk pinned_acquire(size_t bytes) {
  {
    std::lock_guard<std::mutex> lk(g_mu);
    for (size_t i = 0; i < g_free.size(); ++i)
      if (g_free[i].size >= bytes) {
        PinnedChunk c = g_free[i];
        g_free.erase(g_free.begin() + i);
        return c;
      }
  }
  PinnedChunk c;
  c.size = bytes < (size_t(16) << 20) ? (size_t(16) << 20) : bytes;
  if (hipHostMalloc(reinterpret_cast<void**>(&c.p), c.size, hipHostMallocDefault) != hipSuccess || !c.p)
    throw Error(SPAQR_ENOMEM, "pinned host allocation failed");
  return c;
}

void pinned_release(PinnedChunk c) {
  if (!c.p) return;
  std::lock_guard<std::mutex> lk(g_mu);
  g_free.push_back(c);
}

HostBuffer::HostBuffer(size_t bytes) {
  try {
    c_ = pinned_acquire(bytes);
    pinned_ = true;
  } catch (const Error&) {
    (void)hipGetLastError();
    heap_ = new char[bytes ? bytes : 1];
  }
}

HostBuffer& HostBuffer::operator=(HostBuffer&& o) noexcept {
  if (this != &o) {
    reset();
    c_ = o.c_;
    heap_ = o.heap_;
    pinned_ = o.pinned_;
    o.c_ = PinnedChunk{};
    o.heap_ = nullptr;
    o.pinned_ = false;
  }
  return *this;
}

void HostBuffer::reset() {
  if (pinned_) pinned_release(c_);
  delete[] heap_;
  c_ = PinnedChunk{};
  heap_ = nullptr;
  pinned_ = false;
}

}  // namespace spaqr
