#include "mem.hpp"

#include <cstdint>
#include <mutex>
#include <set>
#include <vector>

#include "common.hpp"

namespace spaqr {

namespace {
std::mutex g_mu;
std::set<int> g_ready;
std::vector<PinnedChunk> g_free;
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
  void* p = nullptr;
  const hipError_t e = hipMallocAsync(&p, bytes ? bytes : 256, s);
  if (e != hipSuccess || !p) throw Error(SPAQR_ENOMEM, "device allocation failed");
  return p;
}

void dev_free(void* p, hipStream_t s) {
  if (p) (void)hipFreeAsync(p, s);
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

}  // namespace spaqr
