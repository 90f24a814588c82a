// Device and pinned-host memory helpers.  Device memory comes from the
// stream-ordered allocator with a release threshold high enough that the
// pool keeps what it maps; blocks the library frees stay in its own cache
// and are reused on the stream they were freed on (the pool's own free path
// can stall the host for milliseconds).  The cache goes back to the pool
// only when an allocation fails.  Streams are expected to outlive the
// blocks freed on them.  Pinned staging chunks are recycled through a
// process-wide free list (allocating pinned memory costs milliseconds).
#pragma once

#include <hip/hip_runtime.h>

#include <cstddef>
#include <utility>

namespace spaqr {

void mem_setup(hipStream_t s);                    // once per device
void* dev_alloc(size_t bytes, hipStream_t s);     // stream-ordered, throws ENOMEM
void dev_free(void* p, hipStream_t s);            // stream-ordered, NULL is a no-op
// Returns every cached device block and every pooled pinned chunk to the
// runtime (after a device synchronization).  Blocks and chunks still held
// by live objects are untouched; the caches refill on demand afterwards.
void mem_release_all();
// When the freed blocks the library keeps for reuse exceed a quarter of the
// device's memory (a large factorization just ended), returns them to the
// stream-ordered pool and the pool's unused pages to the device, so that a
// differently sized factorization can map them (synchronizes the device).
void mem_trim_if_large();

struct PinnedChunk {
  char* p = nullptr;
  size_t size = 0;
};
PinnedChunk pinned_acquire(size_t bytes);          // at least `bytes`
void pinned_release(PinnedChunk c);

// A host buffer in pinned memory from the recycled pool when pinned memory
// can be had (copies from it need no staging), else in ordinary memory.
// Moved, never copied; the pinned chunk goes back to the pool on release.
class HostBuffer {
 public:
  HostBuffer() = default;
  explicit HostBuffer(size_t bytes);
  ~HostBuffer() { reset(); }
  HostBuffer(HostBuffer&& o) noexcept { *this = std::move(o); }
  HostBuffer& operator=(HostBuffer&& o) noexcept;
  HostBuffer(const HostBuffer&) = delete;
  HostBuffer& operator=(const HostBuffer&) = delete;
  char* data() const { return pinned_ ? c_.p : heap_; }
  bool pinned() const { return pinned_; }

 private:
  void reset();
  PinnedChunk c_;
  char* heap_ = nullptr;
  bool pinned_ = false;
};

}  // namespace spaqr
