// Optional per-kernel timing with HIP events on the launching stream, plus the
// algorithmic work each launch performs (flops and bytes the method itself
// must move).  Off by default; spaqr_profile_enable() switches it on.
#pragma once

#include <hip/hip_runtime.h>

namespace spaqr {

bool prof_on();
bool prof_wants(const char* name);
void prof_record(const char* name, hipStream_t s, hipEvent_t a, hipEvent_t b, double flops, double bytes);
// Work known only after the launches ran (e.g. from ranks read back later).
void prof_add(const char* name, double flops, double bytes);
// Host wall time of a driver phase (recorded like a launch of `ms`).
void prof_host(const char* name, double ms);
// Process-wide count of launches per kernel family (the kernel template's
// name, e.g. "k_qr"), always on; read with spaqr_kernel_launches.
void count_launch(const char* kernel);
double now_ms();

struct HostScope {
  explicit HostScope(const char* name) : name_(name), live_(prof_wants(name)), t0_(live_ ? now_ms() : 0.0) {}
  ~HostScope() { stop(); }
  // records now instead of at the end of the scope
  void stop() {
    if (live_) prof_host(name_, now_ms() - t0_);
    live_ = false;
  }
  HostScope(const HostScope&) = delete;
  HostScope& operator=(const HostScope&) = delete;

 private:
  const char* name_;
  bool live_;
  double t0_;
};

struct ProfScope {
  ProfScope(const char* name, hipStream_t s, double flops, double bytes)
      : name_(name), s_(s), flops_(flops), bytes_(bytes) {
    if (prof_wants(name)) {
      (void)hipEventCreate(&a_);
      (void)hipEventCreate(&b_);
      (void)hipEventRecord(a_, s_);
      live_ = true;
    }
  }
  ~ProfScope() {
    if (live_) {
      (void)hipEventRecord(b_, s_);
      prof_record(name_, s_, a_, b_, flops_, bytes_);
    }
  }
  ProfScope(const ProfScope&) = delete;
  ProfScope& operator=(const ProfScope&) = delete;

 private:
  const char* name_;
  hipStream_t s_;
  double flops_, bytes_;
  hipEvent_t a_{}, b_{};
  bool live_ = false;
};

}  // namespace spaqr
