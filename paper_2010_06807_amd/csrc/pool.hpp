// A small persistent host thread pool for the per-problem planning of a
// batched stage (each factorization's launch lists are built from its own
// data only, so the problems of a batch plan in parallel).
#pragma once

#include <algorithm>
#include <atomic>
#include <condition_variable>
#include <exception>
#include <functional>
#include <mutex>
#include <thread>
#include <vector>

namespace spaqr {

// Worker threads for per-problem host work: one per core beside the
// calling thread, at most 15 (a GPU's share of a host is 16 cores).
inline int host_pool_threads() {
  const unsigned hc = std::thread::hardware_concurrency();
  return (int)std::min<unsigned>(15, hc > 1 ? hc - 1 : 0);
}

class HostPool {
 public:
  explicit HostPool(int threads) {
    for (int i = 0; i < threads; ++i) th_.emplace_back([this] { worker(); });
  }
  ~HostPool() {
    {
      std::lock_guard<std::mutex> lk(mu_);
      stop_ = true;
    }
    cv_.notify_all();
    for (auto& t : th_) t.join();
  }
  int size() const { return (int)th_.size(); }  // worker threads (the caller also runs)
  HostPool(const HostPool&) = delete;
  HostPool& operator=(const HostPool&) = delete;

  // fn(i) for i < n on the workers and the calling thread; rethrows the first
  // exception after every index has finished.
  void run(int n, const std::function<void(int)>& fn) {
    if (n <= 0) return;
    if (n == 1 || th_.empty()) {
      for (int i = 0; i < n; ++i) fn(i);
      return;
    }
    {
      std::lock_guard<std::mutex> lk(mu_);
      fn_ = &fn;
      n_ = n;
      next_.store(0);
      left_ = n;
      err_ = nullptr;
      ++gen_;
    }
    cv_.notify_all();
    drain();
    // no worker may still be inside drain() when the next run starts
    std::unique_lock<std::mutex> lk(mu_);
    done_cv_.wait(lk, [this] { return left_ == 0 && busy_ == 0; });
    fn_ = nullptr;
    if (err_) std::rethrow_exception(err_);
  }

 private:
  void drain() {
    for (;;) {
      const int i = next_.fetch_add(1);
      if (i >= n_) return;
      try {
        (*fn_)(i);
      } catch (...) {
        std::lock_guard<std::mutex> lk(mu_);
        if (!err_) err_ = std::current_exception();
      }
      std::lock_guard<std::mutex> lk(mu_);
      if (--left_ == 0) done_cv_.notify_all();
    }
  }
  void worker() {
    unsigned seen = 0;
    std::unique_lock<std::mutex> lk(mu_);
    for (;;) {
      cv_.wait(lk, [&] { return stop_ || (gen_ != seen && fn_ != nullptr); });
      if (stop_) return;
      seen = gen_;
      ++busy_;
      lk.unlock();
      drain();
      lk.lock();
      if (--busy_ == 0) done_cv_.notify_all();
    }
  }

  std::vector<std::thread> th_;
  std::mutex mu_;
  std::condition_variable cv_, done_cv_;
  const std::function<void(int)>* fn_ = nullptr;
  int n_ = 0, left_ = 0, busy_ = 0;
  std::atomic<int> next_{0};
  unsigned gen_ = 0;
  bool stop_ = false;
  std::exception_ptr err_;
};

}  // namespace spaqr
