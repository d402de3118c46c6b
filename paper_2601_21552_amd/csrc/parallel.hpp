// Host thread pool for the per-query stages (bit-blasting, splitting and
// witness checks are independent across queries).  The workers live for
// the whole process.  After a job they spin briefly on the job counter
// before they sleep, so the back-to-back parallel stages of one call (split,
// walk, witness checks) start without a wake-up each.
#pragma once
#include <sched.h>

#include <algorithm>
#include <atomic>
#include <chrono>
#include <condition_variable>
#include <cstdlib>
#include <exception>
#include <functional>
#include <mutex>
#include <thread>
#include <vector>

namespace scuba {

// Threads used by the host stages: SCUBA_HOST_THREADS if set, else the CPUs
// this process may run on, at most 64.
inline unsigned host_threads() {
  if (const char* s = std::getenv("SCUBA_HOST_THREADS")) {
    int v = std::atoi(s);
    if (v > 0) return unsigned(std::min(v, 256));
  }
  cpu_set_t set;
  unsigned n = 0;
  if (sched_getaffinity(0, sizeof(set), &set) == 0) n = unsigned(CPU_COUNT(&set));
  if (!n) n = std::thread::hardware_concurrency();
  return std::max(1u, std::min(n ? n : 1u, 64u));
}

inline void cpu_relax() { __builtin_ia32_pause(); }

class HostPool {
 public:
  static HostPool& get() {
    static HostPool pool(host_threads());
    return pool;
  }

  // fn(i) for i in [0, n) on the caller and the workers; the first exception
  // is rethrown.  A call from inside a job runs serially (no nesting).
  void run(size_t n, const std::function<void(size_t)>& fn) {
    if (in_job_ || workers_.empty() || n <= 1) {
      for (size_t i = 0; i < n; i++) fn(i);
      return;
    }
    std::unique_lock<std::mutex> call(call_mu_);   // one job at a time
    // the job's fields are published by the release store of gen_, which
    // also carries the number of workers that take part
    job_ = &fn;
    n_ = n;
    next_.store(0, std::memory_order_relaxed);
    err_ = nullptr;
    const uint64_t parts = std::min<size_t>(workers_.size(), n - 1);   // < 2^16 workers
    remaining_.store(unsigned(parts), std::memory_order_relaxed);
    seq_++;
    gen_.store((seq_ << 16) | parts, std::memory_order_release);
    {
      // a worker that checked gen_ before the increment is either still
      // spinning (and sees it) or waits on cv_ (and gets the notify)
      std::lock_guard<std::mutex> g(mu_);
    }
    cv_.notify_all();
    work();
    // the caller's share is done: the workers hold at most one item each
    for (uint32_t spins = 0; remaining_.load(std::memory_order_acquire) != 0; spins++) {
      if (spins < 4096) cpu_relax();
      else std::this_thread::yield();
    }
    job_ = nullptr;
    if (err_) std::rethrow_exception(err_);
  }

  ~HostPool() {
    stop_.store(true);
    seq_++;
    gen_.store(seq_ << 16, std::memory_order_release);
    {
      std::lock_guard<std::mutex> g(mu_);
    }
    cv_.notify_all();
    for (auto& t : workers_) t.join();
  }

 private:
  explicit HostPool(unsigned threads) {
    for (unsigned t = 1; t < threads; t++) workers_.emplace_back([this, t] { loop(t); });
  }

  void work() {
    in_job_ = true;
    for (;;) {
      size_t i = next_.fetch_add(1, std::memory_order_relaxed);
      if (i >= n_) break;
      try {
        (*job_)(i);
      } catch (...) {
        std::lock_guard<std::mutex> g(mu_);
        if (!err_) err_ = std::current_exception();
        next_.store(n_);
      }
    }
    in_job_ = false;
  }

  // Waits for a generation other than `seen`: spins for about kSpinUs
  // microseconds, then sleeps on cv_.
  uint64_t wait_job(uint64_t seen) {
    using Clock = std::chrono::steady_clock;
    const auto until = Clock::now() + std::chrono::microseconds(kSpinUs);
    for (uint32_t spins = 0;; spins++) {
      uint64_t g = gen_.load(std::memory_order_acquire);
      if (g != seen) return g;
      cpu_relax();
      if ((spins & 255) == 255 && Clock::now() > until) break;
    }
    std::unique_lock<std::mutex> lk(mu_);
    cv_.wait(lk, [&] { return gen_.load(std::memory_order_acquire) != seen; });
    return gen_.load(std::memory_order_acquire);
  }

  void loop(unsigned id) {
    uint64_t seen = 0;
    for (;;) {
      seen = wait_job(seen);
      if (stop_.load()) return;
      // only the first workers of a job take part (the count is read from
      // the same word as the job's generation, so a worker never joins a
      // job it was not counted in)
      if (id > (seen & 0xffff)) continue;
      work();
      remaining_.fetch_sub(1, std::memory_order_acq_rel);
    }
  }

  static constexpr int kSpinUs = 300;
  std::vector<std::thread> workers_;
  std::mutex mu_, call_mu_;
  std::condition_variable cv_;
  const std::function<void(size_t)>* job_ = nullptr;
  size_t n_ = 0;
  std::atomic<size_t> next_{0};
  std::exception_ptr err_;
  uint64_t seq_ = 0;   // written under call_mu_ (and by the destructor)
  std::atomic<unsigned> remaining_{0};
  std::atomic<uint64_t> gen_{0};
  std::atomic<bool> stop_{false};
  static thread_local bool in_job_;
};

inline thread_local bool HostPool::in_job_ = false;

// Runs fn(i) for i in [0, n) on the host pool (dynamic scheduling).
template <typename F>
void parallel_for(size_t n, F&& fn) {
  const std::function<void(size_t)> f = std::forward<F>(fn);
  HostPool::get().run(n, f);
}

}  // namespace scuba
