// Host thread pool for the per-query stages (bit-blasting, splitting and
// witness checks are independent across queries).  The workers live for
// the whole process and sleep between jobs, so a call costs a wake-up, not
// a thread start.
#pragma once
#include <sched.h>

#include <algorithm>
#include <atomic>
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
    {
      std::lock_guard<std::mutex> g(mu_);
      job_ = &fn;
      n_ = n;
      next_.store(0);
      err_ = nullptr;
      participants_ = unsigned(std::min<size_t>(workers_.size(), n - 1));
      remaining_ = participants_;
      gen_++;
    }
    cv_.notify_all();
    work();
    std::unique_lock<std::mutex> g(mu_);
    done_cv_.wait(g, [&] { return remaining_ == 0; });
    job_ = nullptr;
    if (err_) std::rethrow_exception(err_);
  }

  ~HostPool() {
    {
      std::lock_guard<std::mutex> g(mu_);
      stop_ = true;
      gen_++;
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
      size_t i = next_.fetch_add(1);
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

  void loop(unsigned id) {
    uint64_t seen = 0;
    for (;;) {
      {
        std::unique_lock<std::mutex> g(mu_);
        cv_.wait(g, [&] { return stop_ || gen_ != seen; });
        if (stop_) return;
        seen = gen_;
        // only the first `participants_` workers of a job take part
        if (id > participants_) continue;
      }
      work();
      std::lock_guard<std::mutex> g(mu_);
      if (--remaining_ == 0) done_cv_.notify_all();
    }
  }

  std::vector<std::thread> workers_;
  std::mutex mu_, call_mu_;
  std::condition_variable cv_, done_cv_;
  const std::function<void(size_t)>* job_ = nullptr;
  size_t n_ = 0;
  std::atomic<size_t> next_{0};
  std::exception_ptr err_;
  unsigned participants_ = 0, remaining_ = 0;
  uint64_t gen_ = 0;
  bool stop_ = false;
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
