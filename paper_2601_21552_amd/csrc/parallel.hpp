// Host thread pool for the per-query stages (bit-blasting, splitting and
// witness checks are independent across queries).
#pragma once
#include <algorithm>
#include <atomic>
#include <cstdlib>
#include <exception>
#include <mutex>
#include <thread>
#include <vector>

namespace scuba {

// Threads used by the host stages: SCUBA_HOST_THREADS if set, else the
// hardware concurrency, at most 64.
inline unsigned host_threads() {
  if (const char* s = std::getenv("SCUBA_HOST_THREADS")) {
    int v = std::atoi(s);
    if (v > 0) return unsigned(std::min(v, 256));
  }
  unsigned h = std::thread::hardware_concurrency();
  return std::max(1u, std::min(h ? h : 1u, 64u));
}

// Runs fn(i) for i in [0, n) on up to host_threads() threads (dynamic
// scheduling).  The first exception thrown by any call is rethrown.
template <typename F>
void parallel_for(size_t n, F&& fn) {
  unsigned nt = unsigned(std::min<size_t>(host_threads(), n));
  if (nt <= 1) {
    for (size_t i = 0; i < n; i++) fn(i);
    return;
  }
  std::atomic<size_t> next{0};
  std::exception_ptr err;
  std::mutex mu;
  auto work = [&] {
    for (;;) {
      size_t i = next.fetch_add(1);
      if (i >= n) return;
      try {
        fn(i);
      } catch (...) {
        std::lock_guard<std::mutex> g(mu);
        if (!err) err = std::current_exception();
        next.store(n);
      }
    }
  };
  std::vector<std::thread> ts;
  for (unsigned t = 1; t < nt; t++) ts.emplace_back(work);
  work();
  for (auto& t : ts) t.join();
  if (err) std::rethrow_exception(err);
}

}  // namespace scuba
