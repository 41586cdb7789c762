// Minimal fork-join loop over host threads for the topology and decomposition
// builders (each iteration writes disjoint outputs).
#pragma once

#include <algorithm>
#include <atomic>
#include <cstdint>
#include <exception>
#include <mutex>
#include <thread>
#include <vector>

namespace mw {

inline int host_threads() {
  unsigned h = std::thread::hardware_concurrency();
  if (h == 0) h = 1;
  return (int)std::min<unsigned>(h, 16);
}

// f(i) for i in [0, n); dynamic chunks; the first exception is rethrown.
template <class F>
void parallel_for(int64_t n, F&& f, int64_t chunk = 0) {
  if (n <= 0) return;
  int nth = host_threads();
  if (chunk <= 0) chunk = std::max<int64_t>(1, n / (nth * 16));
  if (nth == 1 || n <= chunk) {
    for (int64_t i = 0; i < n; ++i) f(i);
    return;
  }
  std::atomic<int64_t> next(0);
  std::exception_ptr err;
  std::mutex mu;
  auto work = [&]() {
    try {
      for (;;) {
        int64_t b = next.fetch_add(chunk);
        if (b >= n) break;
        int64_t e = std::min(n, b + chunk);
        for (int64_t i = b; i < e; ++i) f(i);
      }
    } catch (...) {
      std::lock_guard<std::mutex> g(mu);
      if (!err) err = std::current_exception();
      next.store(n);
    }
  };
  std::vector<std::thread> th;
  for (int k = 1; k < nth; ++k) th.emplace_back(work);
  work();
  for (auto& t : th) t.join();
  if (err) std::rethrow_exception(err);
}

}  // namespace mw

namespace mw {

// f(worker, i) for i in [0, n) with one item at a time per worker; `worker`
// in [0, host_threads()) lets each worker keep its own scratch memory.
template <class F>
void parallel_items(int64_t n, F&& f) {
  if (n <= 0) return;
  int nth = (int)std::min<int64_t>(host_threads(), n);
  std::atomic<int64_t> next(0);
  std::exception_ptr err;
  std::mutex mu;
  auto work = [&](int w) {
    try {
      for (;;) {
        int64_t i = next.fetch_add(1);
        if (i >= n) break;
        f(w, i);
      }
    } catch (...) {
      std::lock_guard<std::mutex> g(mu);
      if (!err) err = std::current_exception();
      next.store(n);
    }
  };
  std::vector<std::thread> th;
  for (int k = 1; k < nth; ++k) th.emplace_back(work, k);
  work(0);
  for (auto& t : th) t.join();
  if (err) std::rethrow_exception(err);
}

}  // namespace mw
