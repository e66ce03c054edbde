// Host-side parallel loop for the setup work that is independent per
// surface or per target leaf (octrees, interaction lists, near candidates).
#pragma once

#include <algorithm>
#include <cstdint>
#include <thread>
#include <vector>

namespace pbt {

// Runs f(i) for every i in [0, n), in contiguous chunks on up to 16 host
// threads (fewer when n / min_per_thread is small).  f must only write state
// owned by index i.
template <typename F>
void parallel_for(int64_t n, F&& f, int64_t min_per_thread = 1) {
  const int64_t hw = std::max<int64_t>(1, (int64_t)std::thread::hardware_concurrency());
  const int64_t nt = std::min<int64_t>({16, hw, (n + min_per_thread - 1) / std::max<int64_t>(min_per_thread, 1)});
  if (nt <= 1) {
    for (int64_t i = 0; i < n; ++i) f(i);
    return;
  }
  const int64_t chunk = (n + nt - 1) / nt;
  std::vector<std::thread> pool;
  pool.reserve(nt);
  for (int64_t t = 0; t < nt; ++t)
    pool.emplace_back([&f, t, chunk, n] {
      const int64_t a = t * chunk, b = std::min(n, a + chunk);
      for (int64_t i = a; i < b; ++i) f(i);
    });
  for (auto& th : pool) th.join();
}

}  // namespace pbt
