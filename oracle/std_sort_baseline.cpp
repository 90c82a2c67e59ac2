// std_sort_baseline.cpp -- the library sort as a CPU reference point for the
// benchmark (test infrastructure, like the oracle beside it): std::sort of
// fp64 keys on one thread, timed around the call.
#include <algorithm>
#include <chrono>
#include <cstddef>

extern "C" double stdsort_f64_seconds(double* x, size_t n) {
  const auto t0 = std::chrono::steady_clock::now();
  std::sort(x, x + n);
  const auto t1 = std::chrono::steady_clock::now();
  return std::chrono::duration<double>(t1 - t0).count();
}
