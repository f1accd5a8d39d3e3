// Stable sort on all of the host's cores -- TEST INFRASTRUCTURE ONLY.
//
// The problem's definition (Section 2.3): records in non-decreasing key order,
// equal keys in input order.  The step is libstdc++'s parallel-mode stable
// sort (a multiway merge sort over OpenMP threads); nothing here is shared with
// the GPU path.  Used as the multicore CPU baseline of the benchmark and
// checked against the one-thread definition by the CPU tests.
#include <omp.h>
#include <stddef.h>
#include <stdint.h>

#include <parallel/algorithm>
#include <vector>

extern "C" {

// Sorts keys[0..n) in place with `threads` threads (0 = OpenMP's default);
// returns the number of threads used.
int oracle_psort_u32(uint32_t* keys, size_t n, int threads) {
  const int t = threads > 0 ? threads : omp_get_max_threads();
  omp_set_num_threads(t);
  __gnu_parallel::stable_sort(keys, keys + n);
  return t;
}

// (key, value) records stably ordered by key; keys and values are two arrays.
int oracle_psort_pairs_u64(uint64_t* keys, uint64_t* values, size_t n, int threads) {
  const int t = threads > 0 ? threads : omp_get_max_threads();
  omp_set_num_threads(t);
  struct Rec {
    uint64_t k, v;
  };
  std::vector<Rec> r(n);
#pragma omp parallel for
  for (size_t i = 0; i < n; ++i) r[i] = Rec{keys[i], values[i]};
  __gnu_parallel::stable_sort(r.begin(), r.end(), [](const Rec& a, const Rec& b) { return a.k < b.k; });
#pragma omp parallel for
  for (size_t i = 0; i < n; ++i) {
    keys[i] = r[i].k;
    values[i] = r[i].v;
  }
  return t;
}

}  // extern "C"
