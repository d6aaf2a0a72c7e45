// Host build of the lockstep search of libsfc (search_lockstep_t in
// query_lane.h), checked under the address and undefined-behaviour
// sanitizers against std::lower_bound / std::upper_bound: sorted arrays with
// many repeated keys and lengths 0 to 300 (and a few around powers of two),
// one to four intervals per search, some unused, some empty (klo > khi),
// keys below, inside and above the array, both index widths.  Exits 1 on the
// first disagreement, after printing it.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <cstdio>
#include <cstdlib>
#include <random>
#include <vector>

static inline float __fmaf_rn(float a, float b, float c) { return a * b + c; }
static inline unsigned int __lane_id() { return 0; }

#include "query_lane.h"

using namespace sfc;

static std::mt19937_64 rng(12345);

static uint64_t pick_key(const std::vector<uint64_t>& a) {
  const uint64_t r = rng() % 8;
  if (a.empty() || r == 0) return rng() % 1000;
  if (r == 1) return 0;
  if (r == 2) return ~0ull;
  const uint64_t v = a[rng() % a.size()];
  return r == 3 ? v + 1 : r == 4 ? v - 1 : v;
}

template <typename I, int K>
static bool check(const std::vector<uint64_t>& a, int trial) {
  uint64_t klo[K], khi[K], b[K], e[K];
  bool use[K];
  for (int i = 0; i < K; ++i) {
    klo[i] = pick_key(a);
    khi[i] = pick_key(a);
    if (rng() % 4 != 0 && klo[i] > khi[i]) std::swap(klo[i], khi[i]);
    use[i] = i == 0 || rng() % 3 != 0;
  }
  search_lockstep_t<I, K>(a.data(), (I)a.size(), klo, khi, use, b, e);
  for (int i = 0; i < K; ++i) {
    if (!use[i]) continue;
    const uint64_t wb = std::lower_bound(a.begin(), a.end(), klo[i]) - a.begin();
    const uint64_t we = std::upper_bound(a.begin(), a.end(), khi[i]) - a.begin();
    if (b[i] != wb || e[i] != we) {
      std::printf("trial %d: n=%zu K=%d index bytes=%zu chain %d [%llu, %llu]: got [%llu, %llu) "
                  "want [%llu, %llu)\n",
                  trial, a.size(), K, sizeof(I), i, (unsigned long long)klo[i],
                  (unsigned long long)khi[i], (unsigned long long)b[i], (unsigned long long)e[i],
                  (unsigned long long)wb, (unsigned long long)we);
      return false;
    }
  }
  return true;
}

int main() {
  std::vector<size_t> sizes;
  for (size_t n = 0; n <= 300; ++n) sizes.push_back(n);
  for (size_t p = 512; p <= 8192; p *= 2) {
    sizes.push_back(p - 1);
    sizes.push_back(p);
    sizes.push_back(p + 1);
  }
  int trial = 0;
  for (size_t n : sizes) {
    for (int rep = 0; rep < 40; ++rep, ++trial) {
      std::vector<uint64_t> a(n);
      const uint64_t span = 1 + rng() % (2 * n + 2);   // small spans repeat keys
      for (auto& x : a) x = rng() % 2 == 0 ? rng() % span : 100 + rng() % span;
      if (rep % 5 == 0)
        for (auto& x : a) x = ~0ull - (rng() % span);   // keys near the top
      std::sort(a.begin(), a.end());
      const bool ok = check<uint32_t, 1>(a, trial) && check<uint64_t, 1>(a, trial) &&
                      check<uint32_t, 2>(a, trial) && check<uint64_t, 2>(a, trial) &&
                      check<uint32_t, 4>(a, trial) && check<uint64_t, 4>(a, trial);
      if (!ok) return 1;
    }
  }
  std::printf("%d trials ok\n", trial);
  return 0;
}
