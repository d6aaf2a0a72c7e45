// Learned index over the sorted keys: a monotone router network picks one of
// kLeaves linear leaves, the leaf predicts the rank of a key, and an exact
// per-leaf error window plus a last-mile binary search gives the lower bound.
// A verification of the result falls back to a full binary search, so the
// answer always equals std::lower_bound over the keys.
#pragma once

#include <hip/hip_runtime.h>

#include <cstdint>

namespace sfc {

constexpr int kHidden = 32;
constexpr int kLeaves = 4096;
constexpr uint32_t kSamples = 1u << 16;   // (key, rank) pairs the router trains on
// Parameter layout: w1[32], b1[32], W2[32][32] (row = output unit), b2[32],
// w3[32], b3.
constexpr int kOffW1 = 0;
constexpr int kOffB1 = kOffW1 + kHidden;
constexpr int kOffW2 = kOffB1 + kHidden;
constexpr int kOffB2 = kOffW2 + kHidden * kHidden;
constexpr int kOffW3 = kOffB2 + kHidden;
constexpr int kOffB3 = kOffW3 + kHidden;
constexpr int kParams = kOffB3 + 1;   // 1153

struct LeafRec {
  uint64_t base;   // smallest key of the leaf (0 for an empty leaf)
  double a, b;     // rank ~ a + b * (key - base)
  uint32_t S, E;   // the leaf's keys are keys[S..E)
  int32_t elo, ehi;   // lower bound - prediction lies in [elo, ehi]
};

// Router input: the top 24 bits of the key as a float in [0, 1) (exact, so
// the map key -> x is monotone).
__device__ __forceinline__ float router_input(uint64_t key) {
  return (float)(uint32_t)(key >> 40) * 0x1p-24f;
}

// The network's output for input x: clip-ramp units, fused multiply-adds in
// a fixed order.  With w1, W2, w3 >= 0 every step is non-decreasing in its
// inputs, and so is its rounding: the output is monotone in x.
__device__ __forceinline__ float router_output(const float* __restrict__ P, float x) {
  float h1[kHidden];
#pragma unroll
  for (int j = 0; j < kHidden; ++j)
    h1[j] = fminf(fmaxf(__fmaf_rn(P[kOffW1 + j], x, P[kOffB1 + j]), 0.f), 1.f);
  float y = P[kOffB3];
#pragma unroll 4
  for (int i = 0; i < kHidden; ++i) {
    float a = P[kOffB2 + i];
#pragma unroll
    for (int j = 0; j < kHidden; ++j) a = __fmaf_rn(P[kOffW2 + i * kHidden + j], h1[j], a);
    y = __fmaf_rn(P[kOffW3 + i], fminf(fmaxf(a, 0.f), 1.f), y);
  }
  return y;
}

__device__ __forceinline__ uint32_t router_leaf(const float* __restrict__ P, uint64_t key) {
  const float y = router_output(P, router_input(key));
  float f = floorf(y * (float)kLeaves);
  f = fminf(fmaxf(f, 0.f), (float)(kLeaves - 1));
  return (uint32_t)f;
}

// The leaf's rank prediction, rounded to nearest and clamped to [S, E].
__device__ __forceinline__ int64_t leaf_predict(const LeafRec& L, uint64_t key) {
#pragma clang fp contract(off)
  const double u = key >= L.base ? (double)(key - L.base) : -(double)(L.base - key);
  double p = floor(L.a + L.b * u + 0.5);
  p = fmin(fmax(p, (double)L.S), (double)L.E);
  return (int64_t)p;
}

// First index i in [lo, hi) with keys[i] >= k, hi if none.
__device__ __forceinline__ uint64_t lower_bound_in(const uint64_t* __restrict__ keys, uint64_t lo,
                                                   uint64_t hi, uint64_t k) {
  uint64_t len = hi - lo;
  while (len > 0) {
    const uint64_t h = len >> 1;
    if (keys[lo + h] < k) {
      lo += h + 1;
      len -= h + 1;
    } else {
      len = h;
    }
  }
  return lo;
}

// Lower bound of k through the learned index; *fell_back is set when the
// verification failed and the full binary search answered.
__device__ __forceinline__ uint64_t learned_lower_bound(const uint64_t* __restrict__ keys,
                                                       uint64_t n, const float* __restrict__ P,
                                                       const LeafRec* __restrict__ leaves,
                                                       uint64_t k, bool* fell_back) {
  const LeafRec L = leaves[router_leaf(P, k)];
  const int64_t p = leaf_predict(L, k);
  int64_t wlo = p + L.elo, whi = p + L.ehi;
  wlo = wlo < (int64_t)L.S ? (int64_t)L.S : wlo;
  whi = whi > (int64_t)L.E ? (int64_t)L.E : whi;
  // The leaves describe the keys they were fitted on; the clamp to [0, n]
  // keeps every probe inside the array should they ever be stale.
  whi = whi > (int64_t)n ? (int64_t)n : whi;
  wlo = wlo > whi ? whi : wlo;
  if (whi < wlo) whi = wlo;
  const uint64_t r = lower_bound_in(keys, (uint64_t)wlo, (uint64_t)whi, k);
  const bool ok = (r == 0 || keys[r - 1] < k) && (r == n || keys[r] >= k);
  *fell_back = !ok;
  return ok ? r : lower_bound_in(keys, 0, n, k);
}

}  // namespace sfc
