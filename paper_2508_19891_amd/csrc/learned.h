// Learned index over the sorted keys.  A monotone router network maps a
// key's top bits to one of kLeaves leaves; a leaf holds a contiguous run
// keys[S..E) and is cut into pieces of kPiece keys; a piece predicts a rank
// by linear interpolation from its first key towards the next piece's, with
// the exact window of (lower bound - prediction) stored per piece, and a
// last-mile binary search in that window gives the lower bound.  A check of
// the result falls back to a full binary search, so the answer always equals
// std::lower_bound over the keys.
//
// The router is evaluated in two equivalent ways.  Training and the fit
// evaluate the network itself.  The fit also reads its tabulation: the
// router is monotone in its 24-bit input X, so leaf(X) is a step function,
// fully described by the first input of every leaf (xb); a table over the
// top 16 bits of X brackets the leaf and a short search in xb finds it.
// Both give the same leaf for every X (the table is built from the same
// device function).
//
// The leaves are contiguous key runs and their pieces tile the sorted array
// in key order, so the pieces' first keys fk are sorted and the piece a key
// k lands in is simply the last one with fk < k: a query finds it through a
// table over the top 20 key bits (the number of pieces whose first key lies
// below each 20-bit prefix) and a scan of the few first keys that share k's
// prefix, without evaluating the router.  Each piece's window covers every
// key from its first key up to the next piece's first key, so the lower
// bound of any k lies in the window of that piece.
//
// On the GPU the cost of a lower bound is its chain of dependent loads, so
// the searches below end in a scan of a few sorted entries (16 for one
// bound, 4 for each of two bounds searched in lockstep, where registers
// decide how many waves run) whose loads are independent of each other: a
// binary search over a few hundred keys takes about eight dependent probes,
// the scan one round trip.
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

constexpr uint32_t kPiece = 256;      // keys per piece (the last piece of a leaf may be shorter)
constexpr int kXBits = 24;            // router input: the top 24 key bits
constexpr int kRouteBits = 16;        // leaf bracket table over the top 16 input bits
constexpr uint32_t kRouteSlots = 1u << kRouteBits;
constexpr int kDirectBits = 20;       // piece table over the top 20 key bits
constexpr uint32_t kDirectSlots = 1u << kDirectBits;

struct PieceRec {
  double s;          // ranks per key unit from the piece's first key
  int32_t elo, ehi;  // lower bound - prediction lies in [elo, ehi]
};

// Device view of a fitted learned index (all arrays in device memory).
struct LearnedView {
  const uint32_t* xb;   // kLeaves + 1: first router input X of each leaf (xb[kLeaves] = 2^24)
  const uint32_t* rt;   // kRouteSlots + 1: leaf of X = min(t << 8, 2^24 - 1)
  const uint2* lp;      // kLeaves + 1: (first key index, first piece) of each leaf;
                        // lp[kLeaves] = (n, number of pieces)
  const uint64_t* fk;   // first key of each piece
  const PieceRec* pr;   // model and window of each piece
  const uint32_t* ps;   // pieces + 1: first key index of each piece (ps[pieces] = n)
  const uint32_t* dt;   // kDirectSlots + 1: pieces whose first key is below t << 44
};

// The same arrays, writable, as the fit carves them from one allocation.
struct LearnedArrays {
  uint32_t* xb = nullptr;
  uint32_t* rt = nullptr;
  uint2* lp = nullptr;
  uint64_t* fk = nullptr;
  PieceRec* pr = nullptr;
  uint32_t* ps = nullptr;
  uint32_t* dt = nullptr;
  uint32_t max_pieces = 0;
  __host__ __device__ LearnedView view() const { return LearnedView{xb, rt, lp, fk, pr, ps, dt}; }
};

// Router input: the top 24 bits of the key as a float in [0, 1) (exact, so
// the map key -> x is monotone).
__device__ __forceinline__ float router_input_x(uint32_t X) { return (float)X * 0x1p-24f; }
__device__ __forceinline__ float router_input(uint64_t key) {
  return router_input_x((uint32_t)(key >> 40));
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

// Leaf of router input X (0 <= X < 2^24), by evaluating the network.
__device__ __forceinline__ uint32_t router_leaf_x(const float* __restrict__ P, uint32_t X) {
  const float y = router_output(P, router_input_x(X));
  float f = floorf(y * (float)kLeaves);
  f = fminf(fmaxf(f, 0.f), (float)(kLeaves - 1));
  return (uint32_t)f;
}

// Leaf of router input X through the tabulation (equal to router_leaf_x).
__device__ __forceinline__ uint32_t route(const LearnedView& v, uint32_t X) {
  const uint32_t t = X >> (kXBits - kRouteBits);
  uint32_t lo = v.rt[t], hi = v.rt[t + 1];   // leaf(X) in [lo, hi]
  while (lo < hi) {                          // largest l in [lo, hi] with xb[l] <= X
    const uint32_t mid = (lo + hi + 1) >> 1;
    if (v.xb[mid] <= X) lo = mid;
    else hi = mid - 1;
  }
  return lo;
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

// The piece's rank prediction for a key k > fk: R + round(s * (k - fk)),
// clamped to [R + 1, Rn] (the bracket the lower bound lies in).
__device__ __forceinline__ int64_t piece_predict(double s, uint64_t fk, uint64_t R, uint64_t Rn,
                                                 uint64_t k) {
#pragma clang fp contract(off)
  const double u = (double)(k - fk);
  double p = (double)R + floor(s * u + 0.5);
  p = fmin(fmax(p, (double)(R + 1)), (double)Rn);
  return (int64_t)p;
}

// ---- two lower bounds in lockstep ------------------------------------------
// A range [klo, khi] needs two lower bounds; walking both chains step by step
// keeps two independent loads in flight at every step (as the interleaved
// binary searches of the plain path do), which halves the dependent latency.

constexpr int kScan2 = 4;   // entries scanned at the end of each search

// Lower bounds of k[i] in [lo[i], hi[i]) of the sorted array a, for i = 0, 1.
__device__ __forceinline__ void lower_bound_scan_pair(const uint64_t* __restrict__ a,
                                                      uint64_t lo[2], const uint64_t hi[2],
                                                      const uint64_t k[2]) {
  uint64_t len[2] = {hi[0] - lo[0], hi[1] - lo[1]};
  while (len[0] > (uint64_t)kScan2 || len[1] > (uint64_t)kScan2) {
    uint64_t x[2] = {0, 0}, h[2];
#pragma unroll
    for (int i = 0; i < 2; ++i) {
      h[i] = len[i] >> 1;
      if (len[i] > (uint64_t)kScan2) x[i] = a[lo[i] + h[i]];
    }
#pragma unroll
    for (int i = 0; i < 2; ++i) {
      if (len[i] > (uint64_t)kScan2) {
        if (x[i] < k[i]) {
          lo[i] += h[i] + 1;
          len[i] -= h[i] + 1;
        } else {
          len[i] = h[i];
        }
      }
    }
  }
  // Only the entries left are loaded (a lane's load of an entry it does not
  // need costs as much as one it does).
  uint64_t v[2][kScan2];
#pragma unroll
  for (int i = 0; i < 2; ++i)
#pragma unroll
    for (int t = 0; t < kScan2; ++t) {
      v[i][t] = 0;
      if ((uint64_t)t < len[i]) v[i][t] = a[lo[i] + t];
    }
#pragma unroll
  for (int i = 0; i < 2; ++i) {
    uint32_t c = 0;
#pragma unroll
    for (int t = 0; t < kScan2; ++t) c += ((uint64_t)t < len[i] && v[i][t] < k[i]) ? 1u : 0u;
    lo[i] += c;
  }
}

// r[i] = lower bound of k[i] over keys[0, n) for i = 0, 1 through the learned
// index: the piece whose first key is the last one below k[i] (the prefix
// table's bracket, then a scan of the first keys that share the prefix), its
// prediction and window, a search of the window, and a check of the result
// against its neighbours, which falls back to binary search over the whole
// array when it fails.  Returns the number of checks that fell back.
__device__ __forceinline__ uint32_t learned_lower_bound_pair(const uint64_t* __restrict__ keys,
                                                            uint64_t n, const LearnedView& v,
                                                            const uint64_t k[2], uint64_t r[2]) {
  // The two keys of a range mostly share their prefix and their piece: the
  // second key then takes the first one's loads.
  uint64_t c[2], chi[2];
  const uint32_t t0 = (uint32_t)(k[0] >> (64 - kDirectBits));
  const uint32_t t1 = (uint32_t)(k[1] >> (64 - kDirectBits));
  c[0] = v.dt[t0];
  chi[0] = v.dt[t0 + 1];
  c[1] = c[0];
  chi[1] = chi[0];
  if (t1 != t0) {
    c[1] = v.dt[t1];
    chi[1] = v.dt[t1 + 1];
  }
  lower_bound_scan_pair(v.fk, c, chi, k);
  // The bracketing piece, its prediction and window.
  uint64_t R[2] = {0, 0}, Rn[2] = {0, 0}, fkj[2] = {0, 0};
  PieceRec pc[2] = {};
  if (c[0] > 0) {
    const uint64_t j = c[0] - 1;
    R[0] = v.ps[j];
    Rn[0] = v.ps[j + 1];
    pc[0] = v.pr[j];
    fkj[0] = v.fk[j];
  }
  R[1] = R[0];
  Rn[1] = Rn[0];
  pc[1] = pc[0];
  fkj[1] = fkj[0];
  if (c[1] > 0 && c[1] != c[0]) {
    const uint64_t j = c[1] - 1;
    R[1] = v.ps[j];
    Rn[1] = v.ps[j + 1];
    pc[1] = v.pr[j];
    fkj[1] = v.fk[j];
  }
  uint64_t wlo[2], whi[2];
#pragma unroll
  for (int i = 0; i < 2; ++i) {
    wlo[i] = whi[i] = 0;
    if (c[i] > 0) {
      const int64_t p = piece_predict(pc[i].s, fkj[i], R[i], Rn[i], k[i]);
      int64_t a = p + pc[i].elo, b = p + pc[i].ehi;
      a = a < (int64_t)(R[i] + 1) ? (int64_t)(R[i] + 1) : a;
      b = b > (int64_t)Rn[i] ? (int64_t)Rn[i] : b;
      if (b < a) b = a;
      wlo[i] = (uint64_t)a;
      whi[i] = (uint64_t)b;
    }
  }
  lower_bound_scan_pair(keys, wlo, whi, k);
  uint32_t fb = 0;
  uint64_t below[2], at[2];
#pragma unroll
  for (int i = 0; i < 2; ++i) {
    r[i] = wlo[i] > n ? n : wlo[i];
    below[i] = r[i] > 0 ? keys[r[i] - 1] : 0;
    at[i] = r[i] < n ? keys[r[i]] : 0;
  }
#pragma unroll
  for (int i = 0; i < 2; ++i) {
    const bool ok = (r[i] == 0 || below[i] < k[i]) && (r[i] == n || at[i] >= k[i]);
    if (!ok) {
      r[i] = lower_bound_in(keys, 0, n, k[i]);
      ++fb;
    }
  }
  return fb;
}

}  // namespace sfc
