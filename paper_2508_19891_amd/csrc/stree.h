// Static search tree over the sorted keys (Sec. 2.1 "Storing P twice": the
// keys are searched through a static B-tree whose lowest layer is the sorted
// key array itself).  Our layout: layer 0 is the key array; layer k+1 holds
// the first key of every block of kStreeFan consecutive entries of layer k
// (a 128-byte line), so layer k+1[b] = keys[b * kStreeFan^(k+1)].  A layer of
// at most kStreeFan entries is the top.
//
// Counting the entries of layer 0 below x: let c be the number of entries of
// layer k+1 below x, i.e. of blocks of layer k whose first entry is below x.
// All entries of the blocks before block c-1 are then below x too, and none
// after it, so the count in layer k is kStreeFan * (c - 1) plus the count
// inside block c-1 (and 0 when c = 0).  One line per layer, top down.  The
// same holds with "at most x" for the upper end of a key interval, so a key
// interval [lo, hi] maps to the index range [#(< lo), #(<= hi)), equal to
// std::lower_bound / std::upper_bound over the keys.
#pragma once

#include <hip/hip_runtime.h>

#include <cstdint>

namespace sfc {

constexpr int kStreeFan = 16;          // entries per block: one 128-byte line of u64 keys
constexpr int kStreeMaxLayers = 9;     // 2^32 keys: layers of 2^32, 2^28, ..., 16

// Device view: layer[0] is the key array (16-byte aligned), layers 1..top
// live in one buffer, each 256-byte aligned.
struct StreeView {
  const uint64_t* layer[kStreeMaxLayers];
  uint64_t size[kStreeMaxLayers];
  int top;
};

// Entries of block [base, base + kStreeFan) of a layer of `size` entries
// that are below x (LE: at most x).
template <bool LE>
__device__ __forceinline__ uint32_t stree_block_count(const uint64_t* __restrict__ layer,
                                                      uint64_t size, uint64_t base, uint64_t x) {
  uint32_t c = 0;
  if (base + kStreeFan <= size) {
    const ulonglong2* p = (const ulonglong2*)(layer + base);
    ulonglong2 w[kStreeFan / 2];
#pragma unroll
    for (int t = 0; t < kStreeFan / 2; ++t) w[t] = p[t];
#pragma unroll
    for (int t = 0; t < kStreeFan / 2; ++t)
      c += LE ? (uint32_t)(w[t].x <= x) + (uint32_t)(w[t].y <= x)
              : (uint32_t)(w[t].x < x) + (uint32_t)(w[t].y < x);
  } else {
    for (uint64_t t = base; t < size; ++t) c += LE ? layer[t] <= x : layer[t] < x;
  }
  return c;
}

// The index range [b, e) of the key interval [lo, hi]: both descents run
// level by level together, so their line loads overlap.
__device__ __forceinline__ void stree_range(const StreeView& v, uint64_t lo, uint64_t hi,
                                            uint64_t& b, uint64_t& e) {
  const int top = v.top;
  uint64_t cb = stree_block_count<false>(v.layer[top], v.size[top], 0, lo);
  uint64_t ce = stree_block_count<true>(v.layer[top], v.size[top], 0, hi);
  for (int k = top - 1; k >= 0; --k) {
    const uint64_t* L = v.layer[k];
    const uint64_t sz = v.size[k];
    if (cb > 0) {
      const uint64_t base = (cb - 1) * kStreeFan;
      cb = base + stree_block_count<false>(L, sz, base, lo);
    }
    if (ce > 0) {
      const uint64_t base = (ce - 1) * kStreeFan;
      ce = base + stree_block_count<true>(L, sz, base, hi);
    }
  }
  b = cb;
  e = ce;
}

// Host: bytes of layers 1..top for n keys, and the view over keys and buf.
size_t stree_bytes(uint64_t n);
StreeView stree_view(const uint64_t* keys, uint64_t n, void* buf);
// Writes layers 1..top of v from its layer 0.
hipError_t stree_build(const StreeView& v, hipStream_t s);

}  // namespace sfc
