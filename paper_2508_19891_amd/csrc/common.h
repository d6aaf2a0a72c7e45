// Shared host/device helpers of libsfc (gfx950, wave64).
#pragma once

#include <hip/hip_runtime.h>

#include <atomic>
#include <cstddef>
#include <cstdint>

#include "sfc.h"

namespace sfc {

constexpr int kWave = 64;

// Status words of the single-pass (decoupled look-back) scans: the two top
// bits hold the state, the low 62 bits the value.
constexpr uint64_t kFlagAggregate = 1ull << 62;
constexpr uint64_t kFlagInclusive = 2ull << 62;
constexpr uint64_t kValueMask = (1ull << 62) - 1;
// Upper bound on the polls of one look-back step.  A predecessor that has
// started always publishes within a few microseconds; the bound only makes
// every wave terminate if an invariant is ever broken (the kernel then raises
// the error flag instead of hanging).
constexpr uint32_t kSpinLimit = 1u << 22;

// Error flag bits written by kernels into a device word.
constexpr uint32_t kErrDomain = 1u;
constexpr uint32_t kErrInvalidQuery = 2u;
constexpr uint32_t kErrLookback = 4u;
constexpr uint32_t kErrInternal = 8u;   // an index outside its array (never expected)
constexpr uint32_t kErrOverflow = 16u;  // more candidate rows than a fixed plan holds

__device__ __forceinline__ uint64_t ld_acquire_agent(const uint64_t* p) {
  return __hip_atomic_load(p, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
}
__device__ __forceinline__ void st_release_agent(uint64_t* p, uint64_t v) {
  __hip_atomic_store(p, v, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
}

__device__ __forceinline__ uint32_t lane_id() { return __lane_id(); }

// Mask of the lanes below this one.
__device__ __forceinline__ uint64_t lanemask_lt() {
  uint32_t l = lane_id();
  return l == 0 ? 0ull : (~0ull >> (64 - l));
}

// Decoupled look-back: sum of the values of all tiles before `tile` in a
// status array of (flag | value) words, then publish this tile's inclusive
// value.  Called by one lane per (tile, column).
__device__ __forceinline__ uint64_t lookback_publish(uint64_t* status, uint64_t tile,
                                                     uint64_t stride, uint64_t col,
                                                     uint64_t aggregate,
                                                     uint32_t* err) {
  uint64_t excl = 0;
  if (tile > 0) {
    int64_t t = (int64_t)tile - 1;
    uint32_t spins = 0;
    while (t >= 0) {
      uint64_t v = ld_acquire_agent(status + (uint64_t)t * stride + col);
      uint64_t flag = v & ~kValueMask;
      if (flag == 0) {
        if (++spins > kSpinLimit) {
          atomicOr(err, kErrLookback);
          break;
        }
        __builtin_amdgcn_s_sleep(1);
        continue;
      }
      excl += v & kValueMask;
      if (flag == kFlagInclusive) break;
      --t;
    }
  }
  st_release_agent(status + tile * stride + col, kFlagInclusive | (excl + aggregate));
  return excl;
}

}  // namespace sfc

// ---- host-side plumbing ------------------------------------------------------

namespace sfc {

struct Allocator {
  void* (*alloc)(size_t, void*) = nullptr;
  void (*release)(void*, void*) = nullptr;
  void* ctx = nullptr;
  void* get(size_t bytes) const;
  void put(void* p) const;
};

// Kernel launch bracketing for sfc_profile_*.
struct ProfScope {
  const char* name;
  hipStream_t stream;
  void* ev0 = nullptr;
  ProfScope(const char* name, hipStream_t s);
  ~ProfScope();
};

// Nonzero while a stream capture is in progress (no timing events then).
extern std::atomic<int> g_capturing;

// Pinned host scratch for small device-to-host reads.
uint64_t* pinned_scratch();

}  // namespace sfc
