// Shared host/device helpers of libsfc (gfx950, wave64).
#pragma once

#include <hip/hip_runtime.h>

#include <atomic>
#include <cstddef>
#include <cstdint>

#include "sfc.h"

namespace sfc {

constexpr int kWave = 64;

// Error flag bits written by kernels into a device word.
constexpr uint32_t kErrDomain = 1u;
constexpr uint32_t kErrInvalidQuery = 2u;
constexpr uint32_t kErrLookback = 4u;   // reserved (no kernel waits on another)
constexpr uint32_t kErrInternal = 8u;   // an index outside its array (never expected)
constexpr uint32_t kErrOverflow = 16u;  // more candidate rows than a fixed plan holds
constexpr uint32_t kErrOversized = 32u; // a run of equal top key bits too long for the chunked sort

__device__ __forceinline__ uint32_t lane_id() { return __lane_id(); }

// Mask of the lanes below this one.
__device__ __forceinline__ uint64_t lanemask_lt() {
  uint32_t l = lane_id();
  return l == 0 ? 0ull : (~0ull >> (64 - l));
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
