// Device-wide exclusive scan of uint32 counts into uint64 offsets, in three
// launches (block sums, scan of the block sums, block scans).  No block waits
// on another, so no launch depends on forward-progress assumptions.
#include <hip/hip_runtime.h>

#include "common.h"
#include "internal.h"

namespace sfc {
namespace {

constexpr int kScanThreads = 256;
constexpr int kScanItems = 16;
constexpr uint64_t kScanBlock = (uint64_t)kScanThreads * kScanItems;   // 4096

// Sum of the kScanItems consecutive inputs owned by this thread.
__device__ __forceinline__ uint32_t load_items(const uint32_t* __restrict__ in, uint64_t count,
                                               uint64_t first, uint32_t v[kScanItems]) {
  uint32_t s = 0;
  if (first + kScanItems <= count) {
    const uint4* p = (const uint4*)(in + first);
#pragma unroll
    for (int i = 0; i < kScanItems / 4; ++i) {
      const uint4 x = p[i];
      v[4 * i] = x.x;
      v[4 * i + 1] = x.y;
      v[4 * i + 2] = x.z;
      v[4 * i + 3] = x.w;
    }
  } else {
#pragma unroll
    for (int i = 0; i < kScanItems; ++i) v[i] = first + i < count ? in[first + i] : 0u;
  }
#pragma unroll
  for (int i = 0; i < kScanItems; ++i) s += v[i];
  return s;
}

__device__ __forceinline__ uint64_t block_scan_u64(uint64_t v, uint64_t* s_tmp, uint64_t* total) {
  const uint32_t lane = threadIdx.x & 63, w = threadIdx.x >> 6;
  const uint32_t nw = blockDim.x >> 6;
  uint64_t x = v;
#pragma unroll
  for (int o = 1; o < 64; o <<= 1) {
    const uint64_t y = __shfl_up(x, o, 64);
    if (lane >= (uint32_t)o) x += y;
  }
  if (lane == 63) s_tmp[w] = x;
  __syncthreads();
  uint64_t add = 0, tot = 0;
  for (uint32_t i = 0; i < nw; ++i) {
    if (i < w) add += s_tmp[i];
    tot += s_tmp[i];
  }
  __syncthreads();
  *total = tot;
  return x - v + add;
}

__global__ __launch_bounds__(kScanThreads) void scan_block_sums(const uint32_t* __restrict__ in,
                                                                uint64_t count,
                                                                uint64_t* __restrict__ partial) {
  __shared__ uint64_t s_tmp[kScanThreads / 64];
  uint32_t v[kScanItems];
  const uint64_t first = (uint64_t)blockIdx.x * kScanBlock + (uint64_t)threadIdx.x * kScanItems;
  const uint64_t s = load_items(in, count, first, v);
  uint64_t tot;
  block_scan_u64(s, s_tmp, &tot);
  if (threadIdx.x == 0) partial[blockIdx.x] = tot;
}

// One block of 1024 threads: exclusive scan of nb block sums (in place), plus
// the carry-in; partial[nb] receives the grand total.
__global__ __launch_bounds__(1024) void scan_partials(uint64_t* partial, uint64_t nb,
                                                      const uint64_t* carry_in) {
  __shared__ uint64_t s_tmp[16];
  __shared__ uint64_t s_carry;
  if (threadIdx.x == 0) s_carry = carry_in ? carry_in[0] : 0;
  __syncthreads();
  for (uint64_t base = 0; base < nb; base += 1024) {
    const uint64_t i = base + threadIdx.x;
    const uint64_t v = i < nb ? partial[i] : 0;
    uint64_t tot;
    const uint64_t ex = block_scan_u64(v, s_tmp, &tot);
    const uint64_t c = s_carry;
    if (i < nb) partial[i] = c + ex;
    __syncthreads();
    if (threadIdx.x == 0) s_carry = c + tot;
    __syncthreads();
  }
  if (threadIdx.x == 0) partial[nb] = s_carry;
}

__global__ __launch_bounds__(kScanThreads) void scan_blocks(const uint32_t* __restrict__ in,
                                                            uint64_t count,
                                                            const uint64_t* __restrict__ partial,
                                                            uint64_t* __restrict__ out) {
  __shared__ uint64_t s_tmp[kScanThreads / 64];
  uint32_t v[kScanItems];
  const uint64_t first = (uint64_t)blockIdx.x * kScanBlock + (uint64_t)threadIdx.x * kScanItems;
  const uint64_t s = load_items(in, count, first, v);
  uint64_t tot;
  uint64_t run = partial[blockIdx.x] + block_scan_u64(s, s_tmp, &tot);
#pragma unroll
  for (int i = 0; i < kScanItems; ++i) {
    if (first + i < count) out[first + i] = run;
    run += v[i];
  }
  if (blockIdx.x == gridDim.x - 1 && threadIdx.x == 0) out[count] = partial[gridDim.x];
}

// Device-sized variant: the element count is read from device memory, and a
// fixed number of blocks (chosen from an upper bound of the count) each scan
// one contiguous chunk in steps of kScanBlock elements.
__device__ __forceinline__ void dev_chunk(uint64_t count, uint64_t* first, uint64_t* last) {
  const uint64_t per = ((count + gridDim.x - 1) / gridDim.x + kScanItems - 1) / kScanItems *
                       kScanItems;
  *first = (uint64_t)blockIdx.x * per;
  *last = *first + per < count ? *first + per : count;
  if (*first > count) *first = count;
}

__global__ __launch_bounds__(kScanThreads) void scan_dev_sums(const uint32_t* __restrict__ in,
                                                              const uint32_t* __restrict__ count_dev,
                                                              uint64_t* __restrict__ partial) {
  __shared__ uint64_t s_tmp[kScanThreads / 64];
  const uint64_t count = *count_dev;
  uint64_t first, last;
  dev_chunk(count, &first, &last);
  uint64_t acc = 0;
  for (uint64_t b = first; b < last; b += kScanBlock) {
    uint32_t v[kScanItems];
    const uint64_t f = b + (uint64_t)threadIdx.x * kScanItems;
    uint64_t tot;
    block_scan_u64(f < last ? load_items(in, last, f, v) : 0u, s_tmp, &tot);
    acc += tot;
  }
  if (threadIdx.x == 0) partial[blockIdx.x] = acc;
}

__global__ __launch_bounds__(kScanThreads) void scan_dev_blocks(const uint32_t* __restrict__ in,
                                                                const uint32_t* __restrict__ count_dev,
                                                                const uint64_t* __restrict__ partial,
                                                                uint64_t* __restrict__ out) {
  __shared__ uint64_t s_tmp[kScanThreads / 64];
  const uint64_t count = *count_dev;
  uint64_t first, last;
  dev_chunk(count, &first, &last);
  uint64_t carry = partial[blockIdx.x];
  for (uint64_t b = first; b < last; b += kScanBlock) {
    uint32_t v[kScanItems];
    const uint64_t f = b + (uint64_t)threadIdx.x * kScanItems;
    const uint64_t s = f < last ? load_items(in, last, f, v) : 0u;
    if (f >= last) {
#pragma unroll
      for (int i = 0; i < kScanItems; ++i) v[i] = 0;
    }
    uint64_t tot;
    uint64_t run = carry + block_scan_u64(s, s_tmp, &tot);
#pragma unroll
    for (int i = 0; i < kScanItems; ++i) {
      if (f + i < last) out[f + i] = run;
      run += v[i];
    }
    carry += tot;
  }
  if (blockIdx.x == gridDim.x - 1 && threadIdx.x == 0) out[count] = partial[gridDim.x];
}

}  // namespace

uint32_t scan_dev_blocks_for(uint64_t max_count) {
  uint64_t nb = (max_count + kScanBlock - 1) / kScanBlock;
  if (nb > 1024) nb = 1024;
  return nb < 1 ? 1u : (uint32_t)nb;
}

hipError_t scan_excl_dev(const uint32_t* in, uint64_t* out, const uint32_t* count_dev,
                         uint64_t max_count, const uint64_t* carry_in, uint64_t* partial,
                         hipStream_t s) {
  const uint32_t nb = scan_dev_blocks_for(max_count);
  ProfScope ps("scan", s);
  scan_dev_sums<<<nb, kScanThreads, 0, s>>>(in, count_dev, partial);
  scan_partials<<<1, 1024, 0, s>>>(partial, nb, carry_in);
  scan_dev_blocks<<<nb, kScanThreads, 0, s>>>(in, count_dev, partial, out);
  return hipGetLastError();
}

size_t scan_scratch_bytes(uint64_t count) {
  return align256(((count + kScanBlock - 1) / kScanBlock + 1) * 8);
}

hipError_t scan_excl(const uint32_t* in, uint64_t* out, uint64_t count, const uint64_t* carry_in,
                     uint64_t* partial, hipStream_t s) {
  if (count == 0) {
    // out[0] = carry (or 0): one block scanning zero partials writes it.
    scan_partials<<<1, 1024, 0, s>>>(out, 0, carry_in);
    return hipGetLastError();
  }
  const uint64_t nb = (count + kScanBlock - 1) / kScanBlock;
  ProfScope ps("scan", s);
  scan_block_sums<<<(uint32_t)nb, kScanThreads, 0, s>>>(in, count, partial);
  scan_partials<<<1, 1024, 0, s>>>(partial, nb, carry_in);
  scan_blocks<<<(uint32_t)nb, kScanThreads, 0, s>>>(in, count, partial, out);
  return hipGetLastError();
}

}  // namespace sfc
