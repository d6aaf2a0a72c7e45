// Updates of a built index.  The paper's dynamic variant (Section 2,
// implementation details, "Dynamic implementation"; measured in the dynamic
// synthetic experiments of Section 3) keeps the (key, point) pairs in a
// B-tree multimap.  Here the sorted arrays stay flat:
//  * insertion sorts the new points into a run of their own (the
//    construction path) and merges it with the stored run: every element's
//    output position is its own index plus its rank in the other run, so the
//    merge is one pass of independent writes;
//  * erasure finds an id's stored position by a binary search on the
//    (key, id) order and stamps the entry with the erasing epoch (a
//    tombstone);
//  * compaction drops, in one stable stream compaction, the tombstones that
//    no queryable epoch can see.
// An entry is visible at epoch e when ins <= e < era (era = kLive while the
// entry is not erased).
#include <hip/hip_runtime.h>

#include "common.h"
#include "curve.h"
#include "internal.h"

namespace sfc {
namespace {

constexpr int kThreads = 256;
constexpr uint64_t kMergeTile = 2048;          // stored elements per merge block
constexpr uint64_t kCompactBlock = 4096;       // elements per compaction block
constexpr int kCompactRounds = (int)(kCompactBlock / kThreads);

// First j in [lo, hi) with b[j] >= k.
__device__ __forceinline__ uint64_t lower_bound_u64(const uint64_t* __restrict__ b, uint64_t lo,
                                                    uint64_t hi, uint64_t k) {
  uint64_t len = hi - lo;
  while (len > 0) {
    const uint64_t h = len >> 1;
    if (b[lo + h] < k) {
      lo += h + 1;
      len -= h + 1;
    } else {
      len = h;
    }
  }
  return lo;
}

// First j in [lo, hi) with b[j] > k.
__device__ __forceinline__ uint64_t upper_bound_u64(const uint64_t* __restrict__ b, uint64_t lo,
                                                    uint64_t hi, uint64_t k) {
  uint64_t len = hi - lo;
  while (len > 0) {
    const uint64_t h = len >> 1;
    if (b[lo + h] <= k) {
      lo += h + 1;
      len -= h + 1;
    } else {
      len = h;
    }
  }
  return lo;
}

// Stored element i goes to i + #{batch keys < key_i}: on equal keys the
// stored entries come first, and their ids are smaller than every new id,
// so the merged run stays sorted by (key, id).  The block's batch range is
// bracketed once from its first and last key.
__global__ __launch_bounds__(kThreads) void merge_stored(
    const uint64_t* __restrict__ keys, const uint32_t* __restrict__ ids,
    const double2* __restrict__ xy, const uint32_t* __restrict__ ins,
    const uint32_t* __restrict__ era, uint64_t n, const uint64_t* __restrict__ bkeys, uint64_t k,
    uint64_t* __restrict__ okeys, uint32_t* __restrict__ oids, double2* __restrict__ oxy,
    uint32_t* __restrict__ oins, uint32_t* __restrict__ oera, uint64_t* __restrict__ ocells) {
  __shared__ uint64_t s_br[2];
  const uint64_t t0 = (uint64_t)blockIdx.x * kMergeTile;
  const uint64_t t1 = t0 + kMergeTile < n ? t0 + kMergeTile : n;
  if (threadIdx.x == 0) s_br[0] = lower_bound_u64(bkeys, 0, k, keys[t0]);
  if (threadIdx.x == 64) s_br[1] = lower_bound_u64(bkeys, 0, k, keys[t1 - 1]);
  __syncthreads();
  const uint64_t b0 = s_br[0], b1 = s_br[1];
  for (uint64_t i = t0 + threadIdx.x; i < t1; i += kThreads) {
    const uint64_t key = keys[i];
    const uint64_t o = i + lower_bound_u64(bkeys, b0, b1, key);
    const double2 p = xy[i];
    okeys[o] = key;
    oids[o] = ids[i];
    oxy[o] = p;
    oins[o] = ins[i];
    oera[o] = era[i];
    if (ocells) ocells[o] = pack_cell2(p.x, p.y);
  }
}

// Batch element j (sorted, local id bids[j]) goes to j + #{stored keys <=
// its key}; it gets the id id_base + bids[j], the insert epoch `epoch` (with
// run offsets: epoch + the index of the run holding its local id, runs
// inserted one after another), and its key is recorded under its id for
// later erasure.
__global__ __launch_bounds__(kThreads) void merge_batch(
    const uint64_t* __restrict__ keys, uint64_t n, const uint64_t* __restrict__ bkeys,
    const uint32_t* __restrict__ bids, const double2* __restrict__ bxy, uint64_t k,
    uint32_t id_base, uint32_t epoch, const uint64_t* __restrict__ run_off, uint32_t runs,
    uint64_t* __restrict__ okeys, uint32_t* __restrict__ oids,
    double2* __restrict__ oxy, uint32_t* __restrict__ oins, uint32_t* __restrict__ oera,
    uint64_t* __restrict__ ocells, uint64_t* __restrict__ key_of) {
  const uint64_t j = (uint64_t)blockIdx.x * kThreads + threadIdx.x;
  if (j >= k) return;
  const uint32_t lid = bids[j];
  if (lid >= k) return;   // only after a failed sort, whose result is discarded
  const uint64_t key = bkeys[j];
  const uint64_t o = j + upper_bound_u64(keys, 0, n, key);
  const uint32_t id = id_base + lid;
  const double2 p = bxy[j];
  uint32_t ep = epoch;
  if (run_off) {   // last run r with run_off[r] <= lid
    uint32_t lo = 0, len = runs;
    while (len > 0) {
      const uint32_t h = len >> 1;
      if (run_off[lo + h] <= lid) {
        lo += h + 1;
        len -= h + 1;
      } else {
        len = h;
      }
    }
    ep = epoch + (lo - 1);
  }
  okeys[o] = key;
  oids[o] = id;
  oxy[o] = p;
  oins[o] = ep;
  oera[o] = kLiveEpoch;
  if (ocells) ocells[o] = pack_cell2(p.x, p.y);
  key_of[id] = key;
}

// key_of[ids[i]] = keys[i] for the stored run (once, before the first
// update of an index built in one piece).
__global__ __launch_bounds__(kThreads) void scatter_key_of(const uint64_t* __restrict__ keys,
                                                           const uint32_t* __restrict__ ids,
                                                           uint64_t n,
                                                           uint64_t* __restrict__ key_of) {
  const uint64_t stride = (uint64_t)gridDim.x * kThreads;
  for (uint64_t i = (uint64_t)blockIdx.x * kThreads + threadIdx.x; i < n; i += stride)
    key_of[ids[i]] = keys[i];
}

// Tombstones: for each listed id below next_id, the stored position of
// (key_of[id], id) by binary search on the (key, id) order; a live entry
// found there gets era = epoch.  Unknown, dropped and already erased ids
// change nothing; a compare-and-swap makes duplicates in one list count once.
__global__ __launch_bounds__(kThreads) void erase_ids(
    const uint32_t* __restrict__ del, uint64_t k, uint32_t next_id,
    const uint64_t* __restrict__ key_of, const uint64_t* __restrict__ keys,
    const uint32_t* __restrict__ ids, uint64_t n, uint32_t* era, uint32_t epoch,
    unsigned long long* erased) {
  const uint64_t j = (uint64_t)blockIdx.x * kThreads + threadIdx.x;
  bool done = false;
  if (j < k) {
    const uint32_t id = del[j];
    if (id < next_id) {
      const uint64_t key = key_of[id];
      uint64_t lo = 0, len = n;
      while (len > 0) {
        const uint64_t h = len >> 1;
        const uint64_t mk = keys[lo + h];
        if (mk < key || (mk == key && ids[lo + h] < id)) {
          lo += h + 1;
          len -= h + 1;
        } else {
          len = h;
        }
      }
      if (lo < n && keys[lo] == key && ids[lo] == id)
        done = atomicCAS(era + lo, kLiveEpoch, epoch) == kLiveEpoch;
    }
  }
  const uint64_t b = __ballot(done);
  if (__lane_id() == 0 && b) atomicAdd(erased, (unsigned long long)__popcll(b));
}

// Compaction, pass 1: entries kept (era > oldest) per block.
__global__ __launch_bounds__(kThreads) void compact_count(const uint32_t* __restrict__ era,
                                                          uint64_t n, uint32_t oldest,
                                                          uint32_t* __restrict__ block_kept) {
  __shared__ uint32_t s_w[kThreads / 64];
  const uint64_t base = (uint64_t)blockIdx.x * kCompactBlock;
  uint32_t c = 0;
  for (int r = 0; r < kCompactRounds; ++r) {
    const uint64_t i = base + (uint64_t)r * kThreads + threadIdx.x;
    c += (i < n && era[i] > oldest) ? 1u : 0u;
  }
  for (int o = 32; o > 0; o >>= 1) c += __shfl_xor(c, o, 64);
  if (__lane_id() == 0) s_w[threadIdx.x >> 6] = c;
  __syncthreads();
  if (threadIdx.x == 0) block_kept[blockIdx.x] = s_w[0] + s_w[1] + s_w[2] + s_w[3];
}

// Compaction, pass 2: kept entries written in order at the block's offset.
__global__ __launch_bounds__(kThreads) void compact_scatter(
    const uint64_t* __restrict__ keys, const uint32_t* __restrict__ ids,
    const double2* __restrict__ xy, const uint32_t* __restrict__ ins,
    const uint32_t* __restrict__ era, uint64_t n, uint32_t oldest,
    const uint64_t* __restrict__ block_off, uint64_t* __restrict__ okeys,
    uint32_t* __restrict__ oids, double2* __restrict__ oxy, uint32_t* __restrict__ oins,
    uint32_t* __restrict__ oera, const uint64_t* __restrict__ cells,
    uint64_t* __restrict__ ocells) {
  __shared__ uint32_t s_w[kThreads / 64];
  const uint32_t w = threadIdx.x >> 6;
  const uint64_t base = (uint64_t)blockIdx.x * kCompactBlock;
  uint64_t out = block_off[blockIdx.x];
  const uint64_t below = lanemask_lt();
  for (int r = 0; r < kCompactRounds; ++r) {
    const uint64_t i = base + (uint64_t)r * kThreads + threadIdx.x;
    const bool keep = i < n && era[i] > oldest;
    const uint64_t b = __ballot(keep);
    if (__lane_id() == 0) s_w[w] = (uint32_t)__popcll(b);
    __syncthreads();
    uint32_t before = 0, total = 0;
    for (uint32_t v = 0; v < kThreads / 64; ++v) {
      before += v < w ? s_w[v] : 0u;
      total += s_w[v];
    }
    if (keep) {
      const uint64_t o = out + before + (uint64_t)__popcll(b & below);
      okeys[o] = keys[i];
      oids[o] = ids[i];
      oxy[o] = xy[i];
      oins[o] = ins[i];
      oera[o] = era[i];
      if (ocells) ocells[o] = cells[i];
    }
    out += total;
    __syncthreads();
  }
}

__global__ __launch_bounds__(kThreads) void iota_u32(uint32_t* __restrict__ out, uint64_t k,
                                                     uint32_t first) {
  const uint64_t j = (uint64_t)blockIdx.x * kThreads + threadIdx.x;
  if (j < k) out[j] = first + (uint32_t)j;
}

__global__ __launch_bounds__(kThreads) void check_epochs(const uint32_t* __restrict__ qe,
                                                         uint64_t m, uint32_t oldest,
                                                         uint32_t epoch, uint32_t* err) {
  const uint64_t j = (uint64_t)blockIdx.x * kThreads + threadIdx.x;
  const bool bad = j < m && (qe[j] < oldest || qe[j] > epoch);
  if (__ballot(bad) && __lane_id() == 0) atomicOr(err, kErrInvalidQuery);
}

uint32_t grid_for(uint64_t count, uint64_t per_block) {
  return (uint32_t)((count + per_block - 1) / per_block);
}

}  // namespace

hipError_t merge_runs(const Run& stored, uint64_t n, const uint64_t* bkeys, const uint32_t* bids,
                      const double* bxy, uint64_t k, uint32_t id_base, uint32_t epoch,
                      const Run& out, uint64_t* key_of, hipStream_t s, const uint64_t* run_off,
                      uint32_t runs) {
  if (n > 0) {
    ProfScope ps("merge_stored", s);
    merge_stored<<<grid_for(n, kMergeTile), kThreads, 0, s>>>(
        stored.keys, stored.ids, (const double2*)stored.xy, stored.ins, stored.era, n, bkeys, k,
        out.keys, out.ids, (double2*)out.xy, out.ins, out.era, out.cells);
    hipError_t e = hipGetLastError();
    if (e != hipSuccess) return e;
  }
  if (k > 0) {
    ProfScope ps("merge_batch", s);
    merge_batch<<<grid_for(k, kThreads), kThreads, 0, s>>>(
        stored.keys, n, bkeys, bids, (const double2*)bxy, k, id_base, epoch, run_off, runs,
        out.keys, out.ids, (double2*)out.xy, out.ins, out.era, out.cells, key_of);
    return hipGetLastError();
  }
  return hipSuccess;
}

hipError_t record_keys(const uint64_t* keys, const uint32_t* ids, uint64_t n, uint64_t* key_of,
                       hipStream_t s) {
  if (n == 0) return hipSuccess;
  uint32_t g = grid_for(n, kThreads);
  if (g > 4096) g = 4096;
  scatter_key_of<<<g, kThreads, 0, s>>>(keys, ids, n, key_of);
  return hipGetLastError();
}

hipError_t erase_entries(const uint32_t* del, uint64_t k, uint32_t next_id, const uint64_t* key_of,
                         const Run& stored, uint64_t n, uint32_t epoch,
                         unsigned long long* erased, hipStream_t s) {
  if (k == 0) return hipSuccess;
  ProfScope ps("erase_ids", s);
  erase_ids<<<grid_for(k, kThreads), kThreads, 0, s>>>(del, k, next_id, key_of, stored.keys,
                                                       stored.ids, n, stored.era, epoch, erased);
  return hipGetLastError();
}

size_t compact_entries_scratch(uint64_t n) {
  const uint64_t nb = (n + kCompactBlock - 1) / kCompactBlock;
  return align256(nb * 4 + 4) + align256((nb + 1) * 8) + scan_scratch_bytes(nb);
}

hipError_t compact_entries(const Run& stored, uint64_t n, uint32_t oldest, const Run& out,
                           void* scratch, uint64_t** kept_total, hipStream_t s) {
  const uint64_t nb = (n + kCompactBlock - 1) / kCompactBlock;
  char* p = (char*)scratch;
  uint32_t* kept = (uint32_t*)p;   p += align256(nb * 4 + 4);
  uint64_t* off = (uint64_t*)p;    p += align256((nb + 1) * 8);
  uint64_t* tmp = (uint64_t*)p;
  *kept_total = off + nb;
  hipError_t e;
  if (nb == 0) return fill_u64(off, 0, 1, s);
  ProfScope ps("compact_entries", s);
  compact_count<<<(uint32_t)nb, kThreads, 0, s>>>(stored.era, n, oldest, kept);
  if ((e = hipGetLastError()) != hipSuccess) return e;
  if ((e = scan_excl(kept, off, nb, nullptr, tmp, s)) != hipSuccess) return e;
  compact_scatter<<<(uint32_t)nb, kThreads, 0, s>>>(
      stored.keys, stored.ids, (const double2*)stored.xy, stored.ins, stored.era, n, oldest, off,
      out.keys, out.ids, (double2*)out.xy, out.ins, out.era, stored.cells, out.cells);
  return hipGetLastError();
}

hipError_t fill_iota(uint32_t* out, uint64_t k, uint32_t first, hipStream_t s) {
  if (k == 0) return hipSuccess;
  iota_u32<<<grid_for(k, kThreads), kThreads, 0, s>>>(out, k, first);
  return hipGetLastError();
}

hipError_t validate_epochs(const uint32_t* qe, uint64_t m, uint32_t oldest, uint32_t epoch,
                           uint32_t* err, hipStream_t s) {
  if (m == 0) return hipSuccess;
  check_epochs<<<grid_for(m, kThreads), kThreads, 0, s>>>(qe, m, oldest, epoch, err);
  return hipGetLastError();
}

}  // namespace sfc
