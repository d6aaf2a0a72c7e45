// Construction (Sec. 2.1 "Storing P twice"; Alg. 2; Def. 3): curve keys,
// an LSD radix sort of (key, id) and the gather of the points into key order.
//
// Kernels, in launch order for n points (one workgroup per tile of 2048 to
// 4096 points):
//   keygen_tiles   quantise, key, write keys; the tile's counts of the first
//                  digit (LDS histograms per wave).
//   then per 8-bit digit (eight passes, plus one or two passes over the set
//   index for point sets):
//   tile_hist      the tile's digit counts (from the second pass on);
//   digit_scan     one workgroup per digit: exclusive scan of the digit's
//                  counts over the tiles, and the digit's total;
//   scatter_pass   rank the tile in LDS with wave64 ballots and scatter it
//                  through LDS so that writes go out digit-contiguous, at
//                  base(digit) + scan(digit, tile).  The first pass takes ids
//                  from the position (iota); the last pass also gathers the
//                  points into key order.
// No workgroup waits on another.  Tiles are assigned so that each XCD (the
// hardware deals workgroups to the eight XCDs in turn) scatters a contiguous
// range of tiles: the runs that consecutive tiles write for one digit are
// adjacent in the output, and they then meet in the same L2, which writes
// back whole lines.  (A single-pass scheme with a decoupled look-back between
// tiles, measured first, spent much of each pass polling status words across
// the XCDs, and its dynamic tile order cannot be made XCD-contiguous.)
#include <hip/hip_runtime.h>

#include <cstdlib>

#include "common.h"
#include "curve.h"
#include "internal.h"

namespace sfc {

namespace {

constexpr int kRadix = 256;
constexpr int kDigits = 8;
constexpr int kSortWaves = 4;
constexpr int kSortThreads = kSortWaves * kWave;

// True when a kernel of a guarded sequence has nothing to do (SortGuard).
// The word is read by every thread before any barrier: the whole workgroup
// returns or none of it.
__device__ __forceinline__ bool guard_skips(SortGuard g) {
  return g.word && (((*g.word & kErrOversized) != 0u) != g.when_set);
}

// Exclusive scan of one uint32 per thread over a block of 256 threads.
__device__ __forceinline__ uint32_t block_excl_scan256(uint32_t v, uint32_t* s_tmp) {
  const uint32_t lane = threadIdx.x & 63, w = threadIdx.x >> 6;
  uint32_t x = v;
#pragma unroll
  for (int o = 1; o < 64; o <<= 1) {
    uint32_t y = __shfl_up(x, o, 64);
    if (lane >= (uint32_t)o) x += y;
  }
  if (lane == 63) s_tmp[w] = x;
  __syncthreads();
  uint32_t add = 0;
  for (uint32_t i = 0; i < w; ++i) add += s_tmp[i];
  __syncthreads();
  return x - v + add;
}

// Per-wave LDS digit counts of a block, summed and stored digit-major:
// counts[d * tiles + tile].
__device__ __forceinline__ void store_tile_counts(uint32_t (*h)[kRadix], uint32_t* counts,
                                                  uint64_t tiles, uint64_t tile) {
  __syncthreads();
  const uint32_t d = threadIdx.x;
  counts[(uint64_t)d * tiles + tile] = h[0][d] + h[1][d] + h[2][d] + h[3][d];
}

// One workgroup per sort tile of tile_len input points: quantise, key, write
// keys; with counts != null also the tile's counts of the first digit (the
// byte at count_shift).
template <int CURVE>
__global__ __launch_bounds__(256) void keygen_tiles(const double2* __restrict__ xy, uint64_t n,
                                                   uint32_t tile_len, uint64_t* __restrict__ keys,
                                                   uint32_t* __restrict__ err,
                                                   uint32_t* __restrict__ counts, uint64_t tiles,
                                                   double2* __restrict__ xy_copy, int count_shift,
                                                   SortGuard guard) {
  if (guard_skips(guard)) return;
  __shared__ uint32_t h[kSortWaves][kRadix];
  __shared__ uint16_t lut[CURVE == SFC_CURVE_HILBERT ? 1024 : 1];
  for (int i = threadIdx.x; i < kSortWaves * kRadix; i += 256) (&h[0][0])[i] = 0;
  if (CURVE == SFC_CURVE_HILBERT)
    for (int i = threadIdx.x; i < 1024; i += 256) lut[i] = kHilbertLutConst.v[i];
  __syncthreads();
  const uint64_t base = (uint64_t)blockIdx.x * tile_len;
  const uint64_t end = base + tile_len < n ? base + tile_len : n;
  const uint32_t w = threadIdx.x >> 6;
  bool bad = false;
  // Eight points in flight per thread: positions past the tile load its last
  // point (no branch around the loads) and are then skipped.
  constexpr int kBatch = 8;
  for (uint64_t i0 = base + threadIdx.x; i0 < end; i0 += 256 * kBatch) {
    double2 pb[kBatch];
#pragma unroll
    for (int j = 0; j < kBatch; ++j) {
      const uint64_t i = i0 + 256u * j;
      pb[j] = xy[i < end ? i : end - 1];
    }
#pragma unroll
    for (int j = 0; j < kBatch; ++j) {
      const uint64_t i = i0 + 256u * j;
      if (i >= end) continue;
      const double2 p = pb[j];
      if (xy_copy) xy_copy[i] = p;
      uint64_t key = 0;
      if (in_unit(p.x) && in_unit(p.y)) {
        const uint32_t ux = quantize(p.x), uy = quantize(p.y);
        key = CURVE == SFC_CURVE_HILBERT ? hilbert_key_lut(lut, ux, uy) : morton_key(ux, uy);
      } else {
        bad = true;
      }
      keys[i] = key;
      if (counts) atomicAdd(&h[w][(key >> count_shift) & 255u], 1u);
    }
  }
  if (__ballot(bad) != 0 && lane_id() == 0) atomicOr(err, kErrDomain);
  if (counts) store_tile_counts(h, counts, tiles, blockIdx.x);
}

// keygen_tiles for points in [0,1)^3 (three doubles each) and the d = 3
// Morton code.
__global__ __launch_bounds__(256) void keygen3_tiles(const double* __restrict__ xyz, uint64_t n,
                                                    uint32_t tile_len, uint64_t* __restrict__ keys,
                                                    uint32_t* __restrict__ err,
                                                    uint32_t* __restrict__ counts, uint64_t tiles,
                                                    double* __restrict__ xyz_copy, int count_shift,
                                                    SortGuard guard) {
  if (guard_skips(guard)) return;
  __shared__ uint32_t h[kSortWaves][kRadix];
  for (int i = threadIdx.x; i < kSortWaves * kRadix; i += 256) (&h[0][0])[i] = 0;
  __syncthreads();
  const uint64_t base = (uint64_t)blockIdx.x * tile_len;
  const uint64_t end = base + tile_len < n ? base + tile_len : n;
  const uint32_t w = threadIdx.x >> 6;
  bool bad = false;
  for (uint64_t i = base + threadIdx.x; i < end; i += 256) {
    const double x = xyz[3 * i], y = xyz[3 * i + 1], z = xyz[3 * i + 2];
    if (xyz_copy) {
      xyz_copy[3 * i] = x;
      xyz_copy[3 * i + 1] = y;
      xyz_copy[3 * i + 2] = z;
    }
    uint64_t key = 0;
    if (in_unit(x) && in_unit(y) && in_unit(z)) {
      key = morton3_key(quantize3(x), quantize3(y), quantize3(z));
    } else {
      bad = true;
    }
    keys[i] = key;
    if (counts) atomicAdd(&h[w][(key >> count_shift) & 255u], 1u);
  }
  if (__ballot(bad) != 0 && lane_id() == 0) atomicOr(err, kErrDomain);
  if (counts) store_tile_counts(h, counts, tiles, blockIdx.x);
}

// Keys of query centres for ordering a batch: as keygen_tiles, with the
// coordinates clamped into [0, 1) (queries may lie anywhere, NaN becomes 0)
// and no domain check.
template <int CURVE>
__global__ __launch_bounds__(256) void query_keys_tiles(const double2* __restrict__ q, uint64_t m,
                                                       uint32_t tile_len,
                                                       uint64_t* __restrict__ keys,
                                                       uint32_t* __restrict__ counts,
                                                       uint64_t tiles, int count_shift) {
  __shared__ uint32_t h[kSortWaves][kRadix];
  __shared__ uint16_t lut[CURVE == SFC_CURVE_HILBERT ? 1024 : 1];
  for (int i = threadIdx.x; i < kSortWaves * kRadix; i += 256) (&h[0][0])[i] = 0;
  if (CURVE == SFC_CURVE_HILBERT)
    for (int i = threadIdx.x; i < 1024; i += 256) lut[i] = kHilbertLutConst.v[i];
  __syncthreads();
  const uint64_t base = (uint64_t)blockIdx.x * tile_len;
  const uint64_t end = base + tile_len < m ? base + tile_len : m;
  const uint32_t w = threadIdx.x >> 6;
  constexpr double kBelowOne = 1.0 - 0x1p-53;
  for (uint64_t i = base + threadIdx.x; i < end; i += 256) {
    const double2 p = q[i];
    const double x = p.x >= 0.0 ? (p.x < 1.0 ? p.x : kBelowOne) : 0.0;
    const double y = p.y >= 0.0 ? (p.y < 1.0 ? p.y : kBelowOne) : 0.0;
    const uint32_t ux = quantize(x), uy = quantize(y);
    const uint64_t key =
        CURVE == SFC_CURVE_HILBERT ? hilbert_key_lut(lut, ux, uy) : morton_key(ux, uy);
    keys[i] = key;
    atomicAdd(&h[w][(key >> count_shift) & 255u], 1u);
  }
  store_tile_counts(h, counts, tiles, blockIdx.x);
}

// Point sets whose offsets a set pass stages in LDS (one pass, the set found
// by a binary search there); more sets read the set of every input position
// from an array.
constexpr uint32_t kLdsSets = 256;

// The set of input position v: the last s with off[s] <= v (off: the n_sets
// + 1 set offsets; a set that is empty shares its offset with the next one).
__device__ __forceinline__ uint32_t set_of(const uint64_t* off, uint32_t n_sets, uint32_t v) {
  uint32_t lo = 0, len = n_sets + 1;   // off[lo] <= v
  while (len > 1) {
    const uint32_t half = len >> 1;
    if (off[lo + half] <= v) {
      lo += half;
      len -= half;
    } else {
      len = half;
    }
  }
  return lo;
}

// Digit of an element in a pass: a byte of the key, or (SETPASS) a byte of
// the point set the element's id belongs to (from the offsets in LDS when
// s_off is set, else from set_id).  Padding (id 0xFFFFFFFF) takes digit 255
// so that it sorts last.
template <bool SETPASS>
__device__ __forceinline__ uint32_t pass_digit(uint64_t k, uint32_t v, int shift,
                                               const uint32_t* __restrict__ set_id,
                                               const uint64_t* s_off = nullptr,
                                               uint32_t n_sets = 0) {
  if (!SETPASS) return (uint32_t)(k >> shift) & 255u;
  if (v == 0xFFFFFFFFu) return 255u;
  return ((s_off ? set_of(s_off, n_sets, v) : set_id[v]) >> shift) & 255u;
}

// With set_off (at most kLdsSets sets), a set pass's workgroup copies the set
// offsets into LDS; the caller's barrier follows.
template <bool SETPASS>
__device__ __forceinline__ const uint64_t* stage_set_off(uint64_t* s_off,
                                                         const uint64_t* __restrict__ set_off,
                                                         uint32_t n_sets) {
  if (!SETPASS || !set_off) return nullptr;
  for (uint32_t i = threadIdx.x; i <= n_sets; i += blockDim.x) s_off[i] = set_off[i];
  return s_off;
}

// The tile's digit counts for a pass.
template <bool SETPASS>
__global__ __launch_bounds__(256) void tile_hist(const uint64_t* __restrict__ kin,
                                                 const uint32_t* __restrict__ vin, uint64_t n,
                                                 uint32_t tile_len, int shift,
                                                 const uint32_t* __restrict__ set_id,
                                                 uint32_t* __restrict__ counts, uint64_t tiles,
                                                 const uint64_t* __restrict__ set_off,
                                                 uint32_t n_sets, SortGuard guard) {
  if (guard_skips(guard)) return;
  __shared__ uint32_t h[kSortWaves][kRadix];
  __shared__ uint64_t s_off_mem[SETPASS ? kLdsSets + 1 : 1];
  for (int i = threadIdx.x; i < kSortWaves * kRadix; i += 256) (&h[0][0])[i] = 0;
  const uint64_t* s_off = stage_set_off<SETPASS>(s_off_mem, set_off, n_sets);
  __syncthreads();
  const uint64_t base = (uint64_t)blockIdx.x * tile_len;
  const uint64_t end = base + tile_len < n ? base + tile_len : n;
  const uint32_t w = threadIdx.x >> 6;
  // Eight loads in flight per thread before the counts are taken.
  constexpr int kBatch = 8;
  for (uint64_t i0 = base + threadIdx.x; i0 < end; i0 += 256 * kBatch) {
    // Positions past the tile load its last element (no branch around the
    // loads) and are not counted.
    uint32_t dg[kBatch];
#pragma unroll
    for (int j = 0; j < kBatch; ++j) {
      const uint64_t i = i0 + 256u * j;
      const uint64_t ic = i < end ? i : end - 1;
      const uint32_t d = SETPASS ? pass_digit<true>(0, vin[ic], shift, set_id, s_off, n_sets)
                                 : pass_digit<false>(kin[ic], 0, shift, set_id);
      dg[j] = i < end ? d : (uint32_t)kRadix;
    }
#pragma unroll
    for (int j = 0; j < kBatch; ++j)
      if (dg[j] < (uint32_t)kRadix) atomicAdd(&h[w][dg[j]], 1u);
  }
  store_tile_counts(h, counts, tiles, blockIdx.x);
}

// One workgroup per digit d: rel[d * tiles + t] = sum of the digit's counts
// of tiles < t; dtot[d] = the digit's total.
__global__ __launch_bounds__(256) void digit_scan(const uint32_t* __restrict__ counts,
                                                  uint64_t tiles, uint32_t* __restrict__ rel,
                                                  uint32_t* __restrict__ dtot, SortGuard guard) {
  if (guard_skips(guard)) return;
  __shared__ uint32_t s_tmp[kSortWaves];
  const uint32_t* c = counts + (uint64_t)blockIdx.x * tiles;
  uint32_t* r = rel + (uint64_t)blockIdx.x * tiles;
  uint32_t carry = 0;
  for (uint64_t b = 0; b < tiles; b += 256 * 16) {
    const uint64_t f = b + (uint64_t)threadIdx.x * 16;
    // Sixteen loads in flight: entries past the end load the last one (no
    // branch around the loads) and count as zero.
    uint32_t v[16], sum = 0;
#pragma unroll
    for (int i = 0; i < 16; ++i) {
      const uint64_t j = f + i < tiles ? f + i : tiles - 1;
      v[i] = c[j];
    }
#pragma unroll
    for (int i = 0; i < 16; ++i) {
      if (f + i >= tiles) v[i] = 0u;
      sum += v[i];
    }
    const uint32_t excl = block_excl_scan256(sum, s_tmp);
    uint32_t run = carry + excl;
#pragma unroll
    for (int i = 0; i < 16; ++i) {
      if (f + i < tiles) r[f + i] = run;
      run += v[i];
    }
    // The block total: the last thread's exclusive prefix plus its sum.
    if (threadIdx.x == 255) s_tmp[0] = excl + sum;
    __syncthreads();
    carry += s_tmp[0];
    __syncthreads();
  }
  if (threadIdx.x == 0) dtot[blockIdx.x] = carry;
}

// Tile of workgroup b: XCD b % 8 takes the contiguous tiles
// [x * per, (x + 1) * per); tiles past the end are idle workgroups.
__device__ __forceinline__ uint64_t xcd_tile(uint64_t b, uint64_t tiles) {
  const uint64_t per = (tiles + 7) / 8;
  return (b & 7) * per + (b >> 3);
}

// Threads of a scatter workgroup: eight waves share one tile, each holding a
// quarter of what a four-wave histogram workgroup covers per thread.
constexpr int kScatterWaves = 8;
constexpr int kScatterThreads = kScatterWaves * kWave;

// One stable pass of the LSD radix sort over the digit pass_digit(...).  The
// tile holds kSortThreads * ITEMS keys (the histogram kernels' tile); each of
// the kScatterThreads threads ranks ITEMS * kSortThreads / kScatterThreads of
// them.
template <int ITEMS, bool FIRST, bool GATHER, bool SETPASS>
__global__ __launch_bounds__(kScatterThreads) void scatter_pass(
    const uint64_t* __restrict__ kin, const uint32_t* __restrict__ vin,
    uint64_t* __restrict__ kout, uint32_t* __restrict__ vout, uint64_t n, int shift,
    const uint32_t* __restrict__ rel, const uint32_t* __restrict__ dtot, uint64_t tiles,
    uint32_t* err, const double2* __restrict__ xy_in, double2* __restrict__ xy_out,
    uint64_t* __restrict__ cells_out, int cell_curve, const uint32_t* __restrict__ set_id,
    const uint64_t* __restrict__ set_off, uint32_t n_sets, SortGuard guard) {
  if (guard_skips(guard)) return;
  constexpr int kTile = kSortThreads * ITEMS;
  constexpr int IT = kTile / kScatterThreads;
  static_assert(IT * kScatterThreads == kTile, "tile must split over the scatter threads");
  __shared__ union {
    uint32_t wave_hist[kScatterWaves][kRadix];
    struct {
      uint64_t k[kTile];
      uint32_t v[kTile];
    } st;
  } sm;
  __shared__ uint32_t s_local[kRadix];
  __shared__ uint32_t s_gbase[kRadix];
  __shared__ uint32_t s_tmp[kScatterWaves];
  __shared__ uint64_t s_off_mem[SETPASS ? kLdsSets + 1 : 1];

  const uint64_t tile = xcd_tile(blockIdx.x, tiles);
  if (tile >= tiles) return;   // the whole workgroup: no barrier is skipped by part of it
  const uint32_t tid = threadIdx.x, w = tid >> 6, l = tid & 63;
  for (uint32_t i = tid; i < kScatterWaves * kRadix; i += kScatterThreads)
    (&sm.wave_hist[0][0])[i] = 0;
  const uint64_t* s_off = stage_set_off<SETPASS>(s_off_mem, set_off, n_sets);
  const uint64_t base = tile * kTile;
  const uint64_t wbase = base + (uint64_t)w * (kWave * IT);

  uint64_t key[IT];
  uint32_t val[IT];
  uint32_t rank[IT];
#pragma unroll
  for (int i = 0; i < IT; ++i) {
    const uint64_t idx = wbase + (uint64_t)i * kWave + l;
    if (idx < n) {
      key[i] = kin[idx];
      val[i] = FIRST ? (uint32_t)idx : vin[idx];
    } else {
      key[i] = ~0ull;   // padding sorts to the end of the last digit
      val[i] = 0xFFFFFFFFu;
    }
  }
  // Threads d < 256: this tile's offset within digit d's bucket and the
  // digit's total (read early, used after the ranking).
  const uint32_t d = tid;
  const bool digit_thread = d < (uint32_t)kRadix;
  const uint32_t rl = digit_thread ? rel[(uint64_t)d * tiles + tile] : 0u;
  const uint32_t dt = digit_thread ? dtot[d] : 0u;
  __syncthreads();

  // Rank within the wave, in (item, lane) order: lanes holding the same digit
  // are found with eight ballots; the lowest of them bumps the wave's counter.
  // (The counters are indexed in the shared array itself, so that the
  // accesses stay LDS instructions; a wave's LDS accesses complete in order,
  // and the compiler keeps each slot's read after the previous slot's write,
  // which may alias it.)
  uint32_t* wh = sm.wave_hist[w];
  const uint64_t below_mask = lanemask_lt();
#pragma unroll
  for (int i = 0; i < IT; ++i) {
    const uint32_t dg = pass_digit<SETPASS>(key[i], val[i], shift, set_id, s_off, n_sets);
    uint64_t match = ~0ull;
#pragma unroll
    for (int b = 0; b < 8; ++b) {
      const bool bit = (dg >> b) & 1u;
      const uint64_t bal = __ballot(bit);
      match &= bit ? bal : ~bal;
    }
    const uint32_t cnt = (uint32_t)__popcll(match);
    const uint32_t below = (uint32_t)__popcll(match & below_mask);
    const uint32_t pre = wh[dg];
    if (below == 0) wh[dg] = pre + cnt;
    rank[i] = pre + below;
  }
  __syncthreads();

  // Thread d: tile count of digit d and per-wave exclusive bases.  The scans
  // run over the first four waves (one thread per digit); the other waves
  // pass zeros and take part only in the barriers.
  uint32_t tot = 0;
  if (digit_thread) {
#pragma unroll
    for (int ww = 0; ww < kScatterWaves; ++ww) {
      const uint32_t c = sm.wave_hist[ww][d];
      sm.wave_hist[ww][d] = tot;
      tot += c;
    }
  }
  const uint32_t local = block_excl_scan256(tot, s_tmp);
  const uint32_t dbase = block_excl_scan256(dt, s_tmp);
  if (digit_thread) {
    s_local[d] = local;
    s_gbase[d] = dbase + rl - local;
  }
  __syncthreads();

  uint32_t lpos[IT];
#pragma unroll
  for (int i = 0; i < IT; ++i) {
    const uint32_t dd = pass_digit<SETPASS>(key[i], val[i], shift, set_id, s_off, n_sets);
    lpos[i] = s_local[dd] + sm.wave_hist[w][dd] + rank[i];
  }
  __syncthreads();
#pragma unroll
  for (int i = 0; i < IT; ++i) {
    sm.st.k[lpos[i]] = key[i];
    sm.st.v[lpos[i]] = val[i];
  }
  __syncthreads();

  const uint32_t valid = (uint32_t)((n - base) < (uint64_t)kTile ? (n - base) : (uint64_t)kTile);
  for (uint32_t j = tid; j < valid; j += kScatterThreads) {
    const uint64_t k = sm.st.k[j];
    const uint32_t v = sm.st.v[j];
    const uint32_t pos = s_gbase[pass_digit<SETPASS>(k, v, shift, set_id, s_off, n_sets)] + j;
    if (pos >= n || (GATHER && v >= n)) {   // cannot happen with consistent counts
      atomicOr(err, kErrInternal);
      continue;
    }
    kout[pos] = k;
    vout[pos] = v;
    if (GATHER) {
      const double2 p = xy_in[v];
      xy_out[pos] = p;
      if (cells_out) cells_out[pos] = pack_cell2(p.x, p.y);
    } else if (cells_out) {
      cells_out[pos] = cell_of_key(cell_curve, k);   // the key holds the cell
    }
  }
}

// Occupancy bits of every quadtree node down to depth kOccDepth: point i
// marks the depth-k node of its key for each k where its prefix differs from
// point i-1's (the keys are sorted), so each occupied node is marked once.
__global__ __launch_bounds__(256) void occupancy_mark(const uint64_t* __restrict__ keys, uint64_t n,
                                                      uint32_t* occ) {
  const uint64_t stride = (uint64_t)gridDim.x * 256;
  for (uint64_t i = (uint64_t)blockIdx.x * 256 + threadIdx.x; i < n; i += stride) {
    const uint64_t k = keys[i];
    const uint64_t prev = i > 0 ? keys[i - 1] : ~k;
    for (int dep = 0; dep <= kOccDepth; ++dep) {
      const int sh = 64 - 2 * dep;
      const uint64_t p = dep == 0 ? 0 : k >> sh;
      const bool first = i == 0 || (dep > 0 && (prev >> sh) != p);
      if (!first) continue;
      const uint64_t node = occ_level_offset(dep) + p;
      atomicOr(occ + (node >> 5), 1u << (node & 31));
    }
  }
}

__global__ void gather_points(const uint32_t* __restrict__ ids, const double2* __restrict__ xy,
                              double2* __restrict__ out, uint64_t n, SortGuard guard) {
  if (guard_skips(guard)) return;
  const uint64_t i = (uint64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (i < n) out[i] = xy[ids[i]];
}

__global__ void gather_points3(const uint32_t* __restrict__ ids, const double* __restrict__ xyz,
                               double* __restrict__ out, uint64_t* __restrict__ cells_out,
                               uint64_t n, SortGuard guard) {
  if (guard_skips(guard)) return;
  const uint64_t i = (uint64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (i < n) {
    const uint64_t v = ids[i];
    const double x = xyz[3 * v], y = xyz[3 * v + 1], z = xyz[3 * v + 2];
    out[3 * i] = x;
    out[3 * i + 1] = y;
    out[3 * i + 2] = z;
    if (cells_out) cells_out[i] = pack_cell3(x, y, z);
  }
}

// Keys of a radix tile per histogram thread (the tile is 256 times this): 8,
// 12, 16, 20 or 24.  The environment variable SFC_SORT_ITEMS overrides; else
// the autotuner's choice for this size; else 24 from 2^23 keys on (tiles of
// 6144 keys, two scatter workgroups per CU; at 2^24 keys the build takes
// 0.81 ms against 0.84 with 4096-key tiles) and 16 below.
int sort_items(uint64_t n) {
  static const int env = [] {
    const char* e = std::getenv("SFC_SORT_ITEMS");
    return e ? std::atoi(e) : 0;
  }();
  const int k = env ? env : tuned(kTuneSortItems, n);
  if (k == 8 || k == 12 || k == 16 || k == 20 || k == 24) return k;
  return n >= (1ull << 23) ? 24 : 16;
}
uint64_t sort_tile(uint64_t n) { return (uint64_t)kSortThreads * sort_items(n); }

// Set id of every input position (sets are contiguous in the input).
__global__ void fill_set_ids(const uint64_t* __restrict__ set_off, uint32_t n_sets, uint64_t n,
                             uint32_t* __restrict__ set_id, SortGuard guard) {
  if (guard_skips(guard)) return;
  const uint64_t i = (uint64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= n) return;
  uint32_t lo = 0, len = n_sets + 1;   // last s with set_off[s] <= i
  while (len > 0) {
    const uint32_t h = len >> 1;
    if (set_off[lo + h] <= i) {
      lo += h + 1;
      len -= h + 1;
    } else {
      len = h;
    }
  }
  set_id[i] = lo - 1;
}


// ---- chunked construction: four passes over the top 32 bits, then LDS ----
//
// After four stable passes over the key bytes at bits 32..63 the keys are
// ordered by their top 32 bits, and each run of equal top bits (a quadtree
// cell of side 2^-16, or an octree cell of side about 2^-10.3; one or two
// keys on average at the sizes here) only needs its own order by the
// remaining bits.  The array is cut into chunks of whole runs: chunk c spans
// [b(c), b(c + 1)), b(c) the first run start at or after c * kChunkStride
// (b = n past the end).  A chunk of up to kChunkCap keys (always so when no
// run is longer than kChunkCap - kChunkStride) is sorted by one workgroup in
// LDS and written back in place with each key's grid cell: when every run in
// it has at most kShortRun keys, each key's place in its run is counted
// directly (keys of its run that are smaller, or equal and earlier); else
// the whole chunk takes stable LSD passes over the bytes that vary within
// it.  Sorting inside a chunk leaves the top bits at every position
// unchanged.  A longer chunk raises kErrOversized and writes nothing; the
// caller then runs the plain sort instead.
constexpr int kTopShift = 32;
constexpr int kTopPasses = 4;
constexpr uint64_t kChunkStride = 2048;
constexpr uint32_t kChunkCap = 4096;
constexpr uint32_t kShortRun = 64;
constexpr int kChunkWaves = 8;
constexpr int kChunkThreads = kChunkWaves * kWave;
constexpr int kChunkSlots = kChunkCap / kChunkThreads;   // items per lane at capacity

// Entry c (one wave per stride of kChunkStride positions): the first run
// start in [c * kChunkStride, (c + 1) * kChunkStride) (a position p with
// p == 0 or top bits differing from p - 1's), ~0 if the stride has none;
// entry `chunks` is n.
__global__ __launch_bounds__(256) void chunk_firsts(const uint64_t* __restrict__ keys, uint64_t n,
                                                    uint64_t chunks, uint64_t* __restrict__ first) {
  const uint64_t c = (uint64_t)blockIdx.x * 4 + (threadIdx.x >> 6);
  const uint32_t l = lane_id();
  if (c > chunks) return;
  if (c == chunks) {
    if (l == 0) first[c] = n;
    return;
  }
  const uint64_t base = c * kChunkStride;
  uint64_t found = ~0ull;
  // Eight rows of 64 positions per round, their loads all in flight.
  for (uint32_t g = 0; g < kChunkStride / kWave && found == ~0ull; g += 8) {
    uint64_t m[8];
#pragma unroll
    for (int j = 0; j < 8; ++j) {
      const uint64_t p = base + (uint64_t)(g + j) * kWave + l;
      bool hit = false;
      if (p < n) hit = p == 0 || (keys[p] >> kTopShift) != (keys[p - 1] >> kTopShift);
      m[j] = __ballot(hit);
    }
#pragma unroll
    for (int j = 7; j >= 0; --j)
      if (m[j] != 0)
        found = base + (uint64_t)(g + j) * kWave + (uint64_t)(__ffsll((unsigned long long)m[j]) - 1);
  }
  if (l == 0) first[c] = found;
}

// b(c) from the strides' first run starts: the first entry of
// first[c .. c + kChunkLook] that is not ~0 (entries past `chunks` are n),
// or ~0 when none is (the run through c * kChunkStride is longer than a
// chunk can hold).
constexpr int kChunkLook = (int)(kChunkCap / kChunkStride);
__device__ __forceinline__ uint64_t chunk_bound(const uint64_t* first, uint64_t chunks, uint64_t n,
                                                uint64_t c) {
  for (int j = 0; j <= kChunkLook; ++j) {
    const uint64_t v = c + j <= chunks ? first[c + j] : n;
    if (v != ~0ull) return v;
  }
  return ~0ull;
}

__global__ __launch_bounds__(kChunkThreads) void chunk_sort(
    uint64_t* __restrict__ keys, uint32_t* __restrict__ ids, uint64_t n,
    const uint64_t* __restrict__ first, uint64_t chunks, uint64_t* __restrict__ cells_out,
    int cell_curve, uint32_t* err) {
  __shared__ union {
    uint32_t wave_hist[kChunkWaves][kRadix];
    struct {
      uint64_t k[kChunkCap];
      uint32_t v[kChunkCap];
    } st;
  } sm;
  __shared__ uint32_t s_local[kRadix];
  __shared__ uint32_t s_tmp[kChunkWaves];
  __shared__ uint64_t s_bound[2];
  __shared__ uint32_t s_vary[2];
  __shared__ uint32_t s_long;
  __shared__ uint16_t s_inv[1024];   // inverse Hilbert table for the cells

  const uint32_t tid = threadIdx.x, w = tid >> 6, l = tid & 63;
  const uint64_t c = blockIdx.x;
  if (cells_out && cell_curve == SFC_CURVE_HILBERT)
    for (uint32_t i = tid; i < 1024; i += kChunkThreads) s_inv[i] = kHilbertInvLutConst.v[i];
  if (tid == 0) {
    s_bound[0] = chunk_bound(first, chunks, n, c);
    s_bound[1] = chunk_bound(first, chunks, n, c + 1);
    s_vary[0] = 0;
    s_vary[1] = 0;
    s_long = 0;
  }
  __syncthreads();
  const uint64_t start = s_bound[0], end = s_bound[1];
  if (start == ~0ull || end == ~0ull || end - start > kChunkCap) {
    if (tid == 0) atomicOr(err, kErrOversized);
    return;   // the whole workgroup
  }
  if (end <= start) return;
  const uint32_t len = (uint32_t)(end - start);

  // The chunk into LDS in position order (coalesced), every load of a lane
  // in flight at once: slots past the chunk load its last entry and are not
  // stored.
  {
    uint64_t kb[kChunkSlots];
    uint32_t vb[kChunkSlots];
#pragma unroll
    for (int t = 0; t < kChunkSlots; ++t) {
      const uint32_t j = tid + (uint32_t)t * kChunkThreads;
      const uint64_t g = start + (j < len ? j : len - 1);
      kb[t] = keys[g];
      vb[t] = ids[g];
    }
#pragma unroll
    for (int t = 0; t < kChunkSlots; ++t) {
      const uint32_t j = tid + (uint32_t)t * kChunkThreads;
      if (j < len) {
        sm.st.k[j] = kb[t];
        sm.st.v[j] = vb[t];
      }
    }
  }
  __syncthreads();

  // The bytes that vary within the chunk, and whether a run is longer than
  // kShortRun (the keys being ordered by their top bits, a run holds more
  // than kShortRun keys exactly when some key has the top bits of the key
  // kShortRun places before it).
  const uint64_t k0 = sm.st.k[0];
  uint64_t vary = 0;
  bool is_long = false;
  for (uint32_t j = tid; j < len; j += kChunkThreads) {
    const uint64_t kj = sm.st.k[j];
    vary |= kj ^ k0;
    if (j >= kShortRun && (sm.st.k[j - kShortRun] >> kTopShift) == (kj >> kTopShift)) is_long = true;
  }
#pragma unroll
  for (int o = 32; o >= 1; o >>= 1) vary |= __shfl_xor(vary, o, 64);
  const bool wave_long = __ballot(is_long) != 0;
  if (l == 0) {
    if (vary != 0) {
      atomicOr(&s_vary[0], (uint32_t)vary);
      atomicOr(&s_vary[1], (uint32_t)(vary >> 32));
    }
    if (wave_long) atomicOr(&s_long, 1u);
  }
  __syncthreads();

  if (s_long == 0) {
    // Every run is short: a key's place is its run's start plus the number
    // of keys of the run before it in (key, position) order.  Keys move only
    // within their run, so the writes stay nearly contiguous.
    for (uint32_t j = tid; j < len; j += kChunkThreads) {
      const uint64_t kj = sm.st.k[j];
      const uint64_t t = kj >> kTopShift;
      uint32_t b = j;
      while (b > 0 && (sm.st.k[b - 1] >> kTopShift) == t) --b;
      uint32_t r = 0;
      for (uint32_t q = b; q < len; ++q) {
        const uint64_t kq = sm.st.k[q];
        if ((kq >> kTopShift) != t) break;
        r += (kq < kj || (kq == kj && q < j)) ? 1u : 0u;
      }
      const uint64_t dst = start + b + r;
      keys[dst] = kj;
      ids[dst] = sm.st.v[j];
      if (cells_out) cells_out[dst] = cell_of_key_lut(cell_curve, kj, s_inv);
    }
    return;
  } else {
    // Stable LSD passes over the bytes that vary within the chunk.  Each
    // wave holds a contiguous stretch of `slots` rows of 64 positions, so
    // that (wave, slot, lane) order is position order.
    const uint32_t slots = (len + kChunkThreads - 1) / kChunkThreads;
    const uint32_t wbase = w * slots * kWave;
    const uint64_t vmask = (uint64_t)s_vary[0] | ((uint64_t)s_vary[1] << 32);
    uint64_t key[kChunkSlots];
    uint32_t val[kChunkSlots];
#pragma unroll
    for (int i = 0; i < kChunkSlots; ++i) {
      key[i] = ~0ull;   // padding sorts after every key of the chunk
      val[i] = 0xFFFFFFFFu;
      const uint32_t pos = wbase + i * kWave + l;
      if (i < (int)slots && pos < len) {
        key[i] = sm.st.k[pos];
        val[i] = sm.st.v[pos];
      }
    }
    __syncthreads();   // the items are in registers before the histograms reuse LDS
    const uint64_t below_mask = lanemask_lt();
    for (int shift = 0; shift < 64; shift += 8) {
      if (((vmask >> shift) & 255u) == 0) continue;   // the byte is the same for every key
      uint32_t* wh = sm.wave_hist[w];
      for (uint32_t i = l; i < kRadix; i += kWave) wh[i] = 0;
      uint32_t dig[kChunkSlots], rank[kChunkSlots];
#pragma unroll
      for (int i = 0; i < kChunkSlots; ++i) {
        if (i >= (int)slots) continue;
        const uint32_t dg = (uint32_t)(key[i] >> shift) & 255u;
        uint64_t match = ~0ull;
#pragma unroll
        for (int b = 0; b < 8; ++b) {
          const bool bit = (dg >> b) & 1u;
          const uint64_t bal = __ballot(bit);
          match &= bit ? bal : ~bal;
        }
        const uint32_t cnt = (uint32_t)__popcll(match);
        const uint32_t below = (uint32_t)__popcll(match & below_mask);
        const uint32_t pre = wh[dg];
        if (below == 0) wh[dg] = pre + cnt;
        dig[i] = dg;
        rank[i] = pre + below;
      }
      __syncthreads();
      // Digit d (threads 0..255): per-wave exclusive bases and the chunk's
      // exclusive count of smaller digits.
      if (tid < kRadix) {
        uint32_t tot = 0;
#pragma unroll
        for (int ww = 0; ww < kChunkWaves; ++ww) {
          const uint32_t cw = sm.wave_hist[ww][tid];
          sm.wave_hist[ww][tid] = tot;
          tot += cw;
        }
        uint32_t x = tot;
#pragma unroll
        for (int o = 1; o < 64; o <<= 1) {
          const uint32_t y = __shfl_up(x, o, 64);
          if (l >= (uint32_t)o) x += y;
        }
        if (l == 63) s_tmp[w] = x;
        s_local[tid] = x - tot;
      }
      __syncthreads();
      uint32_t lpos[kChunkSlots];
      {
        const uint32_t add1 = s_tmp[0], add2 = add1 + s_tmp[1], add3 = add2 + s_tmp[2];
#pragma unroll
        for (int i = 0; i < kChunkSlots; ++i) {
          if (i >= (int)slots) continue;
          const uint32_t dg = dig[i], q = dg >> 6;
          const uint32_t wadd = q == 0 ? 0u : (q == 1 ? add1 : (q == 2 ? add2 : add3));
          lpos[i] = s_local[dg] + wadd + sm.wave_hist[w][dg] + rank[i];
        }
      }
      __syncthreads();   // every histogram read is done before the items overwrite it
#pragma unroll
      for (int i = 0; i < kChunkSlots; ++i) {
        if (i >= (int)slots) continue;
        sm.st.k[lpos[i]] = key[i];
        sm.st.v[lpos[i]] = val[i];
      }
      __syncthreads();
#pragma unroll
      for (int i = 0; i < kChunkSlots; ++i) {
        if (i >= (int)slots) continue;
        const uint32_t pos = wbase + i * kWave + l;
        key[i] = sm.st.k[pos];
        val[i] = sm.st.v[pos];
      }
      __syncthreads();   // every item is read back before the next pass's histograms
    }
#pragma unroll
    for (int i = 0; i < kChunkSlots; ++i) {
      if (i >= (int)slots) continue;
      const uint32_t pos = wbase + i * kWave + l;
      sm.st.k[pos] = key[i];
      sm.st.v[pos] = val[i];
    }
    __syncthreads();
  }

  // Out in position order: consecutive lanes, consecutive words.
  for (uint32_t j = tid; j < len; j += kChunkThreads) {
    const uint64_t k = sm.st.k[j];
    keys[start + j] = k;
    ids[start + j] = sm.st.v[j];
    if (cells_out) cells_out[start + j] = cell_of_key_lut(cell_curve, k, s_inv);
  }
}

template <int ITEMS>
hipError_t launch_scatter(bool first, bool gather, bool setpass, int shift, uint64_t tiles,
                          const uint64_t* kin, const uint32_t* vin, uint64_t* kout,
                          uint32_t* vout, uint64_t n, const uint32_t* rel, const uint32_t* dtot,
                          uint32_t* err, const double* xy, double* xy_out, uint64_t* cells_out,
                          int cell_curve, const uint32_t* set_id, const uint64_t* set_off,
                          uint32_t n_sets, SortGuard guard, hipStream_t s) {
  const dim3 g((uint32_t)(((tiles + 7) / 8) * 8)), b(kScatterThreads);
  const double2* xi = (const double2*)xy;
  double2* xo = (double2*)xy_out;
#define SFC_PASS(F, G, S)                                                                      \
  scatter_pass<ITEMS, F, G, S><<<g, b, 0, s>>>(kin, vin, kout, vout, n, shift, rel, dtot,     \
                                               tiles, err, G ? xi : nullptr, G ? xo : nullptr, \
                                               cells_out, cell_curve, set_id, set_off,     \
                                               n_sets, guard)
  if (setpass) {
    if (gather) SFC_PASS(false, true, true);
    else SFC_PASS(false, false, true);
  } else if (first) {
    SFC_PASS(true, false, false);
  } else if (gather) {
    SFC_PASS(false, true, false);
  } else {
    SFC_PASS(false, false, false);
  }
#undef SFC_PASS
  return hipGetLastError();
}

// One stable radix pass over the byte at `shift` of the keys (of the set
// index with setpass): the tiles' digit counts (unless the key pass already
// took them: counted), their scan over the tiles, and the scatter.
hipError_t radix_pass(bool counted, bool first, bool gather, bool setpass, int shift, uint64_t n,
                      const uint64_t* kin, const uint32_t* vin, uint64_t* kout, uint32_t* vout,
                      uint32_t* counts, uint32_t* rel, uint32_t* dtot, uint32_t* err,
                      const double* xy, double* xy_out, uint64_t* cells_out, int curve,
                      const uint32_t* set_id, const uint64_t* set_off, uint32_t n_sets,
                      SortGuard guard, hipStream_t s) {
  const uint32_t tile = (uint32_t)sort_tile(n);
  const uint64_t tiles = (n + tile - 1) / tile;
  hipError_t e;
  if (!counted) {
    ProfScope ps("tile_hist", s);
    if (setpass)
      tile_hist<true><<<(uint32_t)tiles, 256, 0, s>>>(kin, vin, n, tile, shift, set_id, counts,
                                                      tiles, set_off, n_sets, guard);
    else
      tile_hist<false><<<(uint32_t)tiles, 256, 0, s>>>(kin, vin, n, tile, shift, set_id, counts,
                                                       tiles, nullptr, 0, guard);
    if ((e = hipGetLastError()) != hipSuccess) return e;
  }
  {
    ProfScope ps("digit_scan", s);
    digit_scan<<<kRadix, 256, 0, s>>>(counts, tiles, rel, dtot, guard);
    if ((e = hipGetLastError()) != hipSuccess) return e;
  }
  ProfScope ps(setpass ? "set_pass" : "scatter_pass", s);
#define SFC_LAUNCH(I)                                                                          \
  launch_scatter<I>(first, gather, setpass, shift, tiles, kin, vin, kout, vout, n, rel, dtot, err, \
                    xy, xy_out, cells_out, curve, set_id, set_off, n_sets, guard, s)
  switch (sort_items(n)) {
    case 16: return SFC_LAUNCH(16);
    case 12: return SFC_LAUNCH(12);
    case 20: return SFC_LAUNCH(20);
    case 24: return SFC_LAUNCH(24);
    default: return SFC_LAUNCH(8);
  }
#undef SFC_LAUNCH
}

}  // namespace

// Number of stable set passes after the key passes: one byte of the set
// index per pass.
int set_passes(uint32_t n_sets) { return n_sets <= 1 ? 0 : (n_sets <= 256 ? 1 : 2); }

// Device bytes of scratch needed by sort_build for n points.
size_t build_scratch_bytes(uint64_t n) {
  const uint64_t tiles = (n + sort_tile(n) - 1) / sort_tile(n);
  const uint64_t cells = tiles * kRadix;   // (digit, tile) counts of a pass
  size_t b = 0;
  b += align256(n * 8);                    // keys ping
  b += align256(n * 4);                    // ids ping
  b += align256(cells * 4);                // tile counts
  b += align256(cells * 4);                // their scan within each digit
  b += align256(kRadix * 4);               // digit totals
  b += align256(n * 4);                    // set id per input point
  return b;
}

hipError_t launch_keys(const double* xy, uint64_t n, int curve, uint64_t* keys, uint32_t* err,
                       uint32_t* counts, hipStream_t s, double* xy_copy, int count_shift,
                       SortGuard guard) {
  if (n == 0) return hipSuccess;
  const uint32_t tile = (uint32_t)sort_tile(n);
  const uint64_t tiles = (n + tile - 1) / tile;
  ProfScope ps("keygen_tiles", s);
  if (curve == SFC_CURVE_MORTON3)
    keygen3_tiles<<<(uint32_t)tiles, 256, 0, s>>>(xy, n, tile, keys, err, counts, tiles, xy_copy,
                                                  count_shift, guard);
  else if (curve == SFC_CURVE_HILBERT)
    keygen_tiles<SFC_CURVE_HILBERT><<<(uint32_t)tiles, 256, 0, s>>>(
        (const double2*)xy, n, tile, keys, err, counts, tiles, (double2*)xy_copy, count_shift,
        guard);
  else
    keygen_tiles<SFC_CURVE_MORTON><<<(uint32_t)tiles, 256, 0, s>>>(
        (const double2*)xy, n, tile, keys, err, counts, tiles, (double2*)xy_copy, count_shift,
        guard);
  return hipGetLastError();
}

// Full construction into the caller's sorted arrays (keys_out, ids_out,
// xy_out, each with room for n entries); scratch holds build_scratch_bytes(n).
// With n_sets > 1 sets (set_off: device, n_sets + 1 offsets into the input),
// stable passes over the set index follow the key passes, so that the result
// is ordered by (set, key, id) and set s keeps the positions
// [set_off[s], set_off[s+1]).  No host synchronisation: the whole sequence can
// be recorded into a graph.
hipError_t sort_build(const double* xy, uint64_t n, int curve, uint64_t* keys_out,
                      uint32_t* ids_out, double* xy_out, void* scratch, uint32_t* err_host_visible,
                      hipStream_t s, const uint64_t* set_off, uint32_t n_sets,
                      uint64_t* cells_out, double* xy_copy, SortGuard guard) {
  if (n == 0) return hipSuccess;
  const uint32_t tile = (uint32_t)sort_tile(n);
  const uint64_t tiles = (n + tile - 1) / tile;
  const uint64_t cells = tiles * kRadix;
  char* p = (char*)scratch;
  uint64_t* keys_b = (uint64_t*)p;      p += align256(n * 8);
  uint32_t* ids_b = (uint32_t*)p;       p += align256(n * 4);
  uint32_t* counts = (uint32_t*)p;      p += align256(cells * 4);
  uint32_t* rel = (uint32_t*)p;         p += align256(cells * 4);
  uint32_t* dtot = (uint32_t*)p;        p += align256(kRadix * 4);
  uint32_t* set_id = (uint32_t*)p;

  const int sp = set_off ? set_passes(n_sets) : 0;
  const int passes = kDigits + sp;
  // Pass p writes the output buffers when passes - 1 - p is even, so that the
  // last pass lands in them; the keys are generated into the other buffer.
  auto out_is_final = [&](int pass) { return ((passes - 1 - pass) & 1) == 0; };
  uint64_t* keys_first = out_is_final(0) ? keys_b : keys_out;

  hipError_t e = launch_keys(xy, n, curve, keys_first, err_host_visible, counts, s, xy_copy, 0,
                             guard);
  if (e != hipSuccess) return e;
  // Up to kLdsSets sets, the set passes find each element's set from the
  // offsets (in LDS); more, from the set of every input position.
  const uint64_t* lds_off = sp == 1 && n_sets <= kLdsSets ? set_off : nullptr;
  if (sp > 0 && !lds_off) {
    ProfScope ps("set_prep", s);
    fill_set_ids<<<(uint32_t)((n + 255) / 256), 256, 0, s>>>(set_off, n_sets, n, set_id, guard);
    if ((e = hipGetLastError()) != hipSuccess) return e;
  }
  const uint64_t* kin = keys_first;
  const uint32_t* vin = nullptr;
  for (int pass = 0; pass < passes; ++pass) {
    const bool fin = out_is_final(pass);
    uint64_t* kout = fin ? keys_out : keys_b;
    uint32_t* vout = fin ? ids_out : ids_b;
    const bool setpass = pass >= kDigits;
    const int shift = setpass ? 8 * (pass - kDigits) : 8 * pass;
    // With xy_out the points travel with the last pass (in 3-D they are
    // gathered after it); else the last pass writes each element's cell,
    // decoded from its key.
    const bool last = pass == passes - 1;
    const bool gather = last && xy_out && curve != SFC_CURVE_MORTON3;
    uint64_t* pass_cells = last && !(xy_out && curve == SFC_CURVE_MORTON3) ? cells_out : nullptr;
    e = radix_pass(pass == 0, pass == 0, gather, setpass, shift, n, kin, vin, kout, vout, counts,
                   rel, dtot, err_host_visible, xy, xy_out, pass_cells, curve, set_id, lds_off,
                   n_sets, guard, s);
    if (e != hipSuccess) return e;
    kin = kout;
    vin = vout;
  }
  if (curve == SFC_CURVE_MORTON3 && xy_out) {
    ProfScope ps("gather_points3", s);
    gather_points3<<<(uint32_t)((n + 255) / 256), 256, 0, s>>>(ids_out, xy, xy_out, cells_out,
                                                                n, guard);
    if ((e = hipGetLastError()) != hipSuccess) return e;
  }
  return hipSuccess;
}

namespace {
// The chunked sort with its buffers named: the sorted keys and ids land in
// (kfin, ifin), (ktmp, itmp) serve as the other side of the passes.
hipError_t chunked_core(const double* xy, uint64_t n, int curve, uint64_t* kfin, uint32_t* ifin,
                        uint64_t* ktmp, uint32_t* itmp, uint32_t* counts, uint32_t* rel,
                        uint32_t* dtot, uint32_t* err, hipStream_t s, uint64_t* cells_out,
                        double* xy_copy) {
  const uint32_t tile = (uint32_t)sort_tile(n);
  const uint64_t tiles = (n + tile - 1) / tile;
  const uint64_t cells = tiles * kRadix;
  // The passes alternate between the two sides so that the last one lands in
  // (kfin, ifin), where the chunks are then sorted in place.
  auto final_pass = [](int pass) { return ((kTopPasses - 1 - pass) & 1) == 0; };
  uint64_t* keys_first = final_pass(0) ? ktmp : kfin;
  hipError_t e = launch_keys(xy, n, curve, keys_first, err, counts, s, xy_copy, kTopShift);
  if (e != hipSuccess) return e;
  const uint64_t* kin = keys_first;
  const uint32_t* vin = nullptr;
  for (int pass = 0; pass < kTopPasses; ++pass) {
    const bool fin = final_pass(pass);
    uint64_t* kout = fin ? kfin : ktmp;
    uint32_t* vout = fin ? ifin : itmp;
    e = radix_pass(pass == 0, pass == 0, false, false, kTopShift + 8 * pass, n, kin, vin, kout,
                   vout, counts, rel, dtot, err, xy, nullptr, nullptr, curve, nullptr, nullptr, 0,
                   {}, s);
    if (e != hipSuccess) return e;
    kin = kout;
    vin = vout;
  }
  // The strides' first run starts go to the tile counts, free after the last
  // pass (tiles * 256 words hold more than chunks + 1 entries).
  const uint64_t chunks = (n + kChunkStride - 1) / kChunkStride;
  if ((chunks + 1) * 8 > cells * 4) return hipErrorInvalidValue;
  uint64_t* first = (uint64_t*)counts;
  {
    ProfScope ps("chunk_firsts", s);
    chunk_firsts<<<(uint32_t)((chunks + 1 + 3) / 4), 256, 0, s>>>(kfin, n, chunks, first);
    if ((e = hipGetLastError()) != hipSuccess) return e;
  }
  ProfScope ps("chunk_sort", s);
  chunk_sort<<<(uint32_t)chunks, kChunkThreads, 0, s>>>(kfin, ifin, n, first, chunks, cells_out,
                                                         curve, err);
  return hipGetLastError();
}
}  // namespace

hipError_t sort_build_chunked(const double* xy, uint64_t n, int curve, uint64_t* keys_out,
                              uint32_t* ids_out, void* scratch, uint32_t* err, hipStream_t s,
                              uint64_t* cells_out, double* xy_copy) {
  if (n == 0) return hipSuccess;
  const uint64_t cells = (n + sort_tile(n) - 1) / sort_tile(n) * kRadix;
  char* p = (char*)scratch;
  uint64_t* keys_b = (uint64_t*)p;      p += align256(n * 8);
  uint32_t* ids_b = (uint32_t*)p;       p += align256(n * 4);
  uint32_t* counts = (uint32_t*)p;      p += align256(cells * 4);
  uint32_t* rel = (uint32_t*)p;         p += align256(cells * 4);
  uint32_t* dtot = (uint32_t*)p;
  return chunked_core(xy, n, curve, keys_out, ids_out, keys_b, ids_b, counts, rel, dtot, err, s,
                      cells_out, xy_copy);
}

hipError_t sort_build_sets_chunked(const double* xy, uint64_t n, int curve, uint64_t* keys_out,
                                   uint32_t* ids_out, double* xy_out, void* scratch, uint32_t* err,
                                   hipStream_t s, const uint64_t* set_off, uint32_t n_sets,
                                   uint64_t* cells_out, double* xy_copy, bool fallback) {
  if (n == 0) return hipSuccess;
  const uint64_t cells = (n + sort_tile(n) - 1) / sort_tile(n) * kRadix;
  char* p = (char*)scratch;
  uint64_t* keys_b = (uint64_t*)p;      p += align256(n * 8);
  uint32_t* ids_b = (uint32_t*)p;       p += align256(n * 4);
  uint32_t* counts = (uint32_t*)p;      p += align256(cells * 4);
  uint32_t* rel = (uint32_t*)p;         p += align256(cells * 4);
  uint32_t* dtot = (uint32_t*)p;        p += align256(kRadix * 4);
  uint32_t* set_id = (uint32_t*)p;
  const int sp = set_off ? set_passes(n_sets) : 0;
  // The chunked sort lands where the set passes, alternating sides, end in
  // the output.
  const bool odd = (sp & 1) != 0;
  uint64_t* kc = odd ? keys_b : keys_out;
  uint32_t* ic = odd ? ids_b : ids_out;
  hipError_t e = chunked_core(xy, n, curve, kc, ic, odd ? keys_out : keys_b,
                              odd ? ids_out : ids_b, counts, rel, dtot, err, s,
                              sp ? nullptr : cells_out, xy_copy);
  if (e != hipSuccess) return e;
  // The set passes run only on a complete chunked sort.
  const SortGuard when_sorted{err, false};
  const uint64_t* lds_off = sp == 1 && n_sets <= kLdsSets ? set_off : nullptr;
  if (sp > 0 && !lds_off) {
    ProfScope ps("set_prep", s);
    fill_set_ids<<<(uint32_t)((n + 255) / 256), 256, 0, s>>>(set_off, n_sets, n, set_id,
                                                             when_sorted);
    if ((e = hipGetLastError()) != hipSuccess) return e;
  }
  const uint64_t* kin = kc;
  const uint32_t* vin = ic;
  // With xy_out the points travel with the last set pass (in 3-D, or
  // without sets, they are gathered after the sort).
  const bool gather2 = xy_out && curve != SFC_CURVE_MORTON3;
  for (int pass = 0; pass < sp; ++pass) {
    const bool fin = ((sp - 1 - pass) & 1) == 0;
    const bool last = pass == sp - 1;
    uint64_t* kout = fin ? keys_out : keys_b;
    uint32_t* vout = fin ? ids_out : ids_b;
    e = radix_pass(false, false, last && gather2, true, 8 * pass, n, kin, vin, kout, vout, counts,
                   rel, dtot, err, xy, xy_out, last ? cells_out : nullptr, curve, set_id, lds_off,
                   n_sets, when_sorted, s);
    if (e != hipSuccess) return e;
    kin = kout;
    vin = vout;
  }
  if (xy_out && (sp == 0 || !gather2)) {
    ProfScope ps("gather_points", s);
    if (curve == SFC_CURVE_MORTON3)
      gather_points3<<<(uint32_t)((n + 255) / 256), 256, 0, s>>>(ids_out, xy, xy_out, nullptr,
                                                                  n, when_sorted);
    else
      gather_points<<<(uint32_t)((n + 255) / 256), 256, 0, s>>>(
          ids_out, (const double2*)xy, (double2*)xy_out, n, when_sorted);
    if ((e = hipGetLastError()) != hipSuccess) return e;
  }
  if (!fallback) return hipSuccess;
  // A run too long for a chunk: the plain sort, recorded here too, runs then.
  return sort_build(xy, n, curve, keys_out, ids_out, xy_out, scratch, err, s, set_off, n_sets,
                    cells_out, xy_copy, SortGuard{err, true});
}

size_t order_scratch_bytes(uint64_t m) {
  const uint64_t tiles = (m + sort_tile(m) - 1) / sort_tile(m);
  return 2 * align256(m * 8) + align256(m * 4) + 2 * align256(tiles * kRadix * 4) +
         align256(kRadix * 4);
}

hipError_t order_queries(const double* q, uint64_t m, int curve, uint32_t* perm, void* scratch,
                         uint32_t* err, hipStream_t s) {
  if (m == 0) return hipSuccess;
  const uint32_t tile = (uint32_t)sort_tile(m);
  const uint64_t tiles = (m + tile - 1) / tile;
  char* p = (char*)scratch;
  uint64_t* keys_a = (uint64_t*)p;   p += align256(m * 8);
  uint64_t* keys_b = (uint64_t*)p;   p += align256(m * 8);
  uint32_t* ids_b = (uint32_t*)p;    p += align256(m * 4);
  uint32_t* counts = (uint32_t*)p;   p += align256(tiles * kRadix * 4);
  uint32_t* rel = (uint32_t*)p;      p += align256(tiles * kRadix * 4);
  uint32_t* dtot = (uint32_t*)p;
  ProfScope ps("query_order", s);
  hipError_t e;
  if (curve == SFC_CURVE_HILBERT)
    query_keys_tiles<SFC_CURVE_HILBERT><<<(uint32_t)tiles, 256, 0, s>>>(
        (const double2*)q, m, tile, keys_a, counts, tiles, 48);
  else
    query_keys_tiles<SFC_CURVE_MORTON><<<(uint32_t)tiles, 256, 0, s>>>(
        (const double2*)q, m, tile, keys_a, counts, tiles, 48);
  if ((e = hipGetLastError()) != hipSuccess) return e;
  // Two stable passes over the top 16 bits: ids from positions, then perm.
  for (int pass = 0; pass < 2; ++pass) {
    const int shift = 48 + 8 * pass;
    const uint64_t* kin = pass == 0 ? keys_a : keys_b;
    uint64_t* kout = pass == 0 ? keys_b : keys_a;
    uint32_t* vout = pass == 0 ? ids_b : perm;
    if (pass > 0) {
      tile_hist<false><<<(uint32_t)tiles, 256, 0, s>>>(kin, ids_b, m, tile, shift, nullptr, counts,
                                                       tiles, nullptr, 0, SortGuard{});
      if ((e = hipGetLastError()) != hipSuccess) return e;
    }
    digit_scan<<<kRadix, 256, 0, s>>>(counts, tiles, rel, dtot, SortGuard{});
    if ((e = hipGetLastError()) != hipSuccess) return e;
#define SFC_LAUNCH(I)                                                                      \
  launch_scatter<I>(pass == 0, false, false, shift, tiles, kin, ids_b, kout, vout, m, rel, dtot, \
                    err, nullptr, nullptr, nullptr, curve, nullptr, nullptr, 0, SortGuard{}, s)
    switch (sort_items(m)) {
      case 16: e = SFC_LAUNCH(16); break;
      case 12: e = SFC_LAUNCH(12); break;
      case 20: e = SFC_LAUNCH(20); break;
      case 24: e = SFC_LAUNCH(24); break;
      default: e = SFC_LAUNCH(8); break;
    }
#undef SFC_LAUNCH
    if (e != hipSuccess) return e;
  }
  return hipSuccess;
}

hipError_t build_occupancy(const uint64_t* keys, uint64_t n, uint32_t* occ, hipStream_t s) {
  hipError_t e = fill_u32(occ, 0, kOccWords, s);
  if (e != hipSuccess || n == 0) return e;
  ProfScope ps("occupancy_mark", s);
  uint64_t blocks = (n + 255) / 256;
  if (blocks > 8192) blocks = 8192;
  occupancy_mark<<<(uint32_t)blocks, 256, 0, s>>>(keys, n, occ);
  return hipGetLastError();
}

hipError_t gather_sorted(const uint32_t* ids, const double* xy, double* out, uint64_t n, int dim,
                         hipStream_t s) {
  if (n == 0) return hipSuccess;
  ProfScope ps("gather_points", s);
  if (dim == 3)
    gather_points3<<<(uint32_t)((n + 255) / 256), 256, 0, s>>>(ids, xy, out, nullptr, n,
                                                                SortGuard{});
  else
    gather_points<<<(uint32_t)((n + 255) / 256), 256, 0, s>>>(ids, (const double2*)xy,
                                                               (double2*)out, n, SortGuard{});
  return hipGetLastError();
}

}  // namespace sfc
