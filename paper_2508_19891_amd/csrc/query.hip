// Batched distance queries (Alg. 1 over cells(Q); Problem Statement).
//
//   ranges_search  one lane per (query, slot), four slots per query.  Every
//                  lane of a query derives the widened integer box, the
//                  level l = ceil(log2 side), the at most four level-l cells
//                  meeting the box and their merged key intervals (the
//                  Observation gives each cell's interval); slot r then runs
//                  the two searches of interval r over the sorted keys.  The
//                  candidate counts are scanned in the same kernel (block
//                  scan + decoupled look-back) into segment offsets.
//   compact        the candidates of all queries form one flat index space;
//                  a block tests 2048 consecutive candidates (four waves of
//                  eight 64-lane rows) with the exact distance test, learns
//                  its output position through a decoupled look-back and
//                  writes the reported ids, in candidate order, plus the CSR
//                  offsets of the queries whose candidates start in it.
#include <hip/hip_runtime.h>

#include "common.h"
#include "curve.h"
#include "internal.h"

namespace sfc {

namespace {

constexpr double kTwo33 = 8589934592.0;        // 2^33
constexpr double kTwoM19 = 1.0 / 524288.0;     // 2^-19
constexpr int64_t kMaxCell = 4294967295LL;     // 2^32 - 1

// The distance test in binary64, fixed order, no contraction.
__device__ __forceinline__ bool within(double px, double py, double qx, double qy, double d) {
#pragma clang fp contract(off)
  const double dx = px - qx;
  const double dy = py - qy;
  const double t = dx * dx;
  const double u = dy * dy;
  const double s = t + u;
  const double r2 = d * d;
  return s <= r2;
}

__device__ __forceinline__ bool finite(double v) { return __builtin_isfinite(v); }

__device__ __forceinline__ int64_t floor_clamped(double v) {
  v = v < -kTwo33 ? -kTwo33 : v;
  v = v > kTwo33 ? kTwo33 : v;
  return (int64_t)__builtin_floor(v);
}

// One axis of the query box, widened by w = 1 + floor((|c| + d) 2^-19)
// quanta on both sides so that it holds every point the rounded distance
// test can accept; then clipped to the grid.  False when it misses the grid.
__device__ __forceinline__ bool axis_box(double c, double d, int64_t& lo, int64_t& hi) {
#pragma clang fp contract(off)
  double wr = __builtin_floor((__builtin_fabs(c) + d) * kTwoM19);
  wr = wr > kTwo33 ? kTwo33 : wr;
  const int64_t w = 1 + (int64_t)wr;
  int64_t l = floor_clamped((c - d) * kTwo32) - w;
  int64_t h = floor_clamped((c + d) * kTwo32) + w;
  l = l < 0 ? 0 : l;
  h = h > kMaxCell ? kMaxCell : h;
  lo = l;
  hi = h;
  return l <= h;
}

template <int CURVE>
__device__ __forceinline__ uint64_t cell_key(const uint16_t* lut, uint32_t x, uint32_t y) {
  return CURVE == SFC_CURVE_HILBERT ? hilbert_key_lut(lut, x, y) : morton_key(x, y);
}

// Merged key intervals of cells(Q) for query (qx, qy, d); returns their
// number (0..4), ascending and non-adjacent.
template <int CURVE>
__device__ int query_ranges(const uint16_t* lut, double qx, double qy, double d, uint64_t lo[4],
                            uint64_t hi[4]) {
  int64_t lx, hx, ly, hy;
  if (!axis_box(qx, d, lx, hx) || !axis_box(qy, d, ly, hy)) return 0;
  const uint64_t sx = (uint64_t)(hx - lx + 1), sy = (uint64_t)(hy - ly + 1);
  const uint64_t side = sx > sy ? sx : sy;
  const int L = side <= 1 ? 0 : 64 - __clzll(side - 1);   // ceil(log2 side)
  if (L >= 32) {
    lo[0] = 0;
    hi[0] = ~0ull;
    return 1;
  }
  const uint64_t span = (1ull << (2 * L)) - 1;
  const uint32_t cx0 = (uint32_t)(lx >> L), cx1 = (uint32_t)(hx >> L);
  const uint32_t cy0 = (uint32_t)(ly >> L), cy1 = (uint32_t)(hy >> L);
  int k = 0;
  for (uint32_t cx = cx0; cx <= cx1; ++cx) {
    for (uint32_t cy = cy0; cy <= cy1; ++cy) {
      const uint64_t key = cell_key<CURVE>(lut, cx << L, cy << L) & ~span;
      lo[k] = key;
      hi[k] = key | span;
      ++k;
    }
  }
  // Sort (at most four) by lower end, then merge intervals that touch.
  for (int i = 1; i < k; ++i) {
    for (int j = i; j > 0 && lo[j - 1] > lo[j]; --j) {
      const uint64_t a = lo[j], b = hi[j];
      lo[j] = lo[j - 1];
      hi[j] = hi[j - 1];
      lo[j - 1] = a;
      hi[j - 1] = b;
    }
  }
  int r = 0;
  for (int i = 0; i < k; ++i) {
    if (r > 0 && hi[r - 1] + 1 == lo[i]) {
      hi[r - 1] = hi[i];
    } else {
      lo[r] = lo[i];
      hi[r] = hi[i];
      ++r;
    }
  }
  return r;
}

// b = first index with keys[i] >= klo; e = first index with keys[i] > khi.
// The two searches are interleaved to keep two loads in flight.
__device__ __forceinline__ void search_pair(const uint64_t* __restrict__ keys, uint64_t n,
                                            uint64_t klo, uint64_t khi, uint64_t& b,
                                            uint64_t& e) {
  uint64_t bl = 0, blen = n, el = 0, elen = n;
  while (blen > 0 || elen > 0) {
    if (blen > 0) {
      const uint64_t h = blen >> 1;
      if (keys[bl + h] < klo) {
        bl += h + 1;
        blen -= h + 1;
      } else {
        blen = h;
      }
    }
    if (elen > 0) {
      const uint64_t h = elen >> 1;
      if (keys[el + h] <= khi) {
        el += h + 1;
        elen -= h + 1;
      } else {
        elen = h;
      }
    }
  }
  b = bl;
  e = el;
}

// Exclusive scan of one uint64 per thread over 256 threads; *total gets the
// block sum (valid after the call in every thread).
__device__ __forceinline__ uint64_t block_excl_scan256_u64(uint64_t v, uint64_t* s_tmp,
                                                           uint64_t* total) {
  const uint32_t lane = threadIdx.x & 63, w = threadIdx.x >> 6;
  uint64_t x = v;
#pragma unroll
  for (int o = 1; o < 64; o <<= 1) {
    const uint64_t y = __shfl_up(x, o, 64);
    if (lane >= (uint32_t)o) x += y;
  }
  if (lane == 63) s_tmp[w] = x;
  __syncthreads();
  uint64_t add = 0, tot = 0;
  for (uint32_t i = 0; i < 4; ++i) {
    if (i < w) add += s_tmp[i];
    tot += s_tmp[i];
  }
  __syncthreads();
  *total = tot;
  return x - v + add;
}

template <int CURVE>
__global__ __launch_bounds__(256) void ranges_search(
    const double2* __restrict__ q, const double* __restrict__ delta, uint64_t m,
    const uint64_t* __restrict__ keys, uint64_t n, uint32_t* __restrict__ slot_begin,
    uint64_t* __restrict__ seg_off, uint64_t* blk_status, uint32_t* counters,
    uint64_t* __restrict__ dbg_lo, uint64_t* __restrict__ dbg_hi, uint64_t* __restrict__ dbg_b,
    uint64_t* __restrict__ dbg_e, uint32_t* __restrict__ dbg_nr) {
  __shared__ uint16_t lut[CURVE == SFC_CURVE_HILBERT ? 1024 : 1];
  __shared__ uint64_t s_tmp[4];
  __shared__ uint64_t s_prefix;
  __shared__ uint32_t s_blk;
  if (threadIdx.x == 0) s_blk = atomicAdd(&counters[0], 1u);
  if (CURVE == SFC_CURVE_HILBERT)
    for (int i = threadIdx.x; i < 1024; i += 256) lut[i] = kHilbertLutConst.v[i];
  __syncthreads();
  const uint64_t blk = s_blk;
  const uint64_t g = blk * 256 + threadIdx.x;
  const uint64_t j = g >> 2;
  const int r = (int)(g & 3);

  uint64_t cnt = 0, b = 0, e = 0, klo = 0, khi = 0;
  int nr = 0;
  bool bad = false;
  if (j < m) {
    const double2 qq = q[j];
    const double d = delta[j];
    if (!(finite(qq.x) && finite(qq.y) && finite(d) && d >= 0.0)) {
      bad = true;
    } else {
      uint64_t lo[4], hi[4];
      nr = query_ranges<CURVE>(lut, qq.x, qq.y, d, lo, hi);
      if (r < nr) {
        klo = lo[r];
        khi = hi[r];
        search_pair(keys, n, klo, khi, b, e);
        cnt = e - b;
      }
    }
  }
  if (__ballot(bad) != 0 && lane_id() == 0) atomicOr(&counters[2], kErrInvalidQuery);
  if (j < m) {
    slot_begin[g] = (uint32_t)b;
    if (dbg_lo) {
      dbg_lo[g] = klo;
      dbg_hi[g] = khi;
      dbg_b[g] = b;
      dbg_e[g] = e;
      if (r == 0) dbg_nr[j] = (uint32_t)nr;
    }
  }

  uint64_t tot;
  const uint64_t excl = block_excl_scan256_u64(cnt, s_tmp, &tot);
  if (threadIdx.x == 0) {
    if (blk > 0) st_release_agent(blk_status + blk, kFlagAggregate | tot);
    s_prefix = lookback_publish(blk_status, blk, 1, 0, tot, &counters[2]);
  }
  __syncthreads();
  const uint64_t nseg = 4 * m;
  if (g < nseg) {
    seg_off[g] = s_prefix + excl;
    if (g == nseg - 1) seg_off[nseg] = s_prefix + excl + cnt;
  }
}

// Largest s in [0, nseg) with seg_off[s] <= c (seg_off[0] = 0 <= c).
__device__ __forceinline__ uint64_t segment_of(const uint64_t* __restrict__ seg_off,
                                               uint64_t nseg, uint64_t c) {
  uint64_t lo = 0, len = nseg + 1;   // first index with seg_off[i] > c, minus one
  while (len > 0) {
    const uint64_t h = len >> 1;
    if (seg_off[lo + h] <= c) {
      lo += h + 1;
      len -= h + 1;
    } else {
      len = h;
    }
  }
  return lo - 1;
}

// First query index qq in [0, m] with seg_off[4 qq] >= v (m if none).
__device__ __forceinline__ uint64_t first_query_at(const uint64_t* __restrict__ seg_off,
                                                   uint64_t m, uint64_t v) {
  uint64_t lo = 0, len = m;
  while (len > 0) {
    const uint64_t h = len >> 1;
    if (seg_off[4 * (lo + h)] < v) {
      lo += h + 1;
      len -= h + 1;
    } else {
      len = h;
    }
  }
  return lo;
}

constexpr int kRows = 8;
static_assert(kCompactTile == 4 * kWave * kRows, "tile shape");

__global__ __launch_bounds__(256) void compact_kernel(
    const double2* __restrict__ q, const double* __restrict__ delta, uint64_t m,
    const double2* __restrict__ pts, const uint32_t* __restrict__ ids, uint64_t npts,
    const uint64_t* __restrict__ seg_off, const uint32_t* __restrict__ slot_begin,
    uint64_t total_cand, uint64_t chunk_base, uint64_t* status, uint32_t* counters,
    const uint64_t* carry_in, uint64_t* carry_out, uint64_t* __restrict__ offsets,
    uint32_t* __restrict__ out_ids, uint64_t cap) {
  __shared__ uint64_t s_rowmask[32];
  __shared__ uint32_t s_rowpre[32];
  __shared__ uint64_t s_prefix;
  __shared__ uint64_t s_qrange[2];
  __shared__ uint32_t s_tile;
  __shared__ uint32_t s_tilehits;

  const uint32_t tid = threadIdx.x, w = tid >> 6, lane = tid & 63;
  if (tid == 0) s_tile = atomicAdd(&counters[1], 1u);
  __syncthreads();
  const uint64_t tile = s_tile;
  const uint64_t tile_start = chunk_base + tile * kCompactTile;
  const uint64_t nseg = 4 * m;
  const uint64_t c0 = tile_start + (uint64_t)w * (kWave * kRows);

  uint64_t seg = 0;
  if (c0 < total_cand) seg = segment_of(seg_off, nseg, c0);

  uint32_t myid[kRows];
  uint64_t bal[kRows];
#pragma unroll
  for (int jr = 0; jr < kRows; ++jr) {
    const uint64_t r0 = c0 + (uint64_t)jr * kWave;
    const uint64_t c = r0 + lane;
    bool hit = false;
    myid[jr] = 0;
    if (r0 < total_cand) {
      const bool active = c < total_cand;
      // Lane i holds the end of segment seg + i, relative to the row start
      // (capped at 64).  The segment of candidate c is seg plus the number
      // of those ends at or before c.
      const uint64_t wi = seg + 1 + lane;
      uint32_t rel = 64;
      if (wi <= nseg) {
        const uint64_t W = seg_off[wi];
        rel = (W - r0) >= 64 ? 64u : (uint32_t)(W - r0);
      }
      uint32_t k = 0;
#pragma unroll
      for (uint32_t bstep = 32; bstep >= 1; bstep >>= 1) {
        const uint32_t v = (uint32_t)__shfl((int)rel, (int)(k + bstep - 1), 64);
        if (v <= lane) k += bstep;
      }
      const uint32_t last = (uint32_t)__shfl((int)rel, 63, 64);
      if (k == 63 && last <= lane) k = 64;
      uint64_t sc = seg + k;
      if (k == 64 && active) sc = segment_of(seg_off, nseg, c);   // window exhausted (rare)
      if (active) {
        const uint64_t qi = sc >> 2;
        const uint64_t pos = (uint64_t)slot_begin[sc] + (c - seg_off[sc]);
        if (pos < npts && qi < m) {
          const double2 p = pts[pos];
          const double2 qq = q[qi];
          hit = within(p.x, p.y, qq.x, qq.y, delta[qi]);
          if (hit) myid[jr] = ids[pos];
        } else {
          atomicOr(&counters[2], kErrLookback);   // inconsistent segment map
        }
      }
      seg = __shfl(sc, 63, 64);
    }
    bal[jr] = __ballot(hit);
  }

  if (lane == 0) {
#pragma unroll
    for (int jr = 0; jr < kRows; ++jr) s_rowmask[w * kRows + jr] = bal[jr];
  }
  __syncthreads();
  if (tid == 0) {
    uint32_t acc = 0;
    for (int r = 0; r < 32; ++r) {
      s_rowpre[r] = acc;
      acc += (uint32_t)__popcll(s_rowmask[r]);
    }
    s_tilehits = acc;
    if (tile > 0) st_release_agent(status + tile, kFlagAggregate | acc);
    const uint64_t excl = lookback_publish(status, tile, 1, 0, acc, &counters[2]);
    s_prefix = carry_in[0] + excl;
  }
  if (tid == 1) s_qrange[0] = first_query_at(seg_off, m, tile_start);
  if (tid == 2) {
    const uint64_t tile_end = tile_start + kCompactTile;
    s_qrange[1] = tile_end >= total_cand ? m : first_query_at(seg_off, m, tile_end);
  }
  __syncthreads();
  const uint64_t prefix = s_prefix;

  const uint64_t below = lanemask_lt();
#pragma unroll
  for (int jr = 0; jr < kRows; ++jr) {
    if ((bal[jr] >> lane) & 1ull) {
      const uint64_t pos = prefix + s_rowpre[w * kRows + jr] + (uint64_t)__popcll(bal[jr] & below);
      if (pos < cap) out_ids[pos] = myid[jr];
    }
  }

  // CSR offsets of the queries whose first candidate lies in this tile (and,
  // for the last tile, of the trailing queries without candidates).
  const uint64_t valid = total_cand - tile_start < kCompactTile ? total_cand - tile_start
                                                                : kCompactTile;
  for (uint64_t qq = s_qrange[0] + tid; qq < s_qrange[1]; qq += 256) {
    const uint64_t x = seg_off[4 * qq] - tile_start;
    uint64_t hb;
    if (x >= valid) {
      hb = s_tilehits;
    } else {
      const uint32_t r = (uint32_t)(x >> 6), bpos = (uint32_t)(x & 63);
      hb = s_rowpre[r] + (uint64_t)__popcll(s_rowmask[r] & ((1ull << bpos) - 1));
    }
    offsets[qq] = prefix + hb;
  }
  if (tid == 0 && tile_start + valid == total_cand) {
    offsets[m] = prefix + s_tilehits;
    carry_out[0] = prefix + s_tilehits;
  } else if (tid == 0 && valid == kCompactTile && tile_start + kCompactTile ==
                                                      chunk_base + kCompactChunkTiles * kCompactTile) {
    carry_out[0] = prefix + s_tilehits;   // last tile of a full chunk
  }
}

__global__ void fill64_kernel(uint64_t* p, uint64_t v, uint64_t count) {
  const uint64_t stride = (uint64_t)gridDim.x * blockDim.x;
  for (uint64_t i = (uint64_t)blockIdx.x * blockDim.x + threadIdx.x; i < count; i += stride)
    p[i] = v;
}
__global__ void fill32_kernel(uint32_t* p, uint32_t v, uint64_t count) {
  const uint64_t stride = (uint64_t)gridDim.x * blockDim.x;
  for (uint64_t i = (uint64_t)blockIdx.x * blockDim.x + threadIdx.x; i < count; i += stride)
    p[i] = v;
}

uint32_t fill_blocks(uint64_t count) {
  uint64_t b = (count + 255) / 256;
  if (b > 2048) b = 2048;
  return b < 1 ? 1 : (uint32_t)b;
}

}  // namespace

hipError_t fill_u64(uint64_t* p, uint64_t value, uint64_t count, hipStream_t s) {
  if (count == 0) return hipSuccess;
  fill64_kernel<<<fill_blocks(count), 256, 0, s>>>(p, value, count);
  return hipGetLastError();
}
hipError_t fill_u32(uint32_t* p, uint32_t value, uint64_t count, hipStream_t s) {
  if (count == 0) return hipSuccess;
  fill32_kernel<<<fill_blocks(count), 256, 0, s>>>(p, value, count);
  return hipGetLastError();
}

size_t query_scratch_bytes(uint64_t m) {
  const uint64_t nseg = 4 * m;
  const uint64_t blocks = (nseg + 255) / 256;
  return align256(nseg * 4) + align256((nseg + 1) * 8) + align256(blocks * 8) + align256(64) +
         align256(64) + align256(kCompactChunkTiles * 8);
}

void query_scratch_carve(void* base, uint64_t m, QueryScratch* qs) {
  const uint64_t nseg = 4 * m;
  const uint64_t blocks = (nseg + 255) / 256;
  char* p = (char*)base;
  qs->slot_begin = (uint32_t*)p;  p += align256(nseg * 4);
  qs->seg_off = (uint64_t*)p;     p += align256((nseg + 1) * 8);
  qs->blk_status = (uint64_t*)p;  p += align256(blocks * 8);
  qs->counters = (uint32_t*)p;    p += align256(64);
  qs->carry = (uint64_t*)p;       p += align256(64);
  qs->tile_status = (uint64_t*)p;
}

hipError_t launch_ranges(const double* q, const double* delta, uint64_t m, const uint64_t* keys,
                         uint64_t n, int curve, const QueryScratch& qs, uint64_t* dbg_lo,
                         uint64_t* dbg_hi, uint64_t* dbg_b, uint64_t* dbg_e, uint32_t* dbg_nr,
                         hipStream_t s) {
  if (m == 0) return hipSuccess;
  const uint64_t blocks = (4 * m + 255) / 256;
  hipError_t e;
  if ((e = fill_u64(qs.blk_status, 0, blocks, s)) != hipSuccess) return e;
  if ((e = fill_u32(qs.counters, 0, 16, s)) != hipSuccess) return e;
  if ((e = fill_u64(qs.carry, 0, 8, s)) != hipSuccess) return e;
  ProfScope ps("ranges_search", s);
  if (curve == SFC_CURVE_HILBERT)
    ranges_search<SFC_CURVE_HILBERT><<<(uint32_t)blocks, 256, 0, s>>>(
        (const double2*)q, delta, m, keys, n, qs.slot_begin, qs.seg_off, qs.blk_status,
        qs.counters, dbg_lo, dbg_hi, dbg_b, dbg_e, dbg_nr);
  else
    ranges_search<SFC_CURVE_MORTON><<<(uint32_t)blocks, 256, 0, s>>>(
        (const double2*)q, delta, m, keys, n, qs.slot_begin, qs.seg_off, qs.blk_status,
        qs.counters, dbg_lo, dbg_hi, dbg_b, dbg_e, dbg_nr);
  return hipGetLastError();
}

hipError_t launch_compact(const double* q, const double* delta, uint64_t m, const double* pts,
                          const uint32_t* ids, uint64_t npts, const QueryScratch& qs,
                          uint64_t total_cand,
                          uint64_t* offsets, uint32_t* out_ids, uint64_t cap, hipStream_t s) {
  hipError_t e;
  if (m == 0) return fill_u64(offsets, 0, 1, s);
  if (total_cand == 0) {
    if ((e = fill_u64(offsets, 0, m + 1, s)) != hipSuccess) return e;
    return fill_u64(qs.carry, 0, 2, s);
  }
  const uint64_t tiles = (total_cand + kCompactTile - 1) / kCompactTile;
  uint64_t chunk = 0;
  for (uint64_t t0 = 0; t0 < tiles; t0 += kCompactChunkTiles, ++chunk) {
    const uint64_t nt = tiles - t0 < kCompactChunkTiles ? tiles - t0 : kCompactChunkTiles;
    if ((e = fill_u64(qs.tile_status, 0, nt, s)) != hipSuccess) return e;
    if ((e = fill_u32(qs.counters + 1, 0, 1, s)) != hipSuccess) return e;
    ProfScope ps("compact", s);
    compact_kernel<<<(uint32_t)nt, 256, 0, s>>>(
        (const double2*)q, delta, m, (const double2*)pts, ids, npts, qs.seg_off, qs.slot_begin,
        total_cand, t0 * kCompactTile, qs.tile_status, qs.counters, qs.carry + (chunk & 1),
        qs.carry + ((chunk + 1) & 1), offsets, out_ids, cap);
    if ((e = hipGetLastError()) != hipSuccess) return e;
  }
  // The final total sits in carry[chunks & 1]; copy it to carry[2].
  (void)chunk;
  return hipSuccess;
}

}  // namespace sfc
