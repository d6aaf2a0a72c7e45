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

// Cells of cells(Q) for the widened box of (qx, qy, d), unmerged and sorted
// by key: cell k covers keys [lo[k], hi[k]] and grid cells
// [cx[k] << L, (cx[k] + 1) << L) x [cy[k] << L, (cy[k] + 1) << L).  Returns the
// number of cells (0..4); *L receives the level, box the widened box.
template <int CURVE>
__device__ int query_cells(const uint16_t* lut, double qx, double qy, double d, uint64_t lo[4],
                           uint64_t hi[4], uint32_t cx[4], uint32_t cy[4], int* Lout,
                           int64_t box[4]) {
  int64_t lx, hx, ly, hy;
  if (!axis_box(qx, d, lx, hx) || !axis_box(qy, d, ly, hy)) return 0;
  box[0] = lx;
  box[1] = hx;
  box[2] = ly;
  box[3] = hy;
  const uint64_t sx = (uint64_t)(hx - lx + 1), sy = (uint64_t)(hy - ly + 1);
  const uint64_t side = sx > sy ? sx : sy;
  const int L = side <= 1 ? 0 : 64 - __clzll(side - 1);
  *Lout = L;
  if (L >= 32) {
    lo[0] = 0;
    hi[0] = ~0ull;
    cx[0] = cy[0] = 0;
    return 1;
  }
  const uint64_t span = (1ull << (2 * L)) - 1;
  int k = 0;
  for (uint32_t x = (uint32_t)(lx >> L); x <= (uint32_t)(hx >> L); ++x) {
    for (uint32_t y = (uint32_t)(ly >> L); y <= (uint32_t)(hy >> L); ++y) {
      const uint64_t key = cell_key<CURVE>(lut, x << L, y << L) & ~span;
      int j = k++;
      for (; j > 0 && lo[j - 1] > key; --j) {
        lo[j] = lo[j - 1];
        hi[j] = hi[j - 1];
        cx[j] = cx[j - 1];
        cy[j] = cy[j - 1];
      }
      lo[j] = key;
      hi[j] = key | span;
      cx[j] = x;
      cy[j] = y;
    }
  }
  return k;
}

__device__ __forceinline__ void search_within(const uint64_t* __restrict__ keys, uint64_t b,
                                              uint64_t e, uint64_t klo, uint64_t khi,
                                              uint64_t& rb, uint64_t& re) {
  uint64_t x, y;
  search_pair(keys + b, e - b, klo, khi, x, y);
  rb = b + x;
  re = b + y;
}

// One lane per (query, slot).
//   REFINE = false: four slots per query, slot r holds the r-th merged key
//     range of cells(Q) and its index range (the method as stated: at most
//     four ranges, two binary searches each).
//   REFINE = true: eight slots per query, lane r handles the r-th cell of
//     cells(Q) (by key).  After the two searches of the cell, a cell holding
//     more than refine_min points is split once: its four children meet the
//     box or not, the children that do are merged into at most two key runs
//     (consecutive children in key order), and each run is located by two
//     searches inside the cell's index range.  Only points outside the box
//     are dropped, so the reported set and its order are unchanged.
template <int CURVE, bool REFINE>
__global__ __launch_bounds__(256) void ranges_search(
    const double2* __restrict__ q, const double* __restrict__ delta, uint64_t m,
    const uint64_t* __restrict__ keys, uint64_t n, uint32_t refine_min,
    uint32_t* __restrict__ slot_begin, uint32_t* __restrict__ slot_count, uint32_t* counters,
    uint64_t* __restrict__ dbg_lo, uint64_t* __restrict__ dbg_hi, uint64_t* __restrict__ dbg_b,
    uint64_t* __restrict__ dbg_e, uint32_t* __restrict__ dbg_nr) {
  __shared__ uint16_t lut[CURVE == SFC_CURVE_HILBERT ? 1024 : 1];
  if (CURVE == SFC_CURVE_HILBERT)
    for (int i = threadIdx.x; i < 1024; i += 256) lut[i] = kHilbertLutConst.v[i];
  __syncthreads();
  const uint64_t g = (uint64_t)blockIdx.x * 256 + threadIdx.x;
  const uint64_t j = g >> 2;
  const int r = (int)(g & 3);

  uint64_t b0 = 0, e0 = 0, b1 = 0, e1 = 0, klo = 0, khi = 0;
  int nr = 0;
  bool bad = false;
  if (j < m) {
    const double2 qq = q[j];
    const double d = delta[j];
    if (!(finite(qq.x) && finite(qq.y) && finite(d) && d >= 0.0)) {
      bad = true;
    } else if (!REFINE) {
      uint64_t lo[4], hi[4];
      nr = query_ranges<CURVE>(lut, qq.x, qq.y, d, lo, hi);
      if (r < nr) {
        klo = lo[r];
        khi = hi[r];
        search_pair(keys, n, klo, khi, b0, e0);
      }
    } else {
      uint64_t lo[4], hi[4];
      uint32_t cx[4], cy[4];
      int64_t box[4];
      int L = 0;
      nr = query_cells<CURVE>(lut, qq.x, qq.y, d, lo, hi, cx, cy, &L, box);
      if (r < nr) {
        search_pair(keys, n, lo[r], hi[r], b0, e0);
        if (e0 - b0 > refine_min && L >= 1 && L < 32) {
          // Children at level L-1 that meet the box, in key order.
          const int Lc = L - 1;
          const uint64_t cspan = (1ull << (2 * Lc)) - 1;
          uint64_t clo[4];
          int nc = 0;
          for (uint32_t dx = 0; dx < 2; ++dx) {
            for (uint32_t dy = 0; dy < 2; ++dy) {
              const int64_t x0 = (int64_t)((2 * cx[r] + dx) << Lc);
              const int64_t y0 = (int64_t)((2 * cy[r] + dy) << Lc);
              const int64_t x1 = x0 + ((int64_t)1 << Lc) - 1, y1 = y0 + ((int64_t)1 << Lc) - 1;
              if (x1 < box[0] || x0 > box[1] || y1 < box[2] || y0 > box[3]) continue;
              const uint64_t key =
                  cell_key<CURVE>(lut, (uint32_t)x0, (uint32_t)y0) & ~cspan;
              int t = nc++;
              for (; t > 0 && clo[t - 1] > key; --t) clo[t] = clo[t - 1];
              clo[t] = key;
            }
          }
          // Runs of consecutive children (at most two of four).
          uint64_t rlo[2] = {0, 0}, rhi[2] = {0, 0};
          int nrun = 0;
          for (int t = 0; t < nc; ++t) {
            if (nrun > 0 && rhi[nrun - 1] + 1 == clo[t]) {
              rhi[nrun - 1] = clo[t] | cspan;
            } else {
              rlo[nrun] = clo[t];
              rhi[nrun] = clo[t] | cspan;
              ++nrun;
            }
          }
          if (nrun == 1 && rlo[0] == lo[r] && rhi[0] == hi[r]) {
            // every child meets the box: keep the cell's range
          } else {
            const uint64_t pb = b0, pe = e0;
            search_within(keys, pb, pe, rlo[0], rhi[0], b0, e0);
            if (nrun > 1) search_within(keys, pb, pe, rlo[1], rhi[1], b1, e1);
          }
        }
      }
    }
  }
  if (__ballot(bad) != 0 && lane_id() == 0) atomicOr(&counters[2], kErrInvalidQuery);
  if (j < m) {
    if (!REFINE) {
      slot_begin[g] = (uint32_t)b0;
      slot_count[g] = (uint32_t)(e0 - b0);
      if (dbg_lo) {
        dbg_lo[g] = klo;
        dbg_hi[g] = khi;
        dbg_b[g] = b0;
        dbg_e[g] = e0;
        if (r == 0) dbg_nr[j] = (uint32_t)nr;
      }
    } else {
      slot_begin[2 * g] = (uint32_t)b0;
      slot_count[2 * g] = (uint32_t)(e0 - b0);
      slot_begin[2 * g + 1] = (uint32_t)b1;
      slot_count[2 * g + 1] = (uint32_t)(e1 - b1);
    }
  }
}

// Largest s in [0, nseg) with seg_off[s] <= c, for c < seg_off[nseg]; the
// whole wave searches with 64 probes per step (wave-uniform result).
__device__ __forceinline__ uint64_t wave_segment_of(const uint64_t* __restrict__ seg_off,
                                                    uint64_t nseg, uint64_t c, uint64_t lo) {
  const uint32_t lane = lane_id();
  uint64_t hi = nseg - 1;   // invariant: seg_off[lo] <= c and the answer lies in [lo, hi]
  while (hi - lo >= 64) {
    const uint64_t stride = (hi - lo) / 64 + 1;
    const uint64_t idx = lo + lane * stride;
    const bool le = idx <= hi && seg_off[idx] <= c;
    const uint64_t bal = __ballot(le);
    const uint64_t nlo = lo + (uint64_t)(63 - __clzll(bal)) * stride;
    hi = nlo + stride - 1 < hi ? nlo + stride - 1 : hi;
    lo = nlo;
  }
  const uint64_t idx = lo + lane;
  const bool le = idx <= hi && seg_off[idx] <= c;
  const uint64_t bal = __ballot(le);
  return lo + (uint64_t)(63 - __clzll(bal));
}

// Largest s in [0, nseg) with seg_off[s] <= c (one lane, scalar search).
__device__ __forceinline__ uint64_t segment_of(const uint64_t* __restrict__ seg_off,
                                               uint64_t nseg, uint64_t c) {
  uint64_t lo = 0, len = nseg + 1;
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

// First query index qq in [0, m] with seg_off[qq << ss] >= v (m if none).
__device__ __forceinline__ uint64_t first_query_at(const uint64_t* __restrict__ seg_off,
                                                   uint64_t m, int ss, uint64_t v) {
  uint64_t lo = 0, len = m;
  while (len > 0) {
    const uint64_t h = len >> 1;
    if (seg_off[(lo + h) << ss] < v) {
      lo += h + 1;
      len -= h + 1;
    } else {
      len = h;
    }
  }
  return lo;
}

// A register window over the flat segment list (one segment per query slot):
// lane i holds the end E of segment base + i and its first sorted index B;
// S0 is the start of segment base.  The segment of candidate c is then
// base + #{i : E_i <= c}, found by a binary search over the lanes.
struct SegWindow {
  uint64_t base = 0, S0 = 0, E = 0, last = 0;
  uint32_t B = 0;
  bool valid = false;

  __device__ __forceinline__ void load(const uint64_t* __restrict__ seg_off,
                                       const uint32_t* __restrict__ slot_begin, uint64_t nseg,
                                       uint64_t b) {
    const uint64_t i = b + lane_id();
    base = b;
    E = i < nseg ? seg_off[i + 1] : ~0ull;
    B = i < nseg ? slot_begin[i] : 0u;
    S0 = seg_off[b];
    last = __shfl(E, 63, 64);
    valid = true;
  }

  // Makes the window start at or before the segment of row start r0 (which
  // must be a valid candidate) and cover it.
  __device__ __forceinline__ void ensure(const uint64_t* __restrict__ seg_off,
                                         const uint32_t* __restrict__ slot_begin, uint64_t nseg,
                                         uint64_t r0) {
    if (valid && r0 < last) return;
    const uint64_t lo = valid ? base + 63 : 0;   // seg_off[base + 63] <= last <= r0
    load(seg_off, slot_begin, nseg, wave_segment_of(seg_off, nseg, r0, lo));
  }

  // Segment sc and sorted position pos of candidate c of the row starting
  // at r0 (wave-wide call; inactive lanes get unspecified values).
  __device__ __forceinline__ void locate(const uint64_t* __restrict__ seg_off,
                                         const uint32_t* __restrict__ slot_begin, uint64_t nseg,
                                         uint64_t r0, uint64_t c, bool active, uint64_t& sc,
                                         uint64_t& pos) const {
    const uint32_t lane = lane_id();
    const uint32_t rel = E <= r0 ? 0u : (E - r0 >= 64 ? 64u : (uint32_t)(E - r0));
    uint32_t k = 0;
#pragma unroll
    for (uint32_t bstep = 32; bstep >= 1; bstep >>= 1) {
      const uint32_t v = (uint32_t)__shfl((int)rel, (int)(k + bstep - 1), 64);
      if (v <= lane) k += bstep;
    }
    const uint32_t lastrel = (uint32_t)__shfl((int)rel, 63, 64);
    if (k == 63 && lastrel <= lane) k = 64;
    const uint64_t e_prev = __shfl(E, (int)(k == 0 ? 0 : (k > 63 ? 63 : k - 1)), 64);
    const uint32_t b_k = (uint32_t)__shfl((int)B, (int)(k > 63 ? 63 : k), 64);
    sc = base + k;
    uint64_t sstart = k == 0 ? S0 : e_prev;
    uint32_t sb = b_k;
    if (k == 64 && active) {   // more than 64 segments end inside this row (rare)
      sc = segment_of(seg_off, nseg, c);
      sstart = seg_off[sc];
      sb = slot_begin[sc];
    }
    pos = (uint64_t)sb + (c - sstart);
  }
};

constexpr int kRows = 8;                                  // rows of 64 per iteration
constexpr int kIters = 2;                                 // iterations per wave
constexpr int kTileRows = 4 * kRows * kIters;             // 64 rows per tile
static_assert(kCompactTile == (uint64_t)kTileRows * kWave, "tile shape");

// Pass 1: exact test of every candidate; per 64-candidate row, the mask of
// accepted lanes, and per tile the number of accepted candidates.
__global__ __launch_bounds__(256) void compact_test(
    const double2* __restrict__ q, const double* __restrict__ delta, uint64_t m,
    const double2* __restrict__ pts, uint64_t npts, const uint64_t* __restrict__ seg_off,
    const uint32_t* __restrict__ slot_begin, int ss, uint64_t total_cand, uint64_t chunk_base,
    uint64_t* __restrict__ masks, uint32_t* __restrict__ tile_hits, uint32_t* counters) {
  __shared__ uint32_t s_cnt[4];
  const uint32_t tid = threadIdx.x, w = tid >> 6, lane = tid & 63;
  const uint64_t tile = blockIdx.x;
  const uint64_t tile_start = chunk_base + tile * kCompactTile;
  const uint64_t nseg = m << ss;
  SegWindow win;
  uint32_t cnt = 0;
  for (int it = 0; it < kIters; ++it) {
    const uint64_t c0 = tile_start + (uint64_t)(w * kIters + it) * (kRows * kWave);
    uint32_t pos[kRows], qix[kRows];
    uint32_t act = 0;
#pragma unroll
    for (int jr = 0; jr < kRows; ++jr) {
      pos[jr] = 0;
      qix[jr] = 0;
      const uint64_t r0 = c0 + (uint64_t)jr * kWave;
      if (r0 >= total_cand) continue;   // wave-uniform
      const uint64_t c = r0 + lane;
      const bool active = c < total_cand;
      win.ensure(seg_off, slot_begin, nseg, r0);
      uint64_t sc, p64;
      win.locate(seg_off, slot_begin, nseg, r0, c, active, sc, p64);
      if (active) {
        if (p64 < npts && (sc >> ss) < m) {
          pos[jr] = (uint32_t)p64;
          qix[jr] = (uint32_t)(sc >> ss);
          act |= 1u << jr;
        } else {
          atomicOr(&counters[2], kErrInternal);
        }
      }
    }
    double2 pv[kRows], qv[kRows];
    double dv[kRows];
#pragma unroll
    for (int jr = 0; jr < kRows; ++jr) {
      if ((act >> jr) & 1u) {
        pv[jr] = pts[pos[jr]];
        qv[jr] = q[qix[jr]];
        dv[jr] = delta[qix[jr]];
      }
    }
#pragma unroll
    for (int jr = 0; jr < kRows; ++jr) {
      const bool hit =
          ((act >> jr) & 1u) && within(pv[jr].x, pv[jr].y, qv[jr].x, qv[jr].y, dv[jr]);
      const uint64_t bal = __ballot(hit);
      cnt += (uint32_t)__popcll(bal);
      if (lane == 0) masks[tile * kTileRows + (uint64_t)(w * kIters + it) * kRows + jr] = bal;
    }
  }
  if (lane == 0) s_cnt[w] = cnt;
  __syncthreads();
  if (tid == 0) tile_hits[tile] = s_cnt[0] + s_cnt[1] + s_cnt[2] + s_cnt[3];
}

// Pass 2: the ids of the accepted candidates, in candidate order, at the
// tile's offset; and the CSR offsets of the queries whose candidates start in
// the tile (for the last tile also of the trailing queries without any).
__global__ __launch_bounds__(256) void compact_write(
    const uint32_t* __restrict__ ids, uint64_t npts, uint64_t m,
    const uint64_t* __restrict__ seg_off, const uint32_t* __restrict__ slot_begin, int ss,
    uint64_t total_cand, uint64_t chunk_base, const uint64_t* __restrict__ masks,
    const uint64_t* __restrict__ tile_off, uint64_t* __restrict__ offsets,
    uint32_t* __restrict__ out_ids, uint64_t cap, uint32_t* counters) {
  __shared__ uint64_t s_mask[kTileRows];
  __shared__ uint32_t s_pre[kTileRows + 1];
  __shared__ uint64_t s_qrange[2];
  const uint32_t tid = threadIdx.x, w = tid >> 6, lane = tid & 63;
  const uint64_t tile = blockIdx.x;
  const uint64_t tile_start = chunk_base + tile * kCompactTile;
  const uint64_t nseg = m << ss;
  if (tid < kTileRows) s_mask[tid] = masks[tile * kTileRows + tid];
  if (tid == 64) s_qrange[0] = first_query_at(seg_off, m, ss, tile_start);
  if (tid == 128) {
    const uint64_t tile_end = tile_start + kCompactTile;
    s_qrange[1] = tile_end >= total_cand ? m : first_query_at(seg_off, m, ss, tile_end);
  }
  __syncthreads();
  if (tid < 64) {   // exclusive scan of the row counts (one wave)
    const uint32_t v = (uint32_t)__popcll(s_mask[tid]);
    uint32_t x = v;
#pragma unroll
    for (int o = 1; o < 64; o <<= 1) {
      const uint32_t y = __shfl_up(x, o, 64);
      if (lane >= (uint32_t)o) x += y;
    }
    s_pre[tid] = x - v;
    if (tid == 63) s_pre[kTileRows] = x;
  }
  __syncthreads();
  const uint64_t prefix = tile_off[tile];
  const uint64_t below = lanemask_lt();

  SegWindow win;
  for (int it = 0; it < kIters; ++it) {
    // Locate the accepted candidates of eight rows, then load their ids
    // together, then store them.
    uint32_t pos[kRows];
    uint64_t opos[kRows];
    uint32_t act = 0;
#pragma unroll
    for (int jr = 0; jr < kRows; ++jr) {
      pos[jr] = 0;
      opos[jr] = 0;
      const int ri = (w * kIters + it) * kRows + jr;
      const uint64_t mask = s_mask[ri];
      if (mask == 0) continue;   // wave-uniform
      const uint64_t r0 = tile_start + (uint64_t)ri * kWave;
      const uint64_t c = r0 + lane;
      const bool hit = (mask >> lane) & 1ull;
      win.ensure(seg_off, slot_begin, nseg, r0);
      uint64_t sc, p64;
      win.locate(seg_off, slot_begin, nseg, r0, c, hit, sc, p64);
      if (hit) {
        if (p64 < npts) {
          pos[jr] = (uint32_t)p64;
          opos[jr] = prefix + s_pre[ri] + (uint64_t)__popcll(mask & below);
          act |= 1u << jr;
        } else {
          atomicOr(&counters[2], kErrInternal);
        }
      }
    }
    uint32_t idv[kRows];
#pragma unroll
    for (int jr = 0; jr < kRows; ++jr) idv[jr] = ((act >> jr) & 1u) ? ids[pos[jr]] : 0u;
#pragma unroll
    for (int jr = 0; jr < kRows; ++jr)
      if (((act >> jr) & 1u) && opos[jr] < cap) out_ids[opos[jr]] = idv[jr];
  }

  const uint64_t valid = total_cand - tile_start < kCompactTile ? total_cand - tile_start
                                                                : kCompactTile;
  for (uint64_t qq = s_qrange[0] + tid; qq < s_qrange[1]; qq += 256) {
    const uint64_t x = seg_off[qq << ss] - tile_start;
    uint64_t hb;
    if (x >= valid) {
      hb = s_pre[kTileRows];
    } else {
      const uint32_t r = (uint32_t)(x >> 6), bpos = (uint32_t)(x & 63);
      hb = s_pre[r] + (uint64_t)__popcll(s_mask[r] & ((1ull << bpos) - 1));
    }
    offsets[qq] = prefix + hb;
  }
  if (tid == 0 && tile_start + valid == total_cand) offsets[m] = prefix + s_pre[kTileRows];
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
  const uint64_t nseg = 8 * m;   // room for the refined layout (eight slots per query)
  return align256(nseg * 4) * 2 + align256((nseg + 1) * 8) + scan_scratch_bytes(nseg) +
         align256(64);
}

void query_scratch_carve(void* base, uint64_t m, QueryScratch* qs) {
  const uint64_t nseg = 8 * m;
  char* p = (char*)base;
  qs->slot_begin = (uint32_t*)p;  p += align256(nseg * 4);
  qs->slot_count = (uint32_t*)p;  p += align256(nseg * 4);
  qs->seg_off = (uint64_t*)p;     p += align256((nseg + 1) * 8);
  qs->scan_tmp = (uint64_t*)p;    p += scan_scratch_bytes(nseg);
  qs->counters = (uint32_t*)p;
  qs->ss = 2;
}

size_t compact_scratch_bytes(uint64_t total_cand) {
  uint64_t tiles = (total_cand + kCompactTile - 1) / kCompactTile;
  if (tiles > kCompactChunkTiles) tiles = kCompactChunkTiles;
  if (tiles == 0) tiles = 1;
  return align256(tiles * kTileRows * 8) + align256(tiles * 4) + 2 * align256((tiles + 1) * 8) +
         scan_scratch_bytes(tiles);
}

hipError_t launch_ranges(const double* q, const double* delta, uint64_t m, const uint64_t* keys,
                         uint64_t n, int curve, bool refine, uint32_t refine_min, QueryScratch& qs,
                         uint64_t* dbg_lo, uint64_t* dbg_hi, uint64_t* dbg_b, uint64_t* dbg_e,
                         uint32_t* dbg_nr, hipStream_t s) {
  if (m == 0) return hipSuccess;
  const uint32_t blocks = (uint32_t)((4 * m + 255) / 256);
  hipError_t e;
  if ((e = fill_u32(qs.counters, 0, 16, s)) != hipSuccess) return e;
  if (dbg_lo) refine = false;   // the inspected ranges are the method's merged ranges
  qs.ss = refine ? 3 : 2;
  {
    ProfScope ps("ranges_search", s);
#define SFC_RANGES(C, R)                                                                       \
  ranges_search<C, R><<<blocks, 256, 0, s>>>((const double2*)q, delta, m, keys, n, refine_min, \
                                             qs.slot_begin, qs.slot_count, qs.counters, dbg_lo, \
                                             dbg_hi, dbg_b, dbg_e, dbg_nr)
    if (curve == SFC_CURVE_HILBERT) {
      if (refine) SFC_RANGES(SFC_CURVE_HILBERT, true);
      else SFC_RANGES(SFC_CURVE_HILBERT, false);
    } else {
      if (refine) SFC_RANGES(SFC_CURVE_MORTON, true);
      else SFC_RANGES(SFC_CURVE_MORTON, false);
    }
#undef SFC_RANGES
    if ((e = hipGetLastError()) != hipSuccess) return e;
  }
  return scan_excl(qs.slot_count, qs.seg_off, m << qs.ss, nullptr, qs.scan_tmp, s);
}

hipError_t launch_compact(const double* q, const double* delta, uint64_t m, const double* pts,
                          const uint32_t* ids, uint64_t npts, const QueryScratch& qs,
                          uint64_t total_cand, void* cscratch, uint64_t* offsets,
                          uint32_t* out_ids, uint64_t cap, hipStream_t s) {
  hipError_t e;
  if (m == 0) return fill_u64(offsets, 0, 1, s);
  if (total_cand == 0) return fill_u64(offsets, 0, m + 1, s);
  const uint64_t tiles = (total_cand + kCompactTile - 1) / kCompactTile;
  const uint64_t ch = tiles < kCompactChunkTiles ? tiles : kCompactChunkTiles;
  char* p = (char*)cscratch;
  uint64_t* masks = (uint64_t*)p;     p += align256(ch * kTileRows * 8);
  uint32_t* hits = (uint32_t*)p;      p += align256(ch * 4);
  uint64_t* toff[2];
  toff[0] = (uint64_t*)p;             p += align256((ch + 1) * 8);
  toff[1] = (uint64_t*)p;             p += align256((ch + 1) * 8);
  uint64_t* stmp = (uint64_t*)p;
  const uint64_t* carry = nullptr;
  int buf = 0;
  for (uint64_t t0 = 0; t0 < tiles; t0 += kCompactChunkTiles, buf ^= 1) {
    const uint64_t nt = tiles - t0 < kCompactChunkTiles ? tiles - t0 : kCompactChunkTiles;
    const uint64_t cbase = t0 * kCompactTile;
    {
      ProfScope ps("compact_test", s);
      compact_test<<<(uint32_t)nt, 256, 0, s>>>((const double2*)q, delta, m, (const double2*)pts,
                                                npts, qs.seg_off, qs.slot_begin, qs.ss,
                                                total_cand, cbase, masks, hits, qs.counters);
      if ((e = hipGetLastError()) != hipSuccess) return e;
    }
    if ((e = scan_excl(hits, toff[buf], nt, carry, stmp, s)) != hipSuccess) return e;
    {
      ProfScope ps("compact_write", s);
      compact_write<<<(uint32_t)nt, 256, 0, s>>>(ids, npts, m, qs.seg_off, qs.slot_begin, qs.ss,
                                                 total_cand, cbase, masks, toff[buf], offsets,
                                                 out_ids, cap, qs.counters);
      if ((e = hipGetLastError()) != hipSuccess) return e;
    }
    carry = toff[buf] + nt;
  }
  return hipSuccess;
}

}  // namespace sfc
