// The per-lane pieces of the search (Alg. 1 with the Observation and the
// definition of cells(Q)): a query's widened box, its cells and their key
// intervals, the searches of an interval, and the helpers of the refinement
// of a crowded cell; query_lane.inc puts them together for one lane.  Plain
// per-lane code with no cross-lane operation, so that the same source also
// compiles as host C++ (a C++ compiler other than the HIP one sees
// __device__ and __forceinline__ as plain inline functions), where the tests
// run it under the address and undefined-behaviour sanitizers against the
// oracle.
#pragma once

#include <hip/hip_runtime.h>

#include <cstdint>

#include "common.h"
#include "curve.h"
#include "internal.h"
#include "learned.h"
#include "stree.h"

namespace sfc {

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

// The square-window test (the experiments' queries, Sec. 4): the closed
// axis-parallel square of half side d around q, in binary64.  The window is
// its own bounding square, so the cells and key ranges are those of the
// Euclidean query of radius d.
__device__ __forceinline__ bool within_window(double px, double py, double qx, double qy,
                                              double d) {
#pragma clang fp contract(off)
  const double dx = px - qx;
  const double dy = py - qy;
  return fabs(dx) <= d && fabs(dy) <= d;
}

__device__ __forceinline__ bool finite64(double v) { return __builtin_isfinite(v); }

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

// Early termination (Sec. 2.2, "Early termination"): one occupancy bit per
// quadtree node down to depth kOccDepth, nodes of depth k numbered by the
// top 2k bits of their keys (the prefix property of the curve) after the
// (4^k - 1) / 3 nodes of the shallower levels.  A level-L cell is a node of
// depth 32 - L; a deeper cell is checked through its depth-kOccDepth
// ancestor.  A cell whose bit is clear holds no point and is skipped, so the
// reported set never changes.
__device__ __forceinline__ bool cell_occupied(const uint32_t* __restrict__ occ, int L,
                                              uint64_t key) {
  const int k = 32 - L;
  const int kk = k < kOccDepth ? k : kOccDepth;
  const uint64_t node = occ_level_offset(kk) + (kk == 0 ? 0 : key >> (64 - 2 * kk));
  return (occ[node >> 5] >> (node & 31)) & 1u;
}

// Merged key intervals of cells(Q) for query (qx, qy, d); returns their
// number (0..4), ascending and non-adjacent.  occ (may be null): skip cells
// that hold no point (counted in *pruned).
template <int CURVE>
__device__ int query_ranges(const uint16_t* lut, double qx, double qy, double d, uint64_t lo[4],
                            uint64_t hi[4], const uint32_t* occ, uint32_t* pruned) {
  int64_t lx, hx, ly, hy;
  if (!axis_box(qx, d, lx, hx) || !axis_box(qy, d, ly, hy)) return 0;
  const uint64_t sx = (uint64_t)(hx - lx + 1), sy = (uint64_t)(hy - ly + 1);
  const uint64_t side = sx > sy ? sx : sy;
  const int L = side <= 1 ? 0 : 64 - __builtin_clzll(side - 1);   // ceil(log2 side)
  if (L >= 32) {
    if (occ && !cell_occupied(occ, 32, 0)) {
      ++*pruned;
      return 0;
    }
    lo[0] = 0;
    hi[0] = ~0ull;
    return 1;
  }
  const uint64_t span = (1ull << (2 * L)) - 1;
  const uint32_t cx0 = (uint32_t)(lx >> L), cx1 = (uint32_t)(hx >> L);
  const uint32_t cy0 = (uint32_t)(ly >> L), cy1 = (uint32_t)(hy >> L);
  int k = 0;
  // Offsets within the box (at most one cell per axis past the first): a
  // coordinate loop ending at cx1 inclusive would wrap at 2^32 - 1, the
  // single cell of a box clamped to the last grid column and row.
  for (uint32_t ax = 0; ax <= cx1 - cx0; ++ax) {
    for (uint32_t ay = 0; ay <= cy1 - cy0; ++ay) {
      const uint32_t cx = cx0 + ax, cy = cy0 + ay;
      const uint64_t key = cell_key<CURVE>(lut, cx << L, cy << L) & ~span;
      if (occ && !cell_occupied(occ, L, key)) {
        ++*pruned;
        continue;
      }
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

// For each of K key intervals [klo[i], khi[i]] whose use flag is set:
// b[i] = first index with keys[idx] >= klo[i], e[i] = first index with
// keys[idx] > khi[i], over keys[0, n) (chains with use[i] false hold no
// result; use[0] must be set).  Every chain keeps only its base and halves one shared length
// (the answer stays in [base, base + len]), so all chains, and all lanes
// that search arrays of one size, probe in lockstep.  All chains start at
// one base and keep sharing it while each probe lies below every key of the
// intervals (all move) or above every key (none moves): such a step takes
// one load and one pair of compares for all.  From the step at which they
// part, each chain loads its own probe, all of them before any compare.
// I is the index type (32 bits whenever n allows: fewer instructions per
// step).
template <typename I, int K>
__device__ __forceinline__ void search_lockstep_t(const uint64_t* __restrict__ keys, I n,
                                                  const uint64_t (&klo)[K],
                                                  const uint64_t (&khi)[K],
                                                  const bool (&use)[K], uint64_t (&ob)[K],
                                                  uint64_t (&oe)[K]) {
  uint64_t alo = ~0ull, ahi = 0;   // the keys' span over the used intervals
#pragma unroll
  for (int i = 0; i < K; ++i) {
    if (use[i]) {
      const uint64_t l = klo[i] < khi[i] ? klo[i] : khi[i];
      const uint64_t h = klo[i] < khi[i] ? khi[i] : klo[i];
      alo = l < alo ? l : alo;
      ahi = h > ahi ? h : ahi;
    }
  }
  I b[K], e[K];
#pragma unroll
  for (int i = 0; i < K; ++i) {
    b[i] = 0;
    e[i] = 0;
  }
  if (n != 0) {
    I len = n;
    bool shared = true;
    for (;;) {
      const I half = len >> 1;   // 0 at the last step: probe the base itself
      const I step = len > 1 ? half : 1;
      const uint64_t v0 = keys[b[0] + half];
      uint64_t vb[K], ve[K];
#pragma unroll
      for (int i = 0; i < K; ++i) {
        vb[i] = v0;
        ve[i] = v0;
      }
      if (!shared) {
#pragma unroll
        for (int i = 0; i < K; ++i) {
          if (use[i]) {
            if (i > 0) vb[i] = keys[b[i] + half];
            ve[i] = keys[e[i] + half];
          }
        }
      }
      if (shared) {
        const bool below = v0 < alo;
        if (below || v0 > ahi) {
          b[0] += below ? step : 0;
        } else {
          // The chains part at this probe: each takes its own side of it.
          const I base = b[0];
#pragma unroll
          for (int i = 0; i < K; ++i) {
            b[i] = base + (v0 < klo[i] ? step : 0);
            e[i] = base + (v0 <= khi[i] ? step : 0);
          }
          shared = false;
        }
      } else {
#pragma unroll
        for (int i = 0; i < K; ++i) {
          if (use[i]) {
            b[i] += vb[i] < klo[i] ? step : 0;
            e[i] += ve[i] <= khi[i] ? step : 0;
          }
        }
      }
      if (len == 1) break;
      len -= half;
    }
    if (shared) {
#pragma unroll
      for (int i = 0; i < K; ++i) {
        b[i] = b[0];
        e[i] = b[0];
      }
    }
  }
#pragma unroll
  for (int i = 0; i < K; ++i) {
    ob[i] = b[i];
    oe[i] = e[i];
  }
}

template <int K>
__device__ __forceinline__ void search_lockstep(const uint64_t* __restrict__ keys, uint64_t n,
                                                const uint64_t (&klo)[K],
                                                const uint64_t (&khi)[K], const bool (&use)[K],
                                                uint64_t (&b)[K], uint64_t (&e)[K]) {
  if (n <= 0xFFFFFFFFull)
    search_lockstep_t<uint32_t, K>(keys, (uint32_t)n, klo, khi, use, b, e);
  else
    search_lockstep_t<uint64_t, K>(keys, n, klo, khi, use, b, e);
}

// b = first index with keys[i] >= klo; e = first index with keys[i] > khi.
__device__ __forceinline__ void search_pair(const uint64_t* __restrict__ keys, uint64_t n,
                                            uint64_t klo, uint64_t khi, uint64_t& b,
                                            uint64_t& e) {
  const uint64_t kl[1] = {klo}, kh[1] = {khi};
  const bool use[1] = {true};
  uint64_t bb[1], ee[1];
  search_lockstep<1>(keys, n, kl, kh, use, bb, ee);
  b = bb[0];
  e = ee[0];
}

// Cells of cells(Q) for the widened box of (qx, qy, d), unmerged and sorted
// by key: cell k covers keys [lo[k], hi[k]] and grid cells
// [cx[k] << L, (cx[k] + 1) << L) x [cy[k] << L, (cy[k] + 1) << L).  Returns the
// number of cells (0..4); *L receives the level, box the widened box.
template <int CURVE>
__device__ int query_cells(const uint16_t* lut, double qx, double qy, double d, uint64_t lo[4],
                           uint64_t hi[4], uint32_t cx[4], uint32_t cy[4], int* Lout,
                           int64_t box[4], const uint32_t* occ, uint32_t* pruned) {
  int64_t lx, hx, ly, hy;
  if (!axis_box(qx, d, lx, hx) || !axis_box(qy, d, ly, hy)) return 0;
  box[0] = lx;
  box[1] = hx;
  box[2] = ly;
  box[3] = hy;
  const uint64_t sx = (uint64_t)(hx - lx + 1), sy = (uint64_t)(hy - ly + 1);
  const uint64_t side = sx > sy ? sx : sy;
  const int L = side <= 1 ? 0 : 64 - __builtin_clzll(side - 1);
  *Lout = L;
  if (L >= 32) {
    if (occ && !cell_occupied(occ, 32, 0)) {
      ++*pruned;
      return 0;
    }
    lo[0] = 0;
    hi[0] = ~0ull;
    cx[0] = cy[0] = 0;
    return 1;
  }
  const uint64_t span = (1ull << (2 * L)) - 1;
  const uint32_t x0 = (uint32_t)(lx >> L), y0 = (uint32_t)(ly >> L);
  const uint32_t nx = (uint32_t)(hx >> L) - x0, ny = (uint32_t)(hy >> L) - y0;
  // The at most 2 x 2 cells at offsets (i >> 1, i & 1) within the box (no
  // coordinate loop that could wrap at 2^32 - 1), absent or pruned ones
  // keyed 2^64 - 1, then sorted by a fixed network of compare-exchanges on
  // (key, offset index): every array index is static, so the cells stay in
  // registers.  A present key equals 2^64 - 1 only at level 0, where the box
  // is one cell (index 0) and no exchange moves it on a tie.
  uint64_t key[4];
  uint32_t id[4];
  int k = 0;
#pragma unroll
  for (int i = 0; i < 4; ++i) {
    id[i] = (uint32_t)i;
    key[i] = ~0ull;
    if ((uint32_t)(i >> 1) <= nx && (uint32_t)(i & 1) <= ny) {
      const uint64_t kk = cell_key<CURVE>(lut, (x0 + (uint32_t)(i >> 1)) << L,
                                          (y0 + (uint32_t)(i & 1)) << L) & ~span;
      if (occ && !cell_occupied(occ, L, kk)) {
        ++*pruned;
      } else {
        key[i] = kk;
        ++k;
      }
    }
  }
  constexpr int kNet[5][2] = {{0, 1}, {2, 3}, {0, 2}, {1, 3}, {1, 2}};
#pragma unroll
  for (int c = 0; c < 5; ++c) {
    const int a = kNet[c][0], b = kNet[c][1];
    const bool sw = key[a] > key[b];
    const uint64_t ka = key[a], kb = key[b];
    const uint32_t ia = id[a], ib = id[b];
    key[a] = sw ? kb : ka;
    key[b] = sw ? ka : kb;
    id[a] = sw ? ib : ia;
    id[b] = sw ? ia : ib;
  }
#pragma unroll
  for (int i = 0; i < 4; ++i) {
    lo[i] = key[i];
    hi[i] = key[i] | span;
    cx[i] = x0 + (id[i] >> 1);
    cy[i] = y0 + (id[i] & 1u);
  }
  return k;
}

// Index range [b, e) of the key interval [klo, khi]: SEARCH 0 two binary
// searches, 1 the learned index (whose lower bounds are verified and fall
// back to binary search, so the result is the same; *fb counts the
// fallbacks), 2 the static search tree.
template <int SEARCH>
__device__ __forceinline__ void find_range(const uint64_t* __restrict__ keys, uint64_t n,
                                           const LearnedView& lv, const StreeView& sv,
                                           uint64_t klo, uint64_t khi, uint64_t& b, uint64_t& e,
                                           uint32_t& fb) {
  if (SEARCH == 0) {
    search_pair(keys, n, klo, khi, b, e);
    return;
  }
  if (SEARCH == 2) {
    stree_range(sv, klo, khi, b, e);
    return;
  }
  // khi = 2^64 - 1 has no successor key: its bound is n, and the second
  // chain then searches klo again (cheaper than a divergent branch).
  const uint64_t k2[2] = {klo, khi == ~0ull ? klo : khi + 1};
  uint64_t r2[2];
  fb += learned_lower_bound_pair(keys, n, lv, k2, r2);
  b = r2[0];
  e = khi == ~0ull ? n : r2[1];
}

// Hilbert frame (as in hilbert_key_lut: bit 0 axes exchanged, bit 1 both
// complemented) of the cell whose key prefix holds `digits` digits: digit 0
// exchanges the axes and digit 3 exchanges and complements them, and frames
// compose by xor, so the frame is the parity of the count of digits 0 or 3
// and the parity of the count of digits 3.
__device__ __forceinline__ uint32_t hilbert_frame(uint64_t prefix, int digits) {
  const uint64_t lowbits = 0x5555555555555555ull & ((1ull << (2 * digits)) - 1);
  const uint32_t c03 = (uint32_t)__builtin_popcountll(~(prefix ^ (prefix >> 1)) & lowbits) & 1u;
  const uint32_t c3 = (uint32_t)__builtin_popcountll(prefix & (prefix >> 1) & lowbits) & 1u;
  return c03 | (c3 << 1);
}

// Rank along the curve of sub-cell (a, b) (offsets in cells D levels down,
// D = 1 or 2) within a cell of Hilbert frame f.
template <int CURVE>
__device__ __forceinline__ uint32_t sub_rank(const uint16_t* lut, uint32_t f, uint32_t a,
                                             uint32_t b, int D) {
  if (CURVE == SFC_CURVE_HILBERT) {
    const uint32_t sh = 4 - D;   // the offsets as the top bits of 4-level nibbles
    return (lut[(f << 8) | ((a << sh) << 4) | (b << sh)] & 0xFFu) >> (8 - 2 * D);
  }
  return D == 2 ? (a & 1u) | ((b & 1u) << 1) | ((a >> 1) << 2) | ((b >> 1) << 3) : a | (b << 1);
}

// The refinement of a crowded cell of cells(Q) (level L, grid cell (cx, cy),
// keys from lo): its sub-cells D levels down (D = 2, or 1 at level 1) that
// meet the widened box, and with the Euclidean metric the disc, as a mask
// over their order along the curve.  kind -1: nothing to refine (level 0 or
// 32, or every sub-cell kept); 0: no sub-cell kept, no point of the cell can
// be reported; 1 or 2: the kept sub-cells as that many key runs [lo0, hi0],
// [lo1, hi1] (consecutive sub-cells in key order; beyond two runs the gaps
// other than the widest are closed).  Unused runs repeat the cell's keys.
struct CellRuns {
  int kind;
  uint64_t lo0, hi0, lo1, hi1;
};

template <int CURVE>
__device__ __forceinline__ CellRuns cell_runs(const uint16_t* lut, uint64_t lo, uint64_t hi,
                                              uint32_t cx, uint32_t cy, int L,
                                              const int64_t (&box)[4], bool ball, double qx,
                                              double qy, double d) {
  CellRuns cr{-1, lo, hi, lo, hi};
  if (L < 1 || L >= 32) return cr;
  const int D = L >= 2 ? 2 : 1;
  const int Ls = L - D;
  const uint32_t per = 1u << D;
  const uint32_t f = CURVE == SFC_CURVE_HILBERT ? hilbert_frame(lo >> (2 * L), 32 - L) : 0u;
  // A sub-cell meets the box when its column and its row do.  With the
  // Euclidean metric it is dropped when its distance from the centre,
  // squared, exceeds d^2 by a relative 2^-40 (far beyond the few units in
  // the last place by which the exact test's binary64 arithmetic can err);
  // that distance is the column's and the row's, each taken once.  Radii
  // below 2^-400 (whose squares approach the subnormal range) keep every
  // sub-cell.
  const bool disc = ball && d >= 0x1p-400;
  const double s = 0x1p-32;
  const double lim = d * d * (1.0 + 0x1p-40);
  uint32_t colm = 0, rowm = 0;
  double ex2[4], ey2[4];
#pragma unroll
  for (uint32_t a = 0; a < 4; ++a) {
    ex2[a] = 0.0;
    ey2[a] = 0.0;
    if (a < per) {
      const int64_t x0 = (int64_t)(((uint64_t)cx * per + a) << Ls);
      const int64_t y0 = (int64_t)(((uint64_t)cy * per + a) << Ls);
      const int64_t x1 = x0 + ((int64_t)1 << Ls), y1 = y0 + ((int64_t)1 << Ls);
      colm |= (uint32_t)!(x1 - 1 < box[0] || x0 > box[1]) << a;
      rowm |= (uint32_t)!(y1 - 1 < box[2] || y0 > box[3]) << a;
      const double ex = fmax(0.0, fmax((double)x0 * s - qx, qx - (double)x1 * s));
      const double ey = fmax(0.0, fmax((double)y0 * s - qy, qy - (double)y1 * s));
      ex2[a] = ex * ex;
      ey2[a] = ey * ey;
    }
  }
  uint32_t mask = 0;
#pragma unroll
  for (uint32_t a = 0; a < 4; ++a) {
#pragma unroll
    for (uint32_t bb = 0; bb < 4; ++bb) {
      if (!((colm >> a) & (rowm >> bb) & 1u)) continue;
      if (disc && ex2[a] + ey2[bb] > lim) continue;
      mask |= 1u << sub_rank<CURVE>(lut, f, a, bb, D);
    }
  }
  const uint32_t full = D == 2 ? 0xFFFFu : 0xFu;
  if (mask == full) return cr;
  if (mask == 0) {
    cr.kind = 0;
    return cr;
  }
  const int first = __builtin_ctz(mask), last = 31 - __builtin_clz(mask);
  int gap_at = 0, gap_len = 0;   // widest run of dropped sub-cells inside
  for (int i = first; i <= last;) {
    if ((mask >> i) & 1u) {
      ++i;
      continue;
    }
    int j = i;
    while (!((mask >> j) & 1u)) ++j;
    if (j - i > gap_len) {
      gap_len = j - i;
      gap_at = i;
    }
    i = j;
  }
  const int sh = 2 * Ls;
  const int end0 = gap_len ? gap_at - 1 : last;
  cr.kind = gap_len ? 2 : 1;
  cr.lo0 = lo | ((uint64_t)first << sh);
  cr.hi0 = lo | ((((uint64_t)end0 + 1) << sh) - 1);
  if (gap_len) {
    cr.lo1 = lo | ((uint64_t)(gap_at + gap_len) << sh);
    cr.hi1 = lo | ((((uint64_t)last + 1) << sh) - 1);
  }
  return cr;
}

}  // namespace sfc
