// Batched distance queries (Alg. 1 over cells(Q); Problem Statement).
//
//   ranges_search  one lane per (query, slot), four slots per query.  Every
//                  lane of a query derives the widened integer box, the
//                  level l = ceil(log2 side), the at most four level-l cells
//                  meeting the box and their merged key intervals (the
//                  Observation gives each cell's interval); slot r then runs
//                  the two searches of interval r over the sorted keys
//                  (binary search or the learned index), optionally split
//                  once into the cell's children that meet the box.
//   cells_pack     with early termination: the cells whose quadtree node
//                  holds a point, as a dense (query, cell) work list, so the
//                  search spends lanes only on them.
//   scan           candidate rows of every slot -> row offsets.
//   expand_rows    rows -> (slot, first candidate) tiles.
//   compact_test   a block tests its tiles' candidates (64-lane rows) with
//                  the exact distance test and counts the hits per tile;
//                  the hit counts are scanned on the device.
//   compact_write  the same tiles again, one lane per reported id: the ids at
//                  the scanned positions, in candidate order, and every
//                  row's output position.
//   query_offsets  the CSR offset of every query, from its first row.
#include <hip/hip_runtime.h>

#include <atomic>

#include <cstdlib>

#include "common.h"
#include "curve.h"
#include "internal.h"
#include "learned.h"
#include "stree.h"
#include "query_lane.h"

namespace sfc {

namespace {

// One lane per (query, slot): four slots per query (the method's ranges),
// or eight (REFINE: two runs per cell of cells(Q)); the lane's work is the
// body in query_lane.inc.
// At least five waves per SIMD (at most 102 registers): the chains of
// dependent probes need waves in flight.  The binary-search variants take 62
// registers (eight waves) now that query_cells indexes its arrays statically;
// the learned-index variants take 92.
template <int CURVE, bool REFINE, int SEARCH>
__global__ __launch_bounds__(256) __attribute__((amdgpu_waves_per_eu(5))) void ranges_search(
    const double2* __restrict__ q, const double* __restrict__ delta, uint64_t m,
    const uint64_t* __restrict__ keys, uint64_t n, LearnedView lv, StreeView sv,
    uint32_t refine_min, bool ball, const uint32_t* __restrict__ occ,
    const uint64_t* __restrict__ pairs,
    const uint64_t* __restrict__ pair_total, const uint32_t* __restrict__ qset,
    const uint64_t* __restrict__ set_off, uint32_t n_sets, uint32_t* __restrict__ slot_begin, uint32_t* __restrict__ slot_count,
    uint32_t* __restrict__ slot_rows, uint32_t* counters, unsigned long long* cand_total,
    const uint32_t* __restrict__ perm,
    uint64_t* __restrict__ dbg_lo, uint64_t* __restrict__ dbg_hi, uint64_t* __restrict__ dbg_b,
    uint64_t* __restrict__ dbg_e, uint32_t* __restrict__ dbg_nr) {
  constexpr bool LEARNED = SEARCH == 1;
  __shared__ uint16_t lut[CURVE == SFC_CURVE_HILBERT ? 1024 : 1];
  // Blocks past the listed pairs have nothing to do (uniform per block).
  if (pairs && (uint64_t)blockIdx.x * 256 >= *pair_total) return;
  if (CURVE == SFC_CURVE_HILBERT)
    for (int i = threadIdx.x; i < 1024; i += 256) lut[i] = kHilbertLutConst.v[i];
  __syncthreads();
  // Lane -> (query, cell): four lanes per query, or (pairs) one lane per
  // cell that survived early termination, packed densely; idle lanes take
  // j = m.
  const uint64_t g = (uint64_t)blockIdx.x * 256 + threadIdx.x;
  uint64_t j, sidx;
  int r;
  if (pairs) {
    const bool act = g < *pair_total;
    const uint64_t pr = act ? pairs[g] : 0;
    j = act ? pr >> 2 : m;
    r = (int)(pr & 3);
    sidx = pr;
  } else {
    // perm non-null: the queries in curve order, so that the searches of a
    // workgroup meet in the same lines of the key array.
    const uint64_t jj = g >> 2;
    j = perm && jj < m ? perm[jj] : jj;
    r = (int)(g & 3);
    sidx = 4 * j + (uint64_t)r;
  }

  uint64_t b0 = 0, e0 = 0, b1 = 0, e1 = 0, klo = 0, khi = 0;
  int nr = 0;
  bool bad = false;
  uint32_t fb = 0, ends = 0, pruned = 0;
  // With point sets, a query searches only its own set's keys: positions
  // [base, base + nn) of the sorted arrays.
  uint64_t base = 0, nn = n;
  if (j < m && qset) {
    const uint32_t sj = qset[j];
    if (sj >= n_sets) {
      bad = true;
      nn = 0;
    } else {
      base = set_off[sj];
      nn = set_off[sj + 1] - base;
    }
  }
#include "query_lane.inc"
  if (__ballot(bad) != 0 && lane_id() == 0) atomicOr(&counters[2], kErrInvalidQuery);
  // Candidates (and learned-index endpoints and fallbacks) of the block, for
  // the statistics: one device atomic per counter and block (atomics on one
  // address from every wave of the grid serialise).
  __shared__ unsigned long long s_stat[4][4];
  uint64_t wc = (e0 - b0) + (e1 - b1);
  uint32_t wf = fb, we = ends, wp = pruned;
#pragma unroll
  for (int o = 32; o >= 1; o >>= 1) {
    wc += __shfl_xor(wc, o, 64);
    wp += __shfl_xor(wp, o, 64);
    if (LEARNED) {
      wf += __shfl_xor(wf, o, 64);
      we += __shfl_xor(we, o, 64);
    }
  }
  const uint32_t wv = threadIdx.x >> 6;
  if (lane_id() == 0) {
    s_stat[0][wv] = wc;
    s_stat[1][wv] = we;
    s_stat[2][wv] = wf;
    s_stat[3][wv] = wp;
  }
  __syncthreads();
  if (threadIdx.x < 4 && (threadIdx.x == 0 || threadIdx.x == 3 || LEARNED)) {
    const unsigned long long t = s_stat[threadIdx.x][0] + s_stat[threadIdx.x][1] +
                                 s_stat[threadIdx.x][2] + s_stat[threadIdx.x][3];
    if (t) atomicAdd(cand_total + threadIdx.x, t);
  }
  if (j < m) {
    if (!REFINE) {
      slot_begin[sidx] = (uint32_t)b0;
      slot_count[sidx] = (uint32_t)(e0 - b0);
      slot_rows[sidx] = (uint32_t)((e0 - b0 + 63) >> 6);
      if (dbg_lo) {
        dbg_lo[sidx] = klo;
        dbg_hi[sidx] = khi;
        dbg_b[sidx] = b0;
        dbg_e[sidx] = e0;
        if (r == 0) dbg_nr[j] = (uint32_t)nr;
      }
    } else {
      slot_begin[2 * sidx] = (uint32_t)b0;
      slot_count[2 * sidx] = (uint32_t)(e0 - b0);
      slot_rows[2 * sidx] = (uint32_t)((e0 - b0 + 63) >> 6);
      slot_begin[2 * sidx + 1] = (uint32_t)b1;
      slot_count[2 * sidx + 1] = (uint32_t)(e1 - b1);
      slot_rows[2 * sidx + 1] = (uint32_t)((e1 - b1 + 63) >> 6);
    }
  }
}

// ---- three dimensions (d = 3 Morton codes) ------------------------------------

constexpr double kTwo22 = 4194304.0;            // 2^22
constexpr double kTwoM29 = 1.0 / 536870912.0;   // 2^-29

// The d = 3 test: the squares summed left to right, no contraction.
__device__ __forceinline__ bool within3(double px, double py, double pz, double qx, double qy,
                                        double qz, double d) {
#pragma clang fp contract(off)
  const double dx = px - qx;
  const double dy = py - qy;
  const double dz = pz - qz;
  const double t = dx * dx;
  const double u = dy * dy;
  const double v = dz * dz;
  const double s = (t + u) + v;
  return s <= d * d;
}

__device__ __forceinline__ bool within_window3(double px, double py, double pz, double qx,
                                               double qy, double qz, double d) {
#pragma clang fp contract(off)
  const double dx = px - qx;
  const double dy = py - qy;
  const double dz = pz - qz;
  return fabs(dx) <= d && fabs(dy) <= d && fabs(dz) <= d;
}

// One axis of the widened box on the 2^21 grid: w = 1 + floor((|c| + d)
// 2^-29) quanta cover the rounding of the test.
__device__ __forceinline__ bool axis_box3(double c, double d, int64_t& lo, int64_t& hi) {
#pragma clang fp contract(off)
  double wr = __builtin_floor((__builtin_fabs(c) + d) * kTwoM29);
  wr = wr > kTwo22 ? kTwo22 : wr;
  const int64_t w = 1 + (int64_t)wr;
  double a = (c - d) * kTwo21, b = (c + d) * kTwo21;
  a = a < -kTwo22 ? -kTwo22 : (a > kTwo22 ? kTwo22 : a);
  b = b < -kTwo22 ? -kTwo22 : (b > kTwo22 ? kTwo22 : b);
  int64_t l = (int64_t)__builtin_floor(a) - w;
  int64_t h = (int64_t)__builtin_floor(b) + w;
  l = l < 0 ? 0 : l;
  h = h > (int64_t)kMaxCell3 ? (int64_t)kMaxCell3 : h;
  lo = l;
  hi = h;
  return l <= h;
}

// Merged key intervals of the level-l cubes meeting the widened box (at most
// 8), ascending and non-adjacent.
__device__ int query_ranges3(double qx, double qy, double qz, double d, uint64_t lo[8],
                             uint64_t hi[8]) {
  int64_t b[6];
  if (!axis_box3(qx, d, b[0], b[1]) || !axis_box3(qy, d, b[2], b[3]) ||
      !axis_box3(qz, d, b[4], b[5]))
    return 0;
  uint64_t side = (uint64_t)(b[1] - b[0] + 1);
  side = (uint64_t)(b[3] - b[2] + 1) > side ? (uint64_t)(b[3] - b[2] + 1) : side;
  side = (uint64_t)(b[5] - b[4] + 1) > side ? (uint64_t)(b[5] - b[4] + 1) : side;
  const int L = side <= 1 ? 0 : 64 - __clzll(side - 1);
  if (L >= 21) {
    lo[0] = 0;
    hi[0] = (1ull << 63) - 1;
    return 1;
  }
  const uint64_t span = (1ull << (3 * L)) - 1;
  int k = 0;
  for (uint32_t cx = (uint32_t)(b[0] >> L); cx <= (uint32_t)(b[1] >> L); ++cx)
    for (uint32_t cy = (uint32_t)(b[2] >> L); cy <= (uint32_t)(b[3] >> L); ++cy)
      for (uint32_t cz = (uint32_t)(b[4] >> L); cz <= (uint32_t)(b[5] >> L); ++cz) {
        const uint64_t key = morton3_key(cx << L, cy << L, cz << L) & ~span;
        int t = k++;
        for (; t > 0 && lo[t - 1] > key; --t) lo[t] = lo[t - 1];
        lo[t] = key;
      }
  int r = 0;
  for (int i = 0; i < k; ++i) {
    if (r > 0 && hi[r - 1] + 1 == lo[i]) {
      hi[r - 1] = lo[i] | span;
    } else {
      lo[r] = lo[i];
      hi[r] = lo[i] | span;
      ++r;
    }
  }
  return r;
}

// The level-l cubes meeting the widened box, unmerged and sorted by key, with
// their coordinates at level l (for the refinement); *L gets l, b the box.
__device__ __forceinline__ void cube_cas(uint64_t* lo, uint32_t* cx, uint32_t* cy, uint32_t* cz,
                                         int i, int j) {
  if (lo[j] < lo[i]) {
    const uint64_t k = lo[i];
    lo[i] = lo[j];
    lo[j] = k;
    uint32_t t = cx[i];
    cx[i] = cx[j];
    cx[j] = t;
    t = cy[i];
    cy[i] = cy[j];
    cy[j] = t;
    t = cz[i];
    cz[i] = cz[j];
    cz[j] = t;
  }
}

__device__ __forceinline__ int query_cubes3(double qx, double qy, double qz, double d,
                                            uint64_t lo[8], uint32_t cx[8], uint32_t cy[8],
                                            uint32_t cz[8], int* L, int64_t b[6]) {
  if (!axis_box3(qx, d, b[0], b[1]) || !axis_box3(qy, d, b[2], b[3]) ||
      !axis_box3(qz, d, b[4], b[5]))
    return 0;
  uint64_t side = (uint64_t)(b[1] - b[0] + 1);
  side = (uint64_t)(b[3] - b[2] + 1) > side ? (uint64_t)(b[3] - b[2] + 1) : side;
  side = (uint64_t)(b[5] - b[4] + 1) > side ? (uint64_t)(b[5] - b[4] + 1) : side;
  const int l = side <= 1 ? 0 : 64 - __clzll(side - 1);
  if (l >= 21) {
    *L = 21;
    lo[0] = 0;
    cx[0] = cy[0] = cz[0] = 0;
    return 1;
  }
  *L = l;
  // A box of side at most 2^l meets at most two level-l cells per axis: the
  // eight candidates (x0 + dx, y0 + dy, z0 + dz), those outside the box keyed
  // past every cube, then sorted by key with a fixed network (Batcher's
  // odd-even merge, 19 exchanges), every array index static so that the
  // arrays stay in registers.
  const uint32_t x0 = (uint32_t)(b[0] >> l), x1 = (uint32_t)(b[1] >> l);
  const uint32_t y0 = (uint32_t)(b[2] >> l), y1 = (uint32_t)(b[3] >> l);
  const uint32_t z0 = (uint32_t)(b[4] >> l), z1 = (uint32_t)(b[5] >> l);
  int k = 0;
#pragma unroll
  for (int c = 0; c < 8; ++c) {
    const uint32_t x = x0 + (c & 1), y = y0 + ((c >> 1) & 1), z = z0 + (c >> 2);
    const bool in = x <= x1 && y <= y1 && z <= z1;
    lo[c] = in ? morton3_key(x << l, y << l, z << l) : ~0ull;
    cx[c] = x;
    cy[c] = y;
    cz[c] = z;
    k += in ? 1 : 0;
  }
  cube_cas(lo, cx, cy, cz, 0, 1); cube_cas(lo, cx, cy, cz, 2, 3);
  cube_cas(lo, cx, cy, cz, 4, 5); cube_cas(lo, cx, cy, cz, 6, 7);
  cube_cas(lo, cx, cy, cz, 0, 2); cube_cas(lo, cx, cy, cz, 1, 3);
  cube_cas(lo, cx, cy, cz, 4, 6); cube_cas(lo, cx, cy, cz, 5, 7);
  cube_cas(lo, cx, cy, cz, 1, 2); cube_cas(lo, cx, cy, cz, 5, 6);
  cube_cas(lo, cx, cy, cz, 0, 4); cube_cas(lo, cx, cy, cz, 1, 5);
  cube_cas(lo, cx, cy, cz, 2, 6); cube_cas(lo, cx, cy, cz, 3, 7);
  cube_cas(lo, cx, cy, cz, 2, 4); cube_cas(lo, cx, cy, cz, 3, 5);
  cube_cas(lo, cx, cy, cz, 1, 2); cube_cas(lo, cx, cy, cz, 3, 4);
  cube_cas(lo, cx, cy, cz, 5, 6);
  return k;
}

// One lane per (query, slot): eight slots per query, each a merged interval
// of the query's cubes.  REFINE: one lane per cube (unmerged); a cube
// holding more than refine_min keys is split once, its children that meet
// the box forming at most four runs of consecutive children in key order
// (four slots per cube, 32 per query), each found by two searches inside the
// cube's index range.  The reported ids and their order do not change.
template <int SEARCH, bool REFINE>
// Five waves per SIMD or more (the cubes sorted by a fixed network, so that
// their arrays stay in registers): 1.71 ms binary, 1.16 ms with the static
// search tree for 2^20 queries over 2^24 keys, against 1.89 and 1.39 ms with
// the arrays in scratch memory.
__global__ __launch_bounds__(256) __attribute__((amdgpu_waves_per_eu(5))) void ranges_search3(
    const double* __restrict__ q, const double* __restrict__ delta, uint64_t m,
    const uint64_t* __restrict__ keys, uint64_t n, LearnedView lv, StreeView sv,
    uint32_t refine_min, uint32_t* __restrict__ slot_begin, uint32_t* __restrict__ slot_count,
    uint32_t* __restrict__ slot_rows, uint32_t* counters, unsigned long long* cand_total) {
  const uint64_t g = (uint64_t)blockIdx.x * 256 + threadIdx.x;
  const uint64_t j = g >> 3;
  const int r = (int)(g & 7);
  uint64_t B[4] = {0, 0, 0, 0}, E[4] = {0, 0, 0, 0};
  uint32_t fb = 0;
  bool bad = false;
  if (j < m) {
    const double qx = q[3 * j], qy = q[3 * j + 1], qz = q[3 * j + 2], d = delta[j];
    if (!(finite64(qx) && finite64(qy) && finite64(qz) && finite64(d) && d >= 0.0)) {
      bad = true;
    } else if (!REFINE) {
      uint64_t lo[8], hi[8];
      const int nr = query_ranges3(qx, qy, qz, d, lo, hi);
      // The lane's range, taken with static indexes (a runtime index into
      // the arrays would put them in scratch memory).
      uint64_t mlo = 0, mhi = 0;
#pragma unroll
      for (int c = 0; c < 8; ++c)
        if (c == r) {
          mlo = lo[c];
          mhi = hi[c];
        }
      if (r < nr) find_range<SEARCH>(keys, n, lv, sv, mlo, mhi, B[0], E[0], fb);
    } else {
      uint64_t lo[8];
      uint32_t cx[8], cy[8], cz[8];
      int64_t b[6];
      int L = 0;
      const int nr = query_cubes3(qx, qy, qz, d, lo, cx, cy, cz, &L, b);
      // The lane's cube, taken with static indexes (a runtime index into the
      // arrays would put them in scratch memory).
      uint64_t mlo = 0;
      uint32_t mx = 0, my = 0, mz = 0;
#pragma unroll
      for (int c = 0; c < 8; ++c)
        if (c == r) {
          mlo = lo[c];
          mx = cx[c];
          my = cy[c];
          mz = cz[c];
        }
      if (r < nr) {
        const uint64_t span = L >= 21 ? (1ull << 63) - 1 : (1ull << (3 * L)) - 1;
        find_range<SEARCH>(keys, n, lv, sv, mlo, mlo | span, B[0], E[0], fb);
        if (E[0] - B[0] > refine_min && L >= 1 && L < 21) {
          const int Lc = L - 1;
          const uint64_t cspan = (1ull << (3 * Lc)) - 1;
          const int64_t hs = (int64_t)1 << Lc;
          uint32_t meet = 0;   // bit c: child c (x + 2y + 4z) meets the box
#pragma unroll
          for (int c = 0; c < 8; ++c) {
            const int64_t x0 = (int64_t)(2 * mx + (c & 1)) << Lc;
            const int64_t y0 = (int64_t)(2 * my + ((c >> 1) & 1)) << Lc;
            const int64_t z0 = (int64_t)(2 * mz + (c >> 2)) << Lc;
            const bool in = x0 <= b[1] && x0 + hs - 1 >= b[0] && y0 <= b[3] &&
                            y0 + hs - 1 >= b[2] && z0 <= b[5] && z0 + hs - 1 >= b[4];
            meet |= (uint32_t)in << c;
          }
          if (meet != 0xFFu) {
            // Runs of consecutive children: the k-th run starts at the k-th
            // set bit of `st` and ends at the k-th set bit of `en`.
            // The runs lie in the cube's index range: searched there, one
            // after the other (four runs in lockstep took longer).
            const uint64_t pb = B[0], pe = E[0];
            uint32_t st = meet & ~(meet << 1);
            uint32_t en = meet & ~(meet >> 1);
#pragma unroll
            for (int k = 0; k < 4; ++k) {
              B[k] = E[k] = 0;
              if (st) {
                const int c0 = __builtin_ctz(st), c1 = __builtin_ctz(en);
                st &= st - 1;
                en &= en - 1;
                const uint64_t klo = mlo | ((uint64_t)c0 << (3 * Lc));
                const uint64_t khi = mlo | ((uint64_t)c1 << (3 * Lc)) | cspan;
                uint64_t x, y;
                search_pair(keys + pb, pe - pb, klo, khi, x, y);
                B[k] = pb + x;
                E[k] = pb + y;
              }
            }
          }
        }
      }
    }
  }
  if (__ballot(bad) != 0 && lane_id() == 0) atomicOr(&counters[2], kErrInvalidQuery);
  __shared__ unsigned long long s_c[4];
  unsigned long long wc = (E[0] - B[0]) + (E[1] - B[1]) + (E[2] - B[2]) + (E[3] - B[3]);
#pragma unroll
  for (int o = 32; o >= 1; o >>= 1) wc += __shfl_xor(wc, o, 64);
  if (lane_id() == 0) s_c[threadIdx.x >> 6] = wc;
  __syncthreads();
  if (threadIdx.x == 0) {
    const unsigned long long t = s_c[0] + s_c[1] + s_c[2] + s_c[3];
    if (t) atomicAdd(cand_total, t);
  }
  if (j < m) {
    if (!REFINE) {
      slot_begin[g] = (uint32_t)B[0];
      slot_count[g] = (uint32_t)(E[0] - B[0]);
      slot_rows[g] = (uint32_t)((E[0] - B[0] + 63) >> 6);
    } else {
#pragma unroll
      for (int t = 0; t < 4; ++t) {
        slot_begin[4 * g + t] = (uint32_t)B[t];
        slot_count[4 * g + t] = (uint32_t)(E[t] - B[t]);
        slot_rows[4 * g + t] = (uint32_t)((E[t] - B[t] + 63) >> 6);
      }
    }
  }
}

// The cells of every query that survive early termination, as (query, cell)
// pairs (4 * query + cell) for the search.  One thread per query; block b
// lists its pairs at the start of its own region pairs[1024 b ..] and its
// counts of pairs and of pruned cells in blk_cnt[b] and blk_pruned[b]
// (pack_scan and pack_move then make the list dense, in query order).  No
// atomic on a shared word: one per block, from every block of the grid,
// serialises across the XCDs.  The slots of cells a query does not have are
// cleared here; invalid queries (and bad set indices) raise the flag and
// list no cell.
template <int CURVE, bool REFINE>
__global__ __launch_bounds__(256) void cells_pack(
    const double2* __restrict__ q, const double* __restrict__ delta, uint64_t m,
    const uint32_t* __restrict__ occ, const uint32_t* __restrict__ qset, uint32_t n_sets,
    uint64_t* __restrict__ pairs, uint32_t* __restrict__ blk_cnt,
    uint32_t* __restrict__ slot_rows, uint32_t* counters,
    uint32_t* __restrict__ blk_pruned, const uint32_t* __restrict__ perm) {
  __shared__ uint16_t lut[CURVE == SFC_CURVE_HILBERT ? 1024 : 1];
  __shared__ uint32_t s_cnt[4];
  __shared__ uint32_t s_pr[4];
  if (CURVE == SFC_CURVE_HILBERT)
    for (int i = threadIdx.x; i < 1024; i += 256) lut[i] = kHilbertLutConst.v[i];
  __syncthreads();
  // perm non-null: queries in curve order, so that the listed pairs (and
  // the searches that follow them) are too.
  const uint64_t jj = (uint64_t)blockIdx.x * 256 + threadIdx.x;
  const uint64_t j = perm && jj < m ? perm[jj] : jj;
  uint32_t nr = 0, pr = 0;
  bool bad = false;
  if (j < m) {
    if (qset && qset[j] >= n_sets) {
      bad = true;
    } else {
      const double2 qq = q[j];
      const double d = delta[j];
      if (!(finite64(qq.x) && finite64(qq.y) && finite64(d) && d >= 0.0)) {
        bad = true;
      } else if (REFINE) {
        uint64_t lo[4], hi[4];
        uint32_t cx[4], cy[4];
        int64_t box[4];
        int L = 0;
        nr = (uint32_t)query_cells<CURVE>(lut, qq.x, qq.y, d, lo, hi, cx, cy, &L, box, occ, &pr);
      } else {
        uint64_t lo[4], hi[4];
        nr = (uint32_t)query_ranges<CURVE>(lut, qq.x, qq.y, d, lo, hi, occ, &pr);
      }
    }
    // The rows of every slot of the query start at zero (one 16- or 32-byte
    // store); the search then writes the slots of the listed cells.  The
    // row scan and the row expansion read a slot's first index and count
    // only when it has rows, so those need no clearing.
    uint4* sr = (uint4*)(slot_rows + (REFINE ? 8 : 4) * j);
    sr[0] = make_uint4(0, 0, 0, 0);
    if (REFINE) sr[1] = make_uint4(0, 0, 0, 0);
  }
  if (__ballot(bad) != 0 && lane_id() == 0) atomicOr(&counters[2], kErrInvalidQuery);
  // Block-exclusive offsets of the cell counts: wave prefix, then waves.
  const uint32_t lane = lane_id(), wv = threadIdx.x >> 6;
  uint32_t inc = nr, wp = pr;
#pragma unroll
  for (int o = 1; o < 64; o <<= 1) {
    const uint32_t t = __shfl_up(inc, o, 64);
    if (lane >= (uint32_t)o) inc += t;
  }
#pragma unroll
  for (int o = 32; o >= 1; o >>= 1) wp += __shfl_xor(wp, o, 64);
  if (lane == 63) s_cnt[wv] = inc;
  if (lane == 0) s_pr[wv] = wp;
  __syncthreads();
  uint32_t before = 0;
  for (uint32_t w = 0; w < wv; ++w) before += s_cnt[w];
  if (threadIdx.x == 0) {
    blk_cnt[blockIdx.x] = s_cnt[0] + s_cnt[1] + s_cnt[2] + s_cnt[3];
    blk_pruned[blockIdx.x] = s_pr[0] + s_pr[1] + s_pr[2] + s_pr[3];
  }
  const uint64_t o = (uint64_t)blockIdx.x * 1024 + before + inc - nr;
  for (uint32_t r = 0; r < nr; ++r) pairs[o + r] = 4 * j + r;
}

// One workgroup: the exclusive scan of the blocks' pair counts (blk_pre, and
// the list's length in *pair_total) and the sum of their pruned cells.
__global__ __launch_bounds__(1024) void pack_scan(const uint32_t* __restrict__ blk_cnt,
                                                  const uint32_t* __restrict__ blk_pruned,
                                                  uint32_t nblk, uint32_t* __restrict__ blk_pre,
                                                  unsigned long long* pair_total,
                                                  unsigned long long* pruned_total) {
  __shared__ uint32_t s_w[16];
  __shared__ unsigned long long s_p[16];
  const uint32_t tid = threadIdx.x, lane = tid & 63, wv = tid >> 6;
  uint32_t carry = 0;
  unsigned long long pruned = 0;
  for (uint32_t b0 = 0; b0 < nblk; b0 += 1024) {
    const uint32_t b = b0 + tid;
    const uint32_t v = b < nblk ? blk_cnt[b] : 0u;
    pruned += b < nblk ? blk_pruned[b] : 0u;
    uint32_t x = v;
#pragma unroll
    for (int o = 1; o < 64; o <<= 1) {
      const uint32_t y = __shfl_up(x, o, 64);
      if (lane >= (uint32_t)o) x += y;
    }
    if (lane == 63) s_w[wv] = x;
    __syncthreads();
    uint32_t before = carry;
    for (uint32_t w = 0; w < wv; ++w) before += s_w[w];
    if (b < nblk) blk_pre[b] = before + x - v;
    uint32_t all = 0;
    for (uint32_t w = 0; w < 16; ++w) all += s_w[w];
    carry += all;
    __syncthreads();
  }
#pragma unroll
  for (int o = 32; o >= 1; o >>= 1) pruned += __shfl_xor(pruned, o, 64);
  if (lane == 0) s_p[wv] = pruned;
  __syncthreads();
  if (tid == 0) {
    unsigned long long p = 0;
    for (int w = 0; w < 16; ++w) p += s_p[w];
    *pair_total = carry;
    *pruned_total = p;
  }
}

// Block b moves its region's pairs to their place in the dense list.
__global__ __launch_bounds__(256) void pack_move(const uint64_t* __restrict__ pairs_in,
                                                 const uint32_t* __restrict__ blk_cnt,
                                                 const uint32_t* __restrict__ blk_pre,
                                                 uint64_t* __restrict__ pairs_out) {
  const uint32_t c = blk_cnt[blockIdx.x], at = blk_pre[blockIdx.x];
  for (uint32_t i = threadIdx.x; i < c; i += 256)
    pairs_out[at + i] = pairs_in[(uint64_t)blockIdx.x * 1024 + i];
}

// The candidates are laid out in rows of 64: each query slot (segment) s
// owns rows [row_off[s], row_off[s+1]), row k of s holding its candidates
// 64k .. 64k+63 (the last row partly filled).  So every row belongs to one
// slot and one query, found by a scalar walk, and the query's data are
// wave-uniform.  A tile is 64 consecutive rows: four waves of kIters x kRows.
constexpr int kRows = 8;                                  // rows per iteration
constexpr int kIters = 2;                                 // iterations per wave
constexpr int kTileRows = 4 * kRows * kIters;             // 64 rows per tile
constexpr uint64_t kWaveRows = (uint64_t)kRows * kIters;  // rows per wave
static_assert(kCompactTileRows == (uint64_t)kTileRows, "tile shape");

// Rows of each query: the sum over its 2^ss slots (the scan that follows
// gives every query its first row).  One lane per slot, so the loads are
// coalesced; a query's slots are 2^ss <= 64 consecutive lanes of one wave,
// summed by shuffles.
__global__ __launch_bounds__(256) void query_rows(const uint32_t* __restrict__ slot_rows,
                                                  uint64_t nseg, int ss, uint32_t* __restrict__ qrows) {
  const uint64_t g = (uint64_t)blockIdx.x * 256 + threadIdx.x;
  uint32_t t = g < nseg ? slot_rows[g] : 0u;
  for (int o = 1; o < (1 << ss); o <<= 1) t += __shfl_xor(t, o, 64);
  if (g < nseg && (g & ((1u << ss) - 1)) == 0) qrows[g >> ss] = t;
}

// Row descriptors of a launch's rows [rbase, rend): for row r of slot s,
// (first sorted index of the row, number of valid lanes, query index).  One
// block per 256 slots (whole queries: 2^ss slots each); a slot's first row is
// its query's first row (row_off, one entry per query) plus the rows of the
// query's earlier slots.  The block's rows are spread over its threads and
// each finds its slot by a binary search in LDS.
__global__ __launch_bounds__(256) void expand_rows(const uint64_t* __restrict__ row_off,
                                                   const uint32_t* __restrict__ slot_rows,
                                                   const uint32_t* __restrict__ slot_begin,
                                                   const uint32_t* __restrict__ slot_count,
                                                   uint64_t nseg, int ss, uint64_t rbase,
                                                   uint64_t row_end, uint4* __restrict__ row_meta) {
  __shared__ uint64_t st[257];
  const uint64_t m = nseg >> ss;
  const uint64_t total = row_off[m];
  const uint64_t rend = total < row_end ? total : row_end;
  const uint64_t s0 = (uint64_t)blockIdx.x * 256;
  const uint32_t tid = threadIdx.x;
  // The rows of the query's earlier slots: an exclusive scan within each
  // group of 2^ss lanes (a query's slots, inside one wave).
  const uint32_t v = s0 + tid < nseg ? slot_rows[s0 + tid] : 0u;
  const uint32_t gl = tid & ((1u << ss) - 1);
  uint32_t x = v;
  for (int o = 1; o < (1 << ss); o <<= 1) {
    const uint32_t y = __shfl_up(x, o, 64);
    if (gl >= (uint32_t)o) x += y;
  }
  st[tid] = s0 + tid < nseg ? row_off[(s0 + tid) >> ss] + (x - v) : total;
  if (tid == 0) st[256] = s0 + 256 < nseg ? row_off[(s0 + 256) >> ss] : total;
  __syncthreads();
  const uint64_t r0 = st[0] > rbase ? st[0] : rbase;
  const uint64_t r1 = st[256] < rend ? st[256] : rend;
  for (uint64_t r = r0 + tid; r < r1; r += 256) {
    uint32_t lo = 0, len = 256;   // largest k with st[k] <= r
    while (len > 0) {
      const uint32_t h = len >> 1;
      if (st[lo + h] <= r) {
        lo += h + 1;
        len -= h + 1;
      } else {
        len = h;
      }
    }
    const uint32_t k = lo - 1;
    const uint64_t sg = s0 + k;
    const uint64_t local = (r - st[k]) * kWave;
    const uint64_t cnt = slot_count[sg];
    const uint64_t nv = cnt - local < (uint64_t)kWave ? cnt - local : (uint64_t)kWave;
    row_meta[r - rbase] = make_uint4((uint32_t)(slot_begin[sg] + local), (uint32_t)nv,
                                     (uint32_t)(sg >> ss), 0u);
  }
}

// ---- deciding the test from a point's grid cell ---------------------------------
//
// A point p with grid cell u = floor(p * S) (S = 2^32 in the plane, 2^21 in
// three dimensions) lies in [u, u + 1) quanta on each axis.  Measured in
// quanta from the query's own cell c = floor(q S), its offset on an axis is
// o = e + th with the integer e = u - c and |th| < 1, so o^2 lies within
// 2|e| + 1 of e^2.  A candidate comes from the query's own cells, which meet
// the box widened by one quantum, so |e| <= E = 6R + 10 with R = d S (exact
// scalings): the sum of the squared offsets lies within the slack
// s = DIM (2E + 1) of the sum of the e^2.  For the Euclidean test:
//   * if sum e^2 <= R^2 (1 - 2^-16) - s, the rounded binary64 test accepts p;
//   * if sum e^2 > R^2 (1 + 2^-16) + s, it rejects p;
// for the square window, |e| <= R (1 - 2^-16) - 1 on every axis accepts and
// |e| > R (1 + 2^-16) + 1 on some axis rejects.  Evaluated in binary32
// (relative errors below 2^-20 all told) these verdicts equal the exact
// test's, whose own rounding is a few 2^-53 relative, when R >= 16 (so the
// slack is small beside R^2).  Other points read their coordinates and take
// the exact test.  A query uses the filter when R >= 16 and its cell lies
// within 2^30 quanta of the domain.  Above R = 2^28 (plane) / 2^17 (three
// dimensions) the cells are compared 2^k quanta wide (u >> k against
// floor(q S 2^-k), k the smallest shift that brings R 2^-k to that limit,
// at most 24): the same bounds hold there with R 2^-k for R, since the
// shifted offsets again differ from the exact ones by less than one.  Then
// |e| < 2^31, exact in 32-bit arithmetic.  Cells sit in one word: x | y << 32,
// or x | y << 21 | z << 42.
struct QueryFilter {
  float acc, rej;   // limits on sum e^2 (or per-axis |e|); filter off: acc = not a number
                    // and rej = +inf, so that neither comparison decides a candidate
  uint32_t c[3];    // the query's cell per axis (low 32 bits), 2^shift quanta wide
  uint32_t shift;   // cells are compared 2^shift quanta wide
  uint32_t pad[2];
};
static_assert(sizeof(QueryFilter) == 32, "a record is 32 bytes");
// The batch counter word that flag_coarse sets when some query may compare
// coarser cells (the counters are cleared when the ranges are computed).
constexpr int kShiftWord = 13;   // free: 2 errors, 4-11 statistics, 12 tiles, 14-15 total

// Sets counters[kShiftWord] when some radius of the batch lies above the
// filter's shift limit (delta S > limit): then the test pass reads the cell
// shifts.  One atomic per workgroup that has such a radius.
__global__ __launch_bounds__(256) void flag_coarse(const double* __restrict__ delta, uint64_t m,
                                                   double S, double limit,
                                                   uint32_t* __restrict__ counters) {
  __shared__ uint32_t s_any;
  if (threadIdx.x == 0) s_any = 0;
  __syncthreads();
  const uint64_t j = (uint64_t)blockIdx.x * 256 + threadIdx.x;
  if (j < m && delta[j] * S > limit) s_any = 1;
  __syncthreads();
  if (threadIdx.x == 0 && s_any) atomicOr(&counters[kShiftWord], 1u);
}

template <int DIM>
__global__ __launch_bounds__(256) void query_filters(const double* __restrict__ q,
                                                     const double* __restrict__ delta, uint64_t m,
                                                     bool window, QueryFilter* __restrict__ out) {
  constexpr double S = DIM == 2 ? 4294967296.0 : 2097152.0;
  constexpr double kMaxR = DIM == 2 ? 0x1p28 : 0x1p17;
  const uint64_t j = (uint64_t)blockIdx.x * 256 + threadIdx.x;
  if (j >= m) return;
  const double R0 = delta[j] * S;
  int k = 0;
  while (k < 24 && R0 > kMaxR * __builtin_ldexp(1.0, k)) ++k;
  const double R = __builtin_ldexp(R0, -k);   // exact
  bool on = R0 >= 16.0 && R <= kMaxR;
  QueryFilter f{};
  f.shift = (uint32_t)k;
#pragma unroll
  for (int a = 0; a < DIM; ++a) {
    const double qs = q[DIM * j + a] * S;
    on = on && qs > -0x1p30 && qs < S + 0x1p30;
    f.c[a] = (uint32_t)(int64_t)__builtin_floor(on ? __builtin_ldexp(qs, -k) : 0.0);
  }
  if (window) {
    f.acc = (float)(R * (1.0 - 0x1p-16) - 1.0);
    f.rej = (float)(R * (1.0 + 0x1p-16) + 1.0);
  } else {
    const double slack = DIM * (2.0 * (6.0 * R + 10.0) + 1.0);
    f.acc = (float)(R * R * (1.0 - 0x1p-16) - slack);
    f.rej = (float)(R * R * (1.0 + 0x1p-16) + slack);
  }
  if (!on) {   // undecided for every candidate: the exact test decides
    f.acc = __uint_as_float(0xFFFFFFFFu);
    f.rej = __builtin_inff();
    f.shift = 0;
  }
  out[j] = f;
}

// 1: accepted, 0: rejected, -1: undecided by the cell.  SHIFTED: the cells
// are compared f.shift bits coarser (else f.shift is 0).
template <int DIM, bool WINDOW, bool SHIFTED>
__device__ __forceinline__ int cell_check(uint64_t cell, const QueryFilter& f) {
  constexpr int B = DIM == 2 ? 32 : 21;
  const uint64_t mask = (1ull << B) - 1;
  float e[DIM];
#pragma unroll
  for (int a = 0; a < DIM; ++a) {
    uint32_t u = (uint32_t)((cell >> (B * a)) & mask);
    if (SHIFTED) u >>= f.shift;
    e[a] = (float)(int32_t)(u - f.c[a]);
  }
  if (WINDOW) {
    bool in = true, out = false;
#pragma unroll
    for (int a = 0; a < DIM; ++a) {
      in = in && fabsf(e[a]) <= f.acc;
      out = out || fabsf(e[a]) > f.rej;
    }
    return in ? 1 : out ? 0 : -1;
  }
  float d2 = e[0] * e[0];
#pragma unroll
  for (int a = 1; a < DIM; ++a) d2 = d2 + e[a] * e[a];
  return d2 <= f.acc ? 1 : d2 > f.rej ? 0 : -1;
}

// The exact test of candidate pos against query qs (the point and the query
// read here: only for candidates their cell could not decide).  The point
// is src[pos] (sorted points), or src[via[pos]] (input order, via = ids).
template <int DIM>
__device__ __forceinline__ bool exact_hit(const double* __restrict__ q,
                                          const double* __restrict__ delta,
                                          const double* __restrict__ src,
                                          const uint32_t* __restrict__ via, uint32_t qs,
                                          uint32_t pos, bool window) {
  const double d = delta[qs];
  const uint64_t at = via ? via[pos] : pos;
  if (DIM == 2) {
    const double2 qq = ((const double2*)q)[qs];
    const double2 p = ((const double2*)src)[at];
    return window ? within_window(p.x, p.y, qq.x, qq.y, d) : within(p.x, p.y, qq.x, qq.y, d);
  }
  const double* qp = q + 3 * (uint64_t)qs;
  const double* pp = src + 3 * at;
  return window ? within_window3(pp[0], pp[1], pp[2], qp[0], qp[1], qp[2], d)
                : within3(pp[0], pp[1], pp[2], qp[0], qp[1], qp[2], d);
}

// Pass 1: the exact test of every candidate; per row the 64-bit mask of the
// accepted lanes, per tile their number.  Each wave handles 16 consecutive
// rows as ITERS groups of ROWS rows whose point loads are in flight together,
// writes its 16 masks with one store (lane j: row j) and adds its count to
// the tile's (zeroed before the launch), so that the waves of a workgroup
// never wait for each other.
// EPOCH: a candidate that passes the test also has to be visible at the
// query's epoch (ins <= e < era); only those lanes read the epochs.
// window: the square-window test instead of the Euclidean one.
template <int ROWS, int ITERS, bool EPOCH, int DIM, bool CELLS, bool WINDOW, bool SHIFTS>
__global__ __launch_bounds__(256) void compact_test(
    const double* __restrict__ q, const double* __restrict__ delta, uint64_t m,
    const double* __restrict__ pts, const uint32_t* __restrict__ via,
    const uint64_t* __restrict__ cells,
    const QueryFilter* __restrict__ qfilt, uint64_t npts, const uint4* __restrict__ row_meta,
    const uint64_t* __restrict__ total_rows_dev, uint64_t rbase, uint64_t row_end,
    bool flag_overflow, uint64_t* __restrict__ masks, uint32_t* __restrict__ tile_hits,
    uint32_t* counters, const uint32_t* __restrict__ ins, const uint32_t* __restrict__ era,
    const uint32_t* __restrict__ qepoch, uint32_t epoch) {
  static_assert(ROWS * ITERS == (int)kWaveRows, "a wave's groups cover its rows");
  const uint32_t tid = threadIdx.x, w = tid >> 6, lane = tid & 63;
  // SHIFTS: the batch may hold queries with coarser cells (flag_coarse)
  const bool any_shifted = SHIFTS && CELLS && counters[kShiftWord] != 0u;
  const uint64_t total_all = *total_rows_dev;
  const uint64_t total_rows = total_all < row_end ? total_all : row_end;
  const uint64_t ntiles = total_rows > rbase ? (total_rows - rbase + kTileRows - 1) / kTileRows : 0;
  for (uint64_t tile = blockIdx.x; tile < ntiles; tile += gridDim.x) {
    const uint64_t wrow0 = rbase + tile * kTileRows + (uint64_t)w * kWaveRows;
    uint32_t cnt = 0;
    uint64_t mrow = 0;   // lane j < 16: the mask of the wave's row j
    // The records of the wave's rows, one per lane, in one load.
    uint4 mdw = make_uint4(0, 0, 0, 0);
    if (lane < (uint32_t)kWaveRows && wrow0 + lane < total_rows)
      mdw = row_meta[wrow0 + lane - rbase];
#pragma unroll
    for (int it = 0; it < ITERS; ++it) {
      const uint4 md = mdw;   // rows it * ROWS .. it * ROWS + ROWS - 1 of the wave
      uint32_t pos[ROWS];
      uint32_t qrow[ROWS];
      bool act[ROWS];
#pragma unroll
      for (int jr = 0; jr < ROWS; ++jr) {
        const uint32_t pb = __builtin_amdgcn_readlane(md.x, it * ROWS + jr);
        const uint32_t nv = __builtin_amdgcn_readlane(md.y, it * ROWS + jr);
        const uint32_t qi = __builtin_amdgcn_readlane(md.z, it * ROWS + jr);
        const uint64_t p64 = (uint64_t)pb + lane;
        act[jr] = lane < nv && p64 < npts && qi < m;
        pos[jr] = act[jr] ? (uint32_t)p64 : 0u;
        qrow[jr] = qi < m ? qi : 0u;
      }
      bool hit[ROWS];
      if constexpr (CELLS) {
        // Decide from the cells; the coordinates only for undecided lanes.
        // The rows' filter records (uniform loads) and cells are all
        // requested before any is used.
        // (the plane needs the record's first 16 bytes: limits and x, y; the
        // cell shifts only in a batch with coarser cells)
        QueryFilter qf[ROWS];
#pragma unroll
        for (int jr = 0; jr < ROWS; ++jr) {
          const uint4 a = ((const uint4*)qfilt)[2 * (uint64_t)qrow[jr]];
          qf[jr].acc = __uint_as_float(a.x);
          qf[jr].rej = __uint_as_float(a.y);
          qf[jr].c[0] = a.z;
          qf[jr].c[1] = a.w;
          qf[jr].c[2] = DIM == 3 ? qfilt[qrow[jr]].c[2] : 0u;
          qf[jr].shift = 0;
        }
        uint64_t cv[ROWS];
#pragma unroll
        for (int jr = 0; jr < ROWS; ++jr) cv[jr] = cells[pos[jr]];   // pos 0 when inactive
        bool und[ROWS];
        bool any = false;
        // A batch with coarser cells (radii past the shift limit) takes the
        // shifting check.
        if (!any_shifted) {
#pragma unroll
          for (int jr = 0; jr < ROWS; ++jr) {
            const int vd = act[jr] ? cell_check<DIM, WINDOW, false>(cv[jr], qf[jr]) : 0;
            hit[jr] = vd == 1;
            und[jr] = vd < 0;
            any = any || und[jr];
          }
        } else {
#pragma unroll
          for (int jr = 0; jr < ROWS; ++jr) {
            qf[jr].shift = qfilt[qrow[jr]].shift;
            const int vd = act[jr] ? cell_check<DIM, WINDOW, true>(cv[jr], qf[jr]) : 0;
            hit[jr] = vd == 1;
            und[jr] = vd < 0;
            any = any || und[jr];
          }
        }
        // The candidates their cells leave undecided (rare) take the exact
        // test, behind one branch for the whole group.
        if (__ballot(any) != 0) {
#pragma unroll
          for (int jr = 0; jr < ROWS; ++jr)
            if (und[jr]) hit[jr] = exact_hit<DIM>(q, delta, pts, via, qrow[jr], pos[jr], WINDOW);
        }
      } else {
        double qx[ROWS], qy[ROWS], qz[ROWS], dd[ROWS];
#pragma unroll
        for (int jr = 0; jr < ROWS; ++jr) {
          const uint32_t qs = qrow[jr];
          if (DIM == 2) {
            const double2 qq = ((const double2*)q)[qs];
            qx[jr] = qq.x;
            qy[jr] = qq.y;
          } else {
            qx[jr] = q[3 * (uint64_t)qs];
            qy[jr] = q[3 * (uint64_t)qs + 1];
            qz[jr] = q[3 * (uint64_t)qs + 2];
          }
          dd[jr] = delta[qs];
        }
        double2 pv[ROWS];
        double pz[ROWS];
#pragma unroll
        for (int jr = 0; jr < ROWS; ++jr) {
          if (act[jr]) {
            if (DIM == 2) {
              pv[jr] = ((const double2*)pts)[pos[jr]];
            } else {
              pv[jr].x = pts[3 * (uint64_t)pos[jr]];
              pv[jr].y = pts[3 * (uint64_t)pos[jr] + 1];
              pz[jr] = pts[3 * (uint64_t)pos[jr] + 2];
            }
          }
        }
#pragma unroll
        for (int jr = 0; jr < ROWS; ++jr) {
          if (DIM == 2)
            hit[jr] = act[jr] &&
                      (WINDOW ? within_window(pv[jr].x, pv[jr].y, qx[jr], qy[jr], dd[jr])
                              : within(pv[jr].x, pv[jr].y, qx[jr], qy[jr], dd[jr]));
          else
            hit[jr] = act[jr] && (WINDOW ? within_window3(pv[jr].x, pv[jr].y, pz[jr], qx[jr],
                                                          qy[jr], qz[jr], dd[jr])
                                         : within3(pv[jr].x, pv[jr].y, pz[jr], qx[jr], qy[jr],
                                                   qz[jr], dd[jr]));
        }
      }
#pragma unroll
      for (int jr = 0; jr < ROWS; ++jr) {
        bool h = hit[jr];
        if (EPOCH && h) {
          const uint32_t qe = qepoch ? qepoch[qrow[jr]] : epoch;
          h = ins[pos[jr]] <= qe && qe < era[pos[jr]];
        }
        const uint64_t bal = __ballot(h);
        cnt += (uint32_t)__popcll(bal);
        if (lane == (uint32_t)(it * ROWS + jr)) mrow = bal;
      }
    }
    if (lane < (uint32_t)kWaveRows)
      masks[tile * kTileRows + (uint64_t)w * kWaveRows + lane] = mrow;
    if (lane == 0 && cnt) atomicAdd(&tile_hits[tile], cnt);
  }
  if (blockIdx.x == 0 && tid == 0) {
    counters[12] = (uint32_t)ntiles;   // tile count for the scan that follows
    if (flag_overflow && total_all > row_end) atomicOr(&counters[2], kErrOverflow);
  }
}

// Pass 2: the ids of the accepted candidates at the tile's output offset, in
// row order (= curve order per query), and the absolute output position of
// every row of the tile (row_pre, chunk-relative index; the entry one past a
// tile's last row is the next tile's first, and the one at the batch's last
// row + 1 is the total).  Output-driven: one lane per reported id rather than
// one per candidate.  The waves first map every output o of the tile to its
// row and its candidate within the row (one 16-bit map in LDS, written by the
// lanes whose bit is set); the output's id is then read at the row's first
// candidate position plus that candidate.  Writes are contiguous; a tile
// with few hits costs few lanes.
__global__ __launch_bounds__(256) void compact_write_out(
    const uint32_t* __restrict__ ids, uint64_t npts, const uint4* __restrict__ row_meta,
    const uint64_t* __restrict__ total_rows_dev, uint64_t rbase, uint64_t row_end,
    const uint64_t* __restrict__ masks, const uint64_t* __restrict__ tile_off,
    uint64_t* __restrict__ row_pre, uint32_t* __restrict__ out_ids, uint64_t cap, bool whole) {
  __shared__ uint64_t s_mask[kTileRows];
  __shared__ uint32_t s_pre[kTileRows + 1];
  __shared__ uint32_t s_base[kTileRows];
  // Output o of the tile: its row << 8 | its candidate within the row.
  __shared__ uint16_t s_map[kTileRows * 64];
  const uint32_t tid = threadIdx.x, lane = tid & 63, wv = tid >> 6;
  const uint64_t below = lanemask_lt();
  const uint64_t total_all = *total_rows_dev;
  const uint64_t total_rows = total_all < row_end ? total_all : row_end;
  const uint64_t ntiles = total_rows > rbase ? (total_rows - rbase + kTileRows - 1) / kTileRows : 0;
  const bool write_ids = !whole || ntiles == 0 || tile_off[ntiles] <= cap;
  // The next tile's masks and first positions are loaded while this tile is
  // written (one row per thread of the first wave).
  uint64_t nx_mask = 0;
  uint32_t nx_base = 0;
  uint64_t nx_off = 0;
  auto fetch = [&](uint64_t t) {
    const uint64_t r0 = rbase + t * kTileRows;
    if (t < ntiles && tid < kTileRows) {
      nx_mask = masks[t * kTileRows + tid];
      nx_base = r0 + tid < total_rows ? row_meta[r0 + tid - rbase].x : 0u;
    }
    if (t < ntiles) nx_off = tile_off[t];
  };
  fetch(blockIdx.x);
  for (uint64_t tile = blockIdx.x; tile < ntiles; tile += gridDim.x) {
    const uint64_t trow0 = rbase + tile * kTileRows;
    if (tid < kTileRows) {
      s_mask[tid] = nx_mask;
      s_base[tid] = nx_base;
    }
    const uint64_t prefix = nx_off;
    __syncthreads();
    fetch(tile + gridDim.x);
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
    if (tid <= kTileRows && trow0 + tid <= total_rows)
      row_pre[tile * kTileRows + tid] = prefix + s_pre[tid];
    const uint32_t hits = s_pre[kTileRows];
    if (write_ids) {
      // Each wave maps the outputs of 16 rows (lane l of row r, if its bit
      // is set, is output s_pre[r] + the set bits below it), then every
      // output finds its row and candidate with one read of each map.
      for (uint32_t k = 0; k < kTileRows / 4; ++k) {
        const uint32_t r = wv * (kTileRows / 4) + k;
        const uint64_t mk = s_mask[r];
        if ((mk >> lane) & 1ull) {
          const uint32_t o = s_pre[r] + (uint32_t)__popcll(mk & below);
          s_map[o] = (uint16_t)((r << 8) | lane);
        }
      }
      __syncthreads();
      for (uint32_t o = tid; o < hits; o += 256) {
        const uint32_t mp = s_map[o];
        const uint64_t p64 = (uint64_t)s_base[mp >> 8] + (mp & 0xFFu);
        const uint64_t opos = prefix + o;
        if (p64 < npts && opos < cap) out_ids[opos] = ids[p64];
      }
    }
    __syncthreads();
  }
}

// The CSR offsets of the queries whose first row lies in this chunk: query
// j's offset is the output position of row row_off[j] (a query with no
// rows takes the position of the next row, trailing ones the total).  One
// thread per query; the chunk owns rows [rbase, rend) below the total and,
// if the total falls in (rbase, rend], the total itself.
__global__ __launch_bounds__(256) void query_offsets(
    const uint64_t* __restrict__ row_off, int ss, uint64_t m,
    const uint64_t* __restrict__ total_rows_dev, uint64_t rbase, uint64_t rend, uint64_t row_end,
    const uint64_t* __restrict__ row_pre, uint64_t* __restrict__ offsets) {
  const uint64_t total_all = *total_rows_dev;
  const uint64_t total = total_all < row_end ? total_all : row_end;
  const bool owns_total = total == 0 ? rbase == 0 : (rbase < total && total <= rend);
  const uint64_t stride = (uint64_t)gridDim.x * blockDim.x;
  for (uint64_t j = (uint64_t)blockIdx.x * blockDim.x + threadIdx.x; j <= m; j += stride) {
    uint64_t r = row_off[j];
    if (r > total) r = total;   // past the capacity (flagged as overflow)
    if (r == total) {
      if (owns_total) offsets[j] = total == 0 ? 0 : row_pre[r - rbase];
    } else if (r >= rbase && r < rend) {
      offsets[j] = row_pre[r - rbase];
    }
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

// Tiles per compaction chunk (lowered only by the test hook).
std::atomic<uint64_t> g_chunk_tiles{kCompactChunkTiles};

// Shape of the test kernel's row groups, rows x iterations: 0: 16 x 1,
// 1: 4 x 4, 2: 8 x 2, 3: 2 x 8, 4: 1 x 16 (same results for all).  The
// environment variable SFC_TEST_VARIANT overrides; else the autotuner's choice
// for this number of rows; else 1 (measured fastest: 0.531 ms vs 0.541 ms for
// 8 x 2 and 0.614 ms for 16 x 1 at 8 * 10^6 rows; the 256-set batch 1.96 vs
// 2.09 ms).
int test_variant(uint64_t rows) {
  static const int env = [] {
    const char* e = std::getenv("SFC_TEST_VARIANT");
    return e ? std::atoi(e) + 1 : 0;
  }();
  const int v = env ? env - 1 : tuned(kTuneTestShape, rows);
  return v >= 0 && v <= 4 ? v : 1;
}

uint32_t fill_blocks(uint64_t count) {
  uint64_t b = (count + 255) / 256;
  if (b > 2048) b = 2048;
  return b < 1 ? 1 : (uint32_t)b;
}

}  // namespace

uint64_t compact_chunk_tiles() { return g_chunk_tiles.load(std::memory_order_relaxed); }
bool compact_single_chunk(uint64_t total_rows) {
  return (total_rows + kCompactTileRows - 1) / kCompactTileRows <= compact_chunk_tiles();
}
void set_compact_chunk_tiles(uint64_t tiles) {
  g_chunk_tiles.store(tiles == 0 || tiles > kCompactChunkTiles ? kCompactChunkTiles : tiles,
                      std::memory_order_relaxed);
}

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

size_t query_scratch_bytes(uint64_t m, uint32_t slots) {
  const uint64_t nseg = slots * m;
  return align256(nseg * 4) * 3 + align256((nseg + 1) * 8) + scan_scratch_bytes(nseg) +
         align256(64) + align256(4 * m * 8) + align256(m * 32) + align256(m * 4) +
         order_scratch_bytes(m) + align256(m * 4);
}

void query_scratch_carve(void* base, uint64_t m, QueryScratch* qs, uint32_t slots) {
  const uint64_t nseg = slots * m;
  char* p = (char*)base;
  qs->slot_begin = (uint32_t*)p;  p += align256(nseg * 4);
  qs->slot_count = (uint32_t*)p;  p += align256(nseg * 4);
  qs->slot_rows = (uint32_t*)p;   p += align256(nseg * 4);
  qs->row_off = (uint64_t*)p;     p += align256((nseg + 1) * 8);
  qs->scan_tmp = (uint64_t*)p;    p += scan_scratch_bytes(nseg);
  qs->counters = (uint32_t*)p;    p += align256(64);
  qs->pairs = (uint64_t*)p;       p += align256(4 * m * 8);
  qs->qfilt = p;                  p += align256(m * 32);
  qs->perm = (uint32_t*)p;        p += align256(m * 4);
  qs->qrows = (uint32_t*)p;       p += align256(m * 4);
  qs->order_scratch = p;
  qs->ss = 2;
}

size_t compact_scratch_bytes(uint64_t total_rows) {
  uint64_t tiles = (total_rows + kCompactTileRows - 1) / kCompactTileRows;
  if (tiles > kCompactChunkTiles) tiles = kCompactChunkTiles;
  if (tiles == 0) tiles = 1;
  return align256(tiles * kTileRows * 8) + align256(tiles * 4) + 2 * align256((tiles + 1) * 8) +
         align256(tiles * kTileRows * 16) + align256((tiles * kTileRows + 1) * 8) +
         scan_scratch_bytes(tiles);
}

// Every query's first row (row_off[j], and the total at row_off[m]): its
// slots' rows summed, then scanned over the queries.
hipError_t scan_query_rows(QueryScratch& qs, uint64_t m, hipStream_t s) {
  {
    ProfScope ps("scan", s);
    query_rows<<<(uint32_t)(((m << qs.ss) + 255) / 256), 256, 0, s>>>(qs.slot_rows, m << qs.ss,
                                                                       qs.ss, qs.qrows);
    hipError_t e = hipGetLastError();
    if (e != hipSuccess) return e;
  }
  return scan_excl(qs.qrows, qs.row_off, m, nullptr, qs.scan_tmp, s);
}

// Batches from this size on are ordered along the curve before the search.
constexpr uint64_t kOrderMin = 1u << 14;

hipError_t launch_ranges(const double* q, const double* delta, uint64_t m, const uint64_t* keys,
                         uint64_t n, int curve, bool refine, uint32_t refine_min, bool ball,
                         const LearnedView* lview, const StreeView* sview, const uint32_t* occ,
                         const uint32_t* qset, const uint64_t* set_off, uint32_t n_sets,
                         QueryScratch& qs, uint64_t* dbg_lo, uint64_t* dbg_hi, uint64_t* dbg_b,
                         uint64_t* dbg_e, uint32_t* dbg_nr, hipStream_t s) {
  if (m == 0) return hipSuccess;
  const uint32_t blocks = (uint32_t)((4 * m + 255) / 256);
  hipError_t e;
  if ((e = fill_u32(qs.counters, 0, 16, s)) != hipSuccess) return e;
  flag_coarse<<<(uint32_t)((m + 255) / 256), 256, 0, s>>>(delta, m, 4294967296.0, 0x1p28,
                                                           qs.counters);
  if ((e = hipGetLastError()) != hipSuccess) return e;
  if (dbg_lo) refine = false;   // the inspected ranges are the method's merged ranges
  qs.ss = refine ? 3 : 2;
  const bool learned = lview != nullptr && qset == nullptr;
  const bool stree = !learned && sview != nullptr && qset == nullptr;
  const LearnedView lv = learned ? *lview : LearnedView{};
  const StreeView sv = stree ? *sview : StreeView{};
  unsigned long long* cand = (unsigned long long*)(qs.counters + 4);
  // With early termination (and no inspected ranges) the search runs one
  // lane per surviving cell, from a dense list of (query, cell) pairs.
  const bool dense = occ != nullptr && dbg_lo == nullptr;
  unsigned long long* total = (unsigned long long*)(qs.counters + 14);   // cleared above
  const uint64_t* pairs = nullptr;
  const uint64_t* pair_total = nullptr;
  // Large batches over the whole array are searched in curve order (with
  // early termination: listed in that order).
  const uint32_t* perm = nullptr;
  if (!dbg_lo && !qset && m >= kOrderMin) {
    if ((e = order_queries(q, m, curve, qs.perm, qs.order_scratch, qs.counters + 2, s)) !=
        hipSuccess)
      return e;
    perm = qs.perm;
  }
  if (dense) {
    const uint32_t qb = (uint32_t)((m + 255) / 256);
    // Until the row scan (after the search) fills them: the row offsets hold
    // each block's region of pairs (4m entries at most), and the query row
    // counts the blocks' counts, pruned cells and exclusive prefixes.
    uint64_t* regions = qs.row_off;
    uint32_t* blk_cnt = qs.qrows;
    uint32_t* blk_pruned = qs.qrows + qb;
    uint32_t* blk_pre = qs.qrows + 2 * (uint64_t)qb;
    ProfScope ps("cells_pack", s);
#define SFC_CELLS(C, R)                                                                    \
  cells_pack<C, R><<<qb, 256, 0, s>>>((const double2*)q, delta, m, occ, qset, n_sets,       \
                                      regions, blk_cnt, qs.slot_rows, qs.counters,          \
                                      blk_pruned, perm)
    if (curve == SFC_CURVE_HILBERT) {
      if (refine) SFC_CELLS(SFC_CURVE_HILBERT, true);
      else SFC_CELLS(SFC_CURVE_HILBERT, false);
    } else {
      if (refine) SFC_CELLS(SFC_CURVE_MORTON, true);
      else SFC_CELLS(SFC_CURVE_MORTON, false);
    }
#undef SFC_CELLS
    if ((e = hipGetLastError()) != hipSuccess) return e;
    pack_scan<<<1, 1024, 0, s>>>(blk_cnt, blk_pruned, qb, blk_pre, total, cand + 3);
    if ((e = hipGetLastError()) != hipSuccess) return e;
    pack_move<<<qb, 256, 0, s>>>(regions, blk_cnt, blk_pre, qs.pairs);
    if ((e = hipGetLastError()) != hipSuccess) return e;
    pairs = qs.pairs;
    pair_total = (const uint64_t*)total;
  }
  {
    ProfScope ps(learned ? "ranges_learned" : stree ? "ranges_stree" : "ranges_search", s);
#define SFC_RANGES(C, R, S)                                                                  \
  ranges_search<C, R, S><<<blocks, 256, 0, s>>>(                                              \
      (const double2*)q, delta, m, keys, n, lv, sv, refine_min, ball, dbg_lo ? nullptr : occ, \
      pairs, pair_total, qset, set_off, n_sets, qs.slot_begin,                                \
      qs.slot_count, qs.slot_rows, qs.counters, cand, dense ? nullptr : perm, dbg_lo, dbg_hi, \
      dbg_b, dbg_e, dbg_nr)
#define SFC_RANGES_R(C, R)                      \
  if (learned) SFC_RANGES(C, R, 1);             \
  else if (stree) SFC_RANGES(C, R, 2);          \
  else SFC_RANGES(C, R, 0);
#define SFC_RANGES_C(C)                         \
  if (refine) {                                 \
    SFC_RANGES_R(C, true)                       \
  } else {                                      \
    SFC_RANGES_R(C, false)                      \
  }
    if (curve == SFC_CURVE_HILBERT) {
      SFC_RANGES_C(SFC_CURVE_HILBERT)
    } else {
      SFC_RANGES_C(SFC_CURVE_MORTON)
    }
#undef SFC_RANGES_C
#undef SFC_RANGES_R
#undef SFC_RANGES
    if ((e = hipGetLastError()) != hipSuccess) return e;
  }
  return scan_query_rows(qs, m, s);
}

// Blocks of the compaction kernels (grid-stride over tiles beyond this):
// 16384, 64 per CU, measured best of 4096 to 32768 (the 2^24 batch's test
// and write passes 0.968 -> 0.958 ms against 8192).
constexpr uint64_t kCompactGrid = 16384;

hipError_t launch_ranges3(const double* q, const double* delta, uint64_t m, const uint64_t* keys,
                          uint64_t n, bool refine, uint32_t refine_min, const StreeView* sview,
                          QueryScratch& qs, hipStream_t s) {
  if (m == 0) return hipSuccess;
  hipError_t e;
  if ((e = fill_u32(qs.counters, 0, 16, s)) != hipSuccess) return e;
  flag_coarse<<<(uint32_t)((m + 255) / 256), 256, 0, s>>>(delta, m, 2097152.0, 0x1p17,
                                                           qs.counters);
  if ((e = hipGetLastError()) != hipSuccess) return e;
  qs.ss = refine ? 5 : 3;
  const uint32_t blocks = (uint32_t)((8 * m + 255) / 256);
  unsigned long long* cand = (unsigned long long*)(qs.counters + 4);
  const LearnedView lv{};
  const StreeView sv = sview ? *sview : StreeView{};
  {
    ProfScope ps(sview ? "ranges_stree3" : "ranges_search3", s);
#define SFC_R3(S, R)                                                                         \
  ranges_search3<S, R><<<blocks, 256, 0, s>>>(q, delta, m, keys, n, lv, sv, refine_min,      \
                                              qs.slot_begin, qs.slot_count, qs.slot_rows,    \
                                              qs.counters, cand)
    if (sview) {
      if (refine) SFC_R3(2, true);
      else SFC_R3(2, false);
    } else {
      if (refine) SFC_R3(0, true);
      else SFC_R3(0, false);
    }
#undef SFC_R3
    if ((e = hipGetLastError()) != hipSuccess) return e;
  }
  return scan_query_rows(qs, m, s);
}

hipError_t launch_compact(const double* q, const double* delta, uint64_t m, const double* pts,
                          const double* pts_in, const uint64_t* cells, const uint32_t* ids,
                          uint64_t npts, const QueryScratch& qs,
                          uint64_t max_rows, bool device_sized, void* cscratch,
                          uint64_t* offsets, uint32_t* out_ids, uint64_t cap, bool window,
                          int dim, hipStream_t s, const EpochView* ev, bool write_only,
                          int coarse) {
  hipError_t e;
  if (m == 0) return fill_u64(offsets, 0, 1, s);
  // Whether the test pass may meet queries with coarser cells: known (0, 1)
  // when the caller read the batch's flag, else (-1) the pass reads it.
  const bool shifts = coarse != 0;
  const uint64_t nseg = m << qs.ss;
  const uint64_t* total_dev = qs.row_off + m;
  // Rows are processed in chunks of at most kCompactChunkTiles tiles.
  // Host-sized: max_rows is the exact number of rows.  Device-sized: max_rows
  // is a capacity; each kernel reads the row count on the device, chunks past
  // it do no work, and a count above the capacity is flagged as overflow.
  const uint64_t tiles_all = (max_rows + kCompactTileRows - 1) / kCompactTileRows;
  if (!device_sized && max_rows == 0) return fill_u64(offsets, 0, m + 1, s);
  const uint64_t chunk = compact_chunk_tiles();
  const uint64_t ch_tiles = tiles_all < chunk ? (tiles_all ? tiles_all : 1) : chunk;
  char* p = (char*)cscratch;
  uint64_t* masks = (uint64_t*)p;     p += align256(ch_tiles * kTileRows * 8);
  uint32_t* hits = (uint32_t*)p;      p += align256(ch_tiles * 4);
  uint64_t* toff[2];
  toff[0] = (uint64_t*)p;             p += align256((ch_tiles + 1) * 8);
  toff[1] = (uint64_t*)p;             p += align256((ch_tiles + 1) * 8);
  uint4* meta = (uint4*)p;            p += align256(ch_tiles * kTileRows * 16);
  uint64_t* rpre = (uint64_t*)p;      p += align256((ch_tiles * kTileRows + 1) * 8);
  uint64_t* stmp = (uint64_t*)p;
  const uint64_t* carry = nullptr;
  int buf = 0;
  const uint64_t chunks = tiles_all ? (tiles_all + chunk - 1) / chunk : 1;
  // write_only: the masks and tile offsets of an earlier call on the same
  // batch are still in cscratch (one chunk only); run the write pass again.
  if (write_only && (chunks != 1 || device_sized)) return hipErrorInvalidValue;
  if (cells && !write_only) {
    ProfScope ps("query_filters", s);
    const uint32_t qb = (uint32_t)((m + 255) / 256);
    if (dim == 3)
      query_filters<3><<<qb, 256, 0, s>>>(q, delta, m, window, (QueryFilter*)qs.qfilt);
    else
      query_filters<2><<<qb, 256, 0, s>>>(q, delta, m, window, (QueryFilter*)qs.qfilt);
    if ((e = hipGetLastError()) != hipSuccess) return e;
  }
  for (uint64_t c = 0; c < chunks; ++c, buf ^= 1) {
    const uint64_t rbase = c * chunk * kCompactTileRows;
    const uint64_t nt = tiles_all - c * chunk < chunk ? (tiles_all ? tiles_all - c * chunk : 1)
                                                      : chunk;
    // A full chunk ends at its last tile; the last chunk at the capacity
    // (device-sized) or at the exact count (host-sized, a multiple of 64 rows
    // past it is never read because the kernels clamp to the count).
    const uint64_t row_end = c + 1 < chunks ? rbase + nt * kCompactTileRows
                             : device_sized ? max_rows : rbase + nt * kCompactTileRows;
    const bool flag = device_sized && c + 1 == chunks;
    const uint32_t grid = (uint32_t)(nt < kCompactGrid ? (nt ? nt : 1) : kCompactGrid);
    if (!write_only) {
      ProfScope ps("expand_rows", s);
      expand_rows<<<(uint32_t)((nseg + 255) / 256), 256, 0, s>>>(
          qs.row_off, qs.slot_rows, qs.slot_begin, qs.slot_count, nseg, qs.ss, rbase, row_end,
          meta);
      if ((e = hipGetLastError()) != hipSuccess) return e;
    }
    if (!write_only) {
      if ((e = fill_u32(hits, 0, nt, s)) != hipSuccess) return e;
      ProfScope ps("compact_test", s);
#define SFC_TEST_K(R, I, E, D, C, W, K)                                                    \
  compact_test<R, I, E, D, C, W, K><<<grid, 256, 0, s>>>(                                  \
      q, delta, m, pts ? pts : pts_in, pts ? nullptr : ids, cells,                         \
      (const QueryFilter*)qs.qfilt, npts, meta,                                            \
      total_dev, rbase, row_end, flag, masks, hits, qs.counters,                           \
      ev ? ev->ins : nullptr, ev ? ev->era : nullptr,                                      \
      ev ? ev->qepoch : nullptr, ev ? ev->epoch : 0u)
#define SFC_TEST_W(R, I, E, D, C, W)                                                       \
  if (C && shifts) SFC_TEST_K(R, I, E, D, C, W, C);                                        \
  else SFC_TEST_K(R, I, E, D, C, W, false)
#define SFC_TEST_D(R, I, E, D, C)                                                          \
  if (window) SFC_TEST_W(R, I, E, D, C, true);                                             \
  else SFC_TEST_W(R, I, E, D, C, false)
#define SFC_TEST(R, I, E)                                                                  \
  if (dim == 3) {                                                                          \
    if (cells) SFC_TEST_D(R, I, E, 3, true);                                               \
    else SFC_TEST_D(R, I, E, 3, false);                                                    \
  } else {                                                                                 \
    if (cells) SFC_TEST_D(R, I, E, 2, true);                                               \
    else SFC_TEST_D(R, I, E, 2, false);                                                    \
  }
#define SFC_TEST_SHAPES(E)                  \
  switch (test_variant(max_rows)) {         \
    case 1: SFC_TEST(4, 4, E); break;       \
    case 2: SFC_TEST(8, 2, E); break;       \
    case 3: SFC_TEST(2, 8, E); break;       \
    case 4: SFC_TEST(1, 16, E); break;      \
    default: SFC_TEST(16, 1, E); break;     \
  }
      if (ev && ev->ins) {
        SFC_TEST_SHAPES(true)
      } else {
        SFC_TEST_SHAPES(false)
      }
#undef SFC_TEST_SHAPES
#undef SFC_TEST
#undef SFC_TEST_D
#undef SFC_TEST_W
#undef SFC_TEST_K
      if ((e = hipGetLastError()) != hipSuccess) return e;
    }
    if (!write_only &&
        (e = scan_excl_dev(hits, toff[buf], qs.counters + 12, nt, carry, stmp, s)) != hipSuccess)
      return e;
    {
      ProfScope ps("compact_write", s);
      // One lane per output (0.64 ms at 1.7e8 outputs from 6.3e8 candidates;
      // the candidate-driven version with eight-row groups took 0.72 ms).
      compact_write_out<<<grid, 256, 0, s>>>(ids, npts, meta, total_dev, rbase, row_end, masks,
                                             toff[buf], rpre, out_ids, cap, chunks == 1);
      if ((e = hipGetLastError()) != hipSuccess) return e;
    }
    {
      ProfScope ps("query_offsets", s);
      query_offsets<<<fill_blocks(m + 1), 256, 0, s>>>(qs.row_off, qs.ss, m, total_dev, rbase,
                                                        rbase + nt * kCompactTileRows, row_end,
                                                        rpre, offsets);
      if ((e = hipGetLastError()) != hipSuccess) return e;
    }
    // The chunk's total, read by the next chunk's scan.  A chunk has tiles
    // only when every chunk before it was full, so this slot is always
    // written when it is consumed.
    carry = toff[buf] + nt;
  }
  return hipSuccess;
}

}  // namespace sfc
