// Oracle for distance reporting by sorting along a space-filling curve.
//
// TEST INFRASTRUCTURE ONLY.  Nothing in the product library links, loads or
// calls this file; only the tests, the smoke check and the CPU-baseline leg of
// the benchmark do.  It shares no code, header, table or constant with the HIP
// path: it is a plain, slow, obviously correct restatement of the method.
//
// Paper: "Simpler is Faster: Practical Distance Reporting by Sorting Along a
// Space-Filling Curve" (arXiv 2508.19891).
//
//   problem        Sec. 2, Problem Statement: store P, report P within the
//                  closed ball of radius delta around q.
//   curve labels   Def. 3 (RSFC in Z^d): a cell's label is a prefix of its
//                  children's labels; a point's key is its unit cell's label.
//   Z-order        Alg. 2: bit i of x goes to key position 2i, bit i of y to
//                  position 2i+1.
//   Hilbert        Sec. 2.1 "Choice of RSFC": the ordering of the quadtree
//                  cells follows a Hilbert curve; labels come from a table.
//   cell bounds    Observation after Def. 3: every point of cell C has a key
//                  in [pi(C) o 000..., pi(C) o 111...] (inclusive).
//   cells(Q)       Definition before Alg. 1: cells C of the conceptual
//                  quadtree with |Q| <= |C| < 2|Q| that meet Q.
//   query          Alg. 1: lower_bound on each cell's first key, scan while
//                  inside the cell's key interval, test the distance.
//   sort           Sec. 2.1 "Storing P twice": points sorted by key, keys
//                  kept beside them so that queries never recompute a key.
//
// Readings where the paper is silent or inconsistent (each one is listed in
// the design notes of the repository):
//   * closed ball (<=), as in the problem statement, not Alg. 1's strict <;
//   * the scan's upper bound is inclusive (the Observation), bounded by n,
//     and reports the point id rather than the array index;
//   * coordinates are doubles in [0,1)^2; omega = 32; the quantised cell of
//     a coordinate v is floor(v * 2^32); the distance test runs on the
//     doubles, in binary64, in the fixed order
//        dx = px-qx; dy = py-qy; t = dx*dx; u = dy*dy; s = t+u; r2 = d*d;
//        accept iff s <= r2
//     with no fused multiply-add (this file is built with -ffp-contract=off);
//   * the query box is widened by w quanta on each side,
//        w = 1 + floor((|q_c| + delta) * 2^-19),
//     so that it contains every point the rounded test accepts;
//   * |Q| and |C| are side lengths; level l = ceil(log2 s) for box side s;
//   * Morton: x bits on even key positions, y bits on odd positions;
//   * Hilbert: the four-state machine in hilbert_step() below, most
//     significant level first, starting in state 0 at (0,0);
//   * ranges of adjacent cells are merged (hi + 1 == next lo);
//   * three dimensions (Sec. 1 and Sec. 2.1: the Z-order method generalises
//     to R^d through d-dimensional Morton codes): points in [0,1)^3, 21 bits
//     per axis (a 63-bit key), unit cell floor(v * 2^21); bit i of x, y, z at
//     key positions 3i, 3i+1, 3i+2; cells(Q) are the at most 8 level-l cubes
//     meeting the box; the test sums the three squares left to right,
//        s = (dx*dx + dy*dy) + dz*dz <= d*d;
//     the box widens by w = 1 + floor((|q_c| + delta) * 2^-29) quanta;
//   * square windows (Sec. 4, the experiments' queries: an axis-parallel
//     square of side delta relative to the domain): taken as the closed
//     L-infinity ball of radius r = half the side around q, accepted iff
//        dx = px-qx; dy = py-qy; |dx| <= r and |dy| <= r
//     in binary64.  The window is its own bounding square, so cells(Q) and
//     the widened box are those of the Euclidean query of radius r.
#include <algorithm>
#include <cmath>
#include <cstdint>
#include <cstring>
#include <thread>
#include <utility>
#include <vector>

namespace {

constexpr double kTwo32 = 4294967296.0;       // 2^32
constexpr double kTwo33 = 8589934592.0;       // 2^33
constexpr double kTwoM19 = 1.0 / 524288.0;    // 2^-19
constexpr int64_t kMaxCell = 4294967295LL;    // 2^32 - 1

// ---- keys -----------------------------------------------------------------

// Alg. 2 written out bit by bit: key bit 2i = bit i of x, key bit 2i+1 = bit i
// of y.
uint64_t morton(uint32_t x, uint32_t y) {
  uint64_t key = 0;
  for (int i = 0; i < 32; ++i) {
    key |= (uint64_t)((x >> i) & 1u) << (2 * i);
    key |= (uint64_t)((y >> i) & 1u) << (2 * i + 1);
  }
  return key;
}

// One level of the Hilbert ordering.  The four states are the symmetries of
// the square that keep the sub-curve's shape: 0 identity, 1 swap of x and y,
// 2 complement of both, 3 complement after swap.  For a state and the pair
// (xb, yb) of bits at the current level, returns the base-4 digit of the
// sub-square in curve order and the state its children use.
void hilbert_step(int state, int xb, int yb, int* digit, int* next) {
  // Rows: state; columns: (xb,yb) = (0,0), (0,1), (1,1), (1,0).
  static const int kDigit[4][4] = {
      {0, 1, 2, 3}, {0, 3, 2, 1}, {2, 3, 0, 1}, {2, 1, 0, 3}};
  static const int kNext[4][4] = {
      {1, 0, 0, 3}, {0, 2, 1, 1}, {2, 1, 3, 2}, {3, 3, 2, 0}};
  int col;
  if (xb == 0 && yb == 0) col = 0;
  else if (xb == 0 && yb == 1) col = 1;
  else if (xb == 1 && yb == 1) col = 2;
  else col = 3;
  *digit = kDigit[state][col];
  *next = kNext[state][col];
}

uint64_t hilbert(uint32_t x, uint32_t y) {
  uint64_t key = 0;
  int state = 0;
  for (int b = 31; b >= 0; --b) {
    int digit, next;
    hilbert_step(state, (x >> b) & 1, (y >> b) & 1, &digit, &next);
    key = (key << 2) | (uint64_t)digit;
    state = next;
  }
  return key;
}

uint64_t curve_key(int curve, uint32_t x, uint32_t y) {
  return curve == 0 ? morton(x, y) : hilbert(x, y);
}

// Quantisation of a coordinate in [0,1): the unit cell floor(v * 2^32).
// Returns false when v is outside [0,1) (NaN included).
bool quantize(double v, uint32_t* u) {
  if (!(v >= 0.0 && v < 1.0)) return false;
  double s = std::floor(v * kTwo32);   // exact scaling by a power of two
  if (s > (double)kMaxCell) s = (double)kMaxCell;
  *u = (uint32_t)s;
  return true;
}

// ---- the distance test ----------------------------------------------------

bool within(double px, double py, double qx, double qy, double delta) {
  double dx = px - qx;
  double dy = py - qy;
  double t = dx * dx;
  double u = dy * dy;
  double s = t + u;
  double r2 = delta * delta;
  return s <= r2;
}

// Metric 1: the closed axis-parallel square of half side delta around q.
bool within_window(double px, double py, double qx, double qy, double delta) {
  double dx = px - qx;
  double dy = py - qy;
  return std::fabs(dx) <= delta && std::fabs(dy) <= delta;
}

bool accept(int metric, double px, double py, double qx, double qy, double delta) {
  return metric == 1 ? within_window(px, py, qx, qy, delta) : within(px, py, qx, qy, delta);
}

bool valid_query(double qx, double qy, double delta) {
  return std::isfinite(qx) && std::isfinite(qy) && std::isfinite(delta) &&
         delta >= 0.0;
}

// ---- query box and cells(Q) ------------------------------------------------

int64_t floor_clamped(double v) {
  if (v < -kTwo33) v = -kTwo33;
  if (v > kTwo33) v = kTwo33;
  return (int64_t)std::floor(v);
}

// One axis of the widened integer box.  Returns false if it misses the
// domain [0, 2^32-1].
bool axis_box(double c, double delta, int64_t* lo, int64_t* hi) {
  double w_real = std::floor((std::fabs(c) + delta) * kTwoM19);
  if (w_real > kTwo33) w_real = kTwo33;
  int64_t w = 1 + (int64_t)w_real;
  int64_t l = floor_clamped((c - delta) * kTwo32) - w;
  int64_t h = floor_clamped((c + delta) * kTwo32) + w;
  if (l < 0) l = 0;
  if (h > kMaxCell) h = kMaxCell;
  if (l > h) return false;
  *lo = l;
  *hi = h;
  return true;
}

struct Range {
  uint64_t lo, hi;
};

// The key intervals of cells(Q) for an integer box inside the domain,
// sorted and merged.
int box_ranges(int64_t lx, int64_t hx, int64_t ly, int64_t hy, int curve,
               Range out[4]) {
  int64_t side = std::max(hx - lx + 1, hy - ly + 1);
  int level = 0;
  while (((int64_t)1 << level) < side) ++level;   // ceil(log2 side)
  if (level >= 32) {
    out[0] = Range{0, ~(uint64_t)0};
    return 1;
  }
  std::vector<Range> cells;
  for (int64_t cx = lx >> level; cx <= (hx >> level); ++cx) {
    for (int64_t cy = ly >> level; cy <= (hy >> level); ++cy) {
      uint64_t key = curve_key(curve, (uint32_t)(cx << level),
                               (uint32_t)(cy << level));
      uint64_t span = ((uint64_t)1 << (2 * level)) - 1;
      uint64_t lo = key & ~span;   // pi(C) o 000...
      cells.push_back(Range{lo, lo | span});   // pi(C) o 111...
    }
  }
  std::sort(cells.begin(), cells.end(),
            [](const Range& a, const Range& b) { return a.lo < b.lo; });
  int k = 0;
  for (const Range& r : cells) {
    if (k > 0 && out[k - 1].hi != ~(uint64_t)0 && out[k - 1].hi + 1 == r.lo) {
      out[k - 1].hi = r.hi;
    } else {
      out[k++] = r;
    }
  }
  return k;
}

// The key intervals of cells(Q) for the widened box of a query.
int ranges(double qx, double qy, double delta, int curve, Range out[4]) {
  int64_t lx, hx, ly, hy;
  if (!axis_box(qx, delta, &lx, &hx)) return 0;
  if (!axis_box(qy, delta, &ly, &hy)) return 0;
  return box_ranges(lx, hx, ly, hy, curve, out);
}

// Alg. 1 for one query: report ids in array order within each key range.
void query_one(const uint64_t* keys, const uint32_t* ids, const double* xy,
               uint64_t n, double qx, double qy, double delta, int curve, int metric,
               std::vector<uint32_t>* out) {
  Range r[4];
  int k = ranges(qx, qy, delta, curve, r);
  for (int i = 0; i < k; ++i) {
    const uint64_t* b = std::lower_bound(keys, keys + n, r[i].lo);
    const uint64_t* e = std::upper_bound(keys, keys + n, r[i].hi);
    for (const uint64_t* p = b; p < e; ++p) {
      uint64_t j = (uint64_t)(p - keys);
      if (accept(metric, xy[2 * j], xy[2 * j + 1], qx, qy, delta)) out->push_back(ids[j]);
    }
  }
}

// ---- three dimensions --------------------------------------------------------

constexpr double kTwo21 = 2097152.0;            // 2^21
constexpr double kTwo22 = 4194304.0;            // 2^22
constexpr double kTwoM29 = 1.0 / 536870912.0;   // 2^-29
constexpr int64_t kMaxCell3 = 2097151;          // 2^21 - 1

bool quantize3(double v, uint32_t* u) {
  if (!(v >= 0.0 && v < 1.0)) return false;
  double s = std::floor(v * kTwo21);
  if (s > (double)kMaxCell3) s = (double)kMaxCell3;
  *u = (uint32_t)s;
  return true;
}

// The d = 3 Morton code, bit by bit: x bit i -> key bit 3i, y -> 3i+1,
// z -> 3i+2.
uint64_t morton3(uint32_t x, uint32_t y, uint32_t z) {
  uint64_t key = 0;
  for (int i = 0; i < 21; ++i) {
    key |= (uint64_t)((x >> i) & 1u) << (3 * i);
    key |= (uint64_t)((y >> i) & 1u) << (3 * i + 1);
    key |= (uint64_t)((z >> i) & 1u) << (3 * i + 2);
  }
  return key;
}

bool within3(const double* p, const double* q, double delta) {
  double dx = p[0] - q[0];
  double dy = p[1] - q[1];
  double dz = p[2] - q[2];
  double t = dx * dx;
  double u = dy * dy;
  double v = dz * dz;
  double s = t + u;
  s = s + v;
  double r2 = delta * delta;
  return s <= r2;
}

bool within_window3(const double* p, const double* q, double delta) {
  double dx = p[0] - q[0];
  double dy = p[1] - q[1];
  double dz = p[2] - q[2];
  return std::fabs(dx) <= delta && std::fabs(dy) <= delta && std::fabs(dz) <= delta;
}

bool valid_query3(const double* q, double delta) {
  return std::isfinite(q[0]) && std::isfinite(q[1]) && std::isfinite(q[2]) &&
         std::isfinite(delta) && delta >= 0.0;
}

int64_t floor_clamped3(double v) {
  if (v < -kTwo22) v = -kTwo22;
  if (v > kTwo22) v = kTwo22;
  return (int64_t)std::floor(v);
}

bool axis_box3(double c, double delta, int64_t* lo, int64_t* hi) {
  double w_real = std::floor((std::fabs(c) + delta) * kTwoM29);
  if (w_real > kTwo22) w_real = kTwo22;
  int64_t w = 1 + (int64_t)w_real;
  int64_t l = floor_clamped3((c - delta) * kTwo21) - w;
  int64_t h = floor_clamped3((c + delta) * kTwo21) + w;
  if (l < 0) l = 0;
  if (h > kMaxCell3) h = kMaxCell3;
  if (l > h) return false;
  *lo = l;
  *hi = h;
  return true;
}

// Key intervals of the level-l cubes meeting the box b = {lx,hx,ly,hy,lz,hz},
// sorted and merged (at most 8).
int box_ranges3(const int64_t* b, Range out[8]) {
  int64_t side = std::max(b[1] - b[0] + 1, std::max(b[3] - b[2] + 1, b[5] - b[4] + 1));
  int level = 0;
  while (((int64_t)1 << level) < side) ++level;
  if (level >= 21) {
    out[0] = Range{0, ((uint64_t)1 << 63) - 1};
    return 1;
  }
  std::vector<Range> cells;
  const uint64_t span = ((uint64_t)1 << (3 * level)) - 1;
  for (int64_t cx = b[0] >> level; cx <= (b[1] >> level); ++cx)
    for (int64_t cy = b[2] >> level; cy <= (b[3] >> level); ++cy)
      for (int64_t cz = b[4] >> level; cz <= (b[5] >> level); ++cz) {
        uint64_t key = morton3((uint32_t)(cx << level), (uint32_t)(cy << level),
                               (uint32_t)(cz << level));
        cells.push_back(Range{key & ~span, (key & ~span) | span});
      }
  std::sort(cells.begin(), cells.end(),
            [](const Range& a, const Range& c) { return a.lo < c.lo; });
  int k = 0;
  for (const Range& r : cells) {
    if (k > 0 && out[k - 1].hi + 1 == r.lo) {
      out[k - 1].hi = r.hi;
    } else {
      out[k++] = r;
    }
  }
  return k;
}

int ranges3(const double* q, double delta, Range out[8]) {
  int64_t b[6];
  for (int a = 0; a < 3; ++a)
    if (!axis_box3(q[a], delta, &b[2 * a], &b[2 * a + 1])) return 0;
  return box_ranges3(b, out);
}

void query3_one(const uint64_t* keys, const uint32_t* ids, const double* xyz, uint64_t n,
                const double* q, double delta, int metric, std::vector<uint32_t>* out) {
  Range r[8];
  int k = ranges3(q, delta, r);
  for (int i = 0; i < k; ++i) {
    const uint64_t* b = std::lower_bound(keys, keys + n, r[i].lo);
    const uint64_t* e = std::upper_bound(keys, keys + n, r[i].hi);
    for (const uint64_t* p = b; p < e; ++p) {
      uint64_t j = (uint64_t)(p - keys);
      bool hit = metric == 1 ? within_window3(xyz + 3 * j, q, delta)
                             : within3(xyz + 3 * j, q, delta);
      if (hit) out->push_back(ids[j]);
    }
  }
}

}  // namespace

extern "C" {

uint64_t oracle_morton3(uint32_t x, uint32_t y, uint32_t z) { return morton3(x, y, z); }

// Keys of n points (xyz interleaved).  Returns 0, or -2 for a coordinate
// outside [0,1).
int oracle_keys3(const double* xyz, uint64_t n, uint64_t* keys) {
  for (uint64_t i = 0; i < n; ++i) {
    uint32_t u[3];
    for (int a = 0; a < 3; ++a)
      if (!quantize3(xyz[3 * i + a], &u[a])) return -2;
    keys[i] = morton3(u[0], u[1], u[2]);
  }
  return 0;
}

// Sort of (key, id) pairs, then the points in that order.
int oracle_build3(const double* xyz, uint64_t n, uint64_t* keys_out, uint32_t* ids_out,
                  double* xyz_out) {
  std::vector<std::pair<uint64_t, uint32_t>> kv(n);
  for (uint64_t i = 0; i < n; ++i) {
    uint32_t u[3];
    for (int a = 0; a < 3; ++a)
      if (!quantize3(xyz[3 * i + a], &u[a])) return -2;
    kv[i] = {morton3(u[0], u[1], u[2]), (uint32_t)i};
  }
  std::sort(kv.begin(), kv.end());
  for (uint64_t i = 0; i < n; ++i) {
    keys_out[i] = kv[i].first;
    ids_out[i] = kv[i].second;
    for (int a = 0; a < 3; ++a) xyz_out[3 * i + a] = xyz[3 * (uint64_t)kv[i].second + a];
  }
  return 0;
}

// Widened integer box {lx,hx,ly,hy,lz,hz}: 1 non-empty, 0 empty, -1 invalid.
int oracle_box3(const double* q, double delta, int64_t* box) {
  if (!valid_query3(q, delta)) return -1;
  for (int a = 0; a < 3; ++a)
    if (!axis_box3(q[a], delta, &box[2 * a], &box[2 * a + 1])) return 0;
  return 1;
}

// Merged key ranges of a query (at most 8), or -1 for an invalid query.
int oracle_ranges3(const double* q, double delta, uint64_t* lo, uint64_t* hi) {
  if (!valid_query3(q, delta)) return -1;
  Range r[8];
  int k = ranges3(q, delta, r);
  for (int i = 0; i < k; ++i) {
    lo[i] = r[i].lo;
    hi[i] = r[i].hi;
  }
  return k;
}

// Merged key ranges of the cubes of an integer box inside [0, 2^21)^3, or -1.
int oracle_box_ranges3(const int64_t* box, uint64_t* lo, uint64_t* hi) {
  for (int a = 0; a < 3; ++a)
    if (box[2 * a] < 0 || box[2 * a] > box[2 * a + 1] || box[2 * a + 1] > kMaxCell3) return -1;
  Range r[8];
  int k = box_ranges3(box, r);
  for (int i = 0; i < k; ++i) {
    lo[i] = r[i].lo;
    hi[i] = r[i].hi;
  }
  return k;
}

// Batched 3-D queries over a built set; conventions as oracle_query.
int64_t oracle_query3(const uint64_t* keys, const uint32_t* ids, const double* xyz, uint64_t n,
                      const double* q, const double* delta, uint64_t m, uint64_t* offsets,
                      uint32_t* out, uint64_t cap, int nthreads, int metric) {
  if (metric != 0 && metric != 1) return -1;
  for (uint64_t j = 0; j < m; ++j)
    if (!valid_query3(q + 3 * j, delta[j])) return -1;
  if (nthreads < 1) nthreads = 1;
  std::vector<std::vector<uint32_t>> part(nthreads);
  std::vector<std::vector<uint64_t>> cnt(nthreads);
  auto work = [&](int t) {
    uint64_t a = m * (uint64_t)t / (uint64_t)nthreads;
    uint64_t b = m * (uint64_t)(t + 1) / (uint64_t)nthreads;
    for (uint64_t j = a; j < b; ++j) {
      size_t before = part[t].size();
      query3_one(keys, ids, xyz, n, q + 3 * j, delta[j], metric, &part[t]);
      cnt[t].push_back(part[t].size() - before);
    }
  };
  if (nthreads == 1) {
    work(0);
  } else {
    std::vector<std::thread> pool;
    for (int t = 0; t < nthreads; ++t) pool.emplace_back(work, t);
    for (auto& th : pool) th.join();
  }
  uint64_t total = 0, j = 0;
  for (int t = 0; t < nthreads; ++t)
    for (uint64_t c : cnt[t]) {
      offsets[j++] = total;
      total += c;
    }
  offsets[m] = total;
  if (cap >= total) {
    uint64_t at = 0;
    for (int t = 0; t < nthreads; ++t) {
      if (!part[t].empty()) std::memcpy(out + at, part[t].data(), part[t].size() * 4);
      at += part[t].size();
    }
  }
  return (int64_t)total;
}

// Brute force in 3-D, ids ascending per query.
int64_t oracle_brute3(const double* xyz, uint64_t n, const double* q, const double* delta,
                      uint64_t m, uint64_t* offsets, uint32_t* out, uint64_t cap, int metric) {
  if (metric != 0 && metric != 1) return -1;
  uint64_t total = 0;
  for (uint64_t j = 0; j < m; ++j) {
    if (!valid_query3(q + 3 * j, delta[j])) return -1;
    offsets[j] = total;
    for (uint64_t i = 0; i < n; ++i) {
      bool hit = metric == 1 ? within_window3(xyz + 3 * i, q + 3 * j, delta[j])
                             : within3(xyz + 3 * i, q + 3 * j, delta[j]);
      if (hit) {
        if (total < cap) out[total] = (uint32_t)i;
        ++total;
      }
    }
  }
  offsets[m] = total;
  return (int64_t)total;
}


uint64_t oracle_morton(uint32_t x, uint32_t y) { return morton(x, y); }
uint64_t oracle_hilbert(uint32_t x, uint32_t y) { return hilbert(x, y); }

// Quantised cells of n points (xy interleaved).  Returns 0, or -2 when a
// coordinate lies outside [0,1).
int oracle_quantize(const double* xy, uint64_t n, uint32_t* ux, uint32_t* uy) {
  for (uint64_t i = 0; i < n; ++i) {
    if (!quantize(xy[2 * i], &ux[i]) || !quantize(xy[2 * i + 1], &uy[i])) return -2;
  }
  return 0;
}

// Keys of n points.  curve 0 = Z-order, 1 = Hilbert.  Returns 0 or -2.
int oracle_keys(const double* xy, uint64_t n, int curve, uint64_t* keys) {
  for (uint64_t i = 0; i < n; ++i) {
    uint32_t ux, uy;
    if (!quantize(xy[2 * i], &ux) || !quantize(xy[2 * i + 1], &uy)) return -2;
    keys[i] = curve_key(curve, ux, uy);
  }
  return 0;
}

// Construction: keys, then a sort of (key, id) pairs in lexicographic order,
// then the points in that order.  Outputs: sorted keys, ids, xy.  Returns 0
// or -2.
int oracle_build(const double* xy, uint64_t n, int curve, uint64_t* keys_out,
                 uint32_t* ids_out, double* xy_out) {
  std::vector<std::pair<uint64_t, uint32_t>> kv(n);
  for (uint64_t i = 0; i < n; ++i) {
    uint32_t ux, uy;
    if (!quantize(xy[2 * i], &ux) || !quantize(xy[2 * i + 1], &uy)) return -2;
    kv[i] = {curve_key(curve, ux, uy), (uint32_t)i};
  }
  std::sort(kv.begin(), kv.end());
  for (uint64_t i = 0; i < n; ++i) {
    keys_out[i] = kv[i].first;
    ids_out[i] = kv[i].second;
    xy_out[2 * i] = xy[2 * (uint64_t)kv[i].second];
    xy_out[2 * i + 1] = xy[2 * (uint64_t)kv[i].second + 1];
  }
  return 0;
}

// Widened integer box of a query: box = {lo_x, hi_x, lo_y, hi_y}.  Returns 1
// for a non-empty box, 0 for an empty one, -1 for an invalid query.
int oracle_box(double qx, double qy, double delta, int64_t* box) {
  if (!valid_query(qx, qy, delta)) return -1;
  if (!axis_box(qx, delta, &box[0], &box[1])) return 0;
  if (!axis_box(qy, delta, &box[2], &box[3])) return 0;
  return 1;
}

// Merged key ranges of a query (at most 4).  Returns their number, or -1 for
// an invalid query.
int oracle_ranges(double qx, double qy, double delta, int curve, uint64_t* lo,
                  uint64_t* hi) {
  if (!valid_query(qx, qy, delta)) return -1;
  Range r[4];
  int k = ranges(qx, qy, delta, curve, r);
  for (int i = 0; i < k; ++i) {
    lo[i] = r[i].lo;
    hi[i] = r[i].hi;
  }
  return k;
}

// Merged key ranges of cells(Q) for an integer box [lx,hx] x [ly,hy] with
// 0 <= lx <= hx < 2^32 and 0 <= ly <= hy < 2^32.  Returns their number, or
// -1 for a box outside the domain.
int oracle_box_ranges(int64_t lx, int64_t hx, int64_t ly, int64_t hy, int curve,
                      uint64_t* lo, uint64_t* hi) {
  if (lx < 0 || ly < 0 || lx > hx || ly > hy || hx > kMaxCell || hy > kMaxCell)
    return -1;
  Range r[4];
  int k = box_ranges(lx, hx, ly, hy, curve, r);
  for (int i = 0; i < k; ++i) {
    lo[i] = r[i].lo;
    hi[i] = r[i].hi;
  }
  return k;
}

// Index ranges [b, e) of the merged key ranges over sorted keys: positions
// 2i and 2i+1 of be[] per range.  Returns the number of ranges or -1.
int oracle_index_ranges(const uint64_t* keys, uint64_t n, double qx, double qy,
                        double delta, int curve, uint64_t* be) {
  if (!valid_query(qx, qy, delta)) return -1;
  Range r[4];
  int k = ranges(qx, qy, delta, curve, r);
  for (int i = 0; i < k; ++i) {
    be[2 * i] = (uint64_t)(std::lower_bound(keys, keys + n, r[i].lo) - keys);
    be[2 * i + 1] = (uint64_t)(std::upper_bound(keys, keys + n, r[i].hi) - keys);
  }
  return k;
}

// Batched queries over a built (sorted) set.  Output CSR: offsets[m+1] and,
// if cap >= total, ids[total] in curve order per query.  Returns the total
// number of reports, or -1 for an invalid query.  Queries are split into
// nthreads contiguous slices whose outputs are concatenated in order.
// metric 0: Euclidean ball of radius delta; 1: square window of half side
// delta.
int64_t oracle_query(const uint64_t* keys, const uint32_t* ids, const double* xy,
                     uint64_t n, const double* q, const double* delta, uint64_t m,
                     int curve, uint64_t* offsets, uint32_t* out, uint64_t cap,
                     int nthreads, int metric) {
  if (metric != 0 && metric != 1) return -1;
  for (uint64_t j = 0; j < m; ++j)
    if (!valid_query(q[2 * j], q[2 * j + 1], delta[j])) return -1;
  if (nthreads < 1) nthreads = 1;
  std::vector<std::vector<uint32_t>> part(nthreads);
  std::vector<std::vector<uint64_t>> cnt(nthreads);
  auto work = [&](int t) {
    uint64_t a = m * (uint64_t)t / (uint64_t)nthreads;
    uint64_t b = m * (uint64_t)(t + 1) / (uint64_t)nthreads;
    for (uint64_t j = a; j < b; ++j) {
      size_t before = part[t].size();
      query_one(keys, ids, xy, n, q[2 * j], q[2 * j + 1], delta[j], curve, metric, &part[t]);
      cnt[t].push_back(part[t].size() - before);
    }
  };
  if (nthreads == 1) {
    work(0);
  } else {
    std::vector<std::thread> pool;
    for (int t = 0; t < nthreads; ++t) pool.emplace_back(work, t);
    for (auto& th : pool) th.join();
  }
  uint64_t total = 0, j = 0;
  for (int t = 0; t < nthreads; ++t) {
    for (uint64_t c : cnt[t]) {
      offsets[j++] = total;
      total += c;
    }
  }
  offsets[m] = total;
  if (cap >= total) {
    uint64_t at = 0;
    for (int t = 0; t < nthreads; ++t) {
      if (!part[t].empty()) std::memcpy(out + at, part[t].data(), part[t].size() * 4);
      at += part[t].size();
    }
  }
  return (int64_t)total;
}

// Brute force O(nm): every point against every query with the same test.
// Ids come in ascending order per query.  Same return convention as above.
int64_t oracle_brute(const double* xy, uint64_t n, const double* q,
                     const double* delta, uint64_t m, uint64_t* offsets,
                     uint32_t* out, uint64_t cap, int metric) {
  if (metric != 0 && metric != 1) return -1;
  uint64_t total = 0;
  for (uint64_t j = 0; j < m; ++j) {
    if (!valid_query(q[2 * j], q[2 * j + 1], delta[j])) return -1;
    offsets[j] = total;
    for (uint64_t i = 0; i < n; ++i) {
      if (accept(metric, xy[2 * i], xy[2 * i + 1], q[2 * j], q[2 * j + 1], delta[j])) {
        if (total < cap) out[total] = (uint32_t)i;
        ++total;
      }
    }
  }
  offsets[m] = total;
  return (int64_t)total;
}

}  // extern "C"
