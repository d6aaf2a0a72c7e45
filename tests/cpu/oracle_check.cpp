// The oracle compiled with the address and undefined-behaviour sanitizers
// (its source included whole): seeded points and queries with the shapes
// that stress it -- duplicates, points on quantum edges and on the border,
// the far corner, radii of zero, tiny and larger than the square, centres
// outside the square -- built on both curves and in three dimensions; every
// query batch is compared with brute force over all points.  Prints "ok" or
// the first disagreement; any out-of-bounds access, undefined shift or
// overflow aborts.
#include "../../oracle/sfc_oracle.cpp"

#include <cstdio>
#include <random>
#include <vector>

namespace {

bool same_csr(const std::vector<uint64_t>& oa, const std::vector<uint32_t>& ia,
              const std::vector<uint64_t>& ob, std::vector<uint32_t> ib) {
  if (oa != ob) return false;
  // brute force reports ids ascending; the query in curve order
  for (size_t j = 0; j + 1 < oa.size(); ++j) {
    std::vector<uint32_t> a(ia.begin() + oa[j], ia.begin() + oa[j + 1]);
    std::sort(a.begin(), a.end());
    if (!std::equal(a.begin(), a.end(), ib.begin() + ob[j])) return false;
  }
  return true;
}

double edge(std::mt19937_64& g) {
  std::uniform_int_distribution<uint64_t> cell(0, 4294967295ull);
  const double q = (double)cell(g) / 4294967296.0;   // a quantum edge
  switch (g() % 4) {
    case 0: return q;
    case 1: return std::nextafter(q, 1.0);
    case 2: return q > 0 ? std::nextafter(q, 0.0) : q;
    default: return 1.0 - 0x1p-53;
  }
}

// A coordinate in the first or last grid cell of an aligned block of 2^s
// cells: the cells holding a key interval's first and last keys.
double corner(std::mt19937_64& g, int s) {
  const uint64_t j = 1 + g() % ((1ull << (32 - s)) - 1);
  const uint64_t cell = j * (1ull << s) - 1 + (g() & 1);
  return ((double)cell + 0.5) / 4294967296.0;
}

}  // namespace

int main() {
  std::mt19937_64 g(12345);
  std::uniform_real_distribution<double> u(0.0, 1.0);
  for (int round = 0; round < 12; ++round) {
    const uint64_t n = 1 + (g() % 5000);
    std::vector<double> xy(2 * n);
    const int levels[6] = {4, 10, 16, 20, 24, 28};
    for (uint64_t i = 0; i < n; ++i) {
      const int kind = (int)(g() % 8);
      xy[2 * i] = kind == 0 ? edge(g) : u(g);
      xy[2 * i + 1] = kind == 1 ? edge(g) : u(g);
      if (kind == 3) {   // a block corner at one of six levels
        const int s = levels[g() % 6];
        xy[2 * i] = corner(g, s);
        xy[2 * i + 1] = corner(g, s);
      }
      if (kind == 2 && i > 0) {   // a duplicate
        xy[2 * i] = xy[2 * (i - 1)];
        xy[2 * i + 1] = xy[2 * (i - 1) + 1];
      }
    }
    const uint64_t m = 400;
    std::vector<double> q(2 * m), d(m);
    for (uint64_t j = 0; j < m; ++j) {
      q[2 * j] = u(g) * 1.4 - 0.2;
      q[2 * j + 1] = u(g) * 1.4 - 0.2;
      const int kind = (int)(g() % 10);
      d[j] = kind == 0 ? 0.0 : kind == 1 ? 1e-300 : kind == 2 ? 2.0 : std::pow(10.0, -4.0 * u(g));
      if (kind == 3) {   // centred on a point
        const uint64_t p = g() % n;
        q[2 * j] = xy[2 * p];
        q[2 * j + 1] = xy[2 * p + 1];
      }
      if (kind == 5) {   // centred on a point, the box about its block's size
        const uint64_t p = g() % n;
        q[2 * j] = xy[2 * p];
        q[2 * j + 1] = xy[2 * p + 1];
        d[j] = std::ldexp(0.3 + 0.2 * u(g), levels[g() % 6] - 32);
      }
      if (kind == 4) {   // the far corner
        q[2 * j] = 1.0 - 0x1p-53;
        q[2 * j + 1] = 1.0 - 0x1p-53;
        d[j] = 1e-12;
      }
    }
    for (int metric = 0; metric < 2; ++metric) {
      std::vector<uint64_t> bo(m + 1);
      const int64_t bt = oracle_brute(xy.data(), n, q.data(), d.data(), m, bo.data(), nullptr, 0,
                                      metric);
      std::vector<uint32_t> bi(bt > 0 ? bt : 1);
      oracle_brute(xy.data(), n, q.data(), d.data(), m, bo.data(), bi.data(), bt, metric);
      bi.resize(bt);
      for (int curve = 0; curve < 2; ++curve) {
        std::vector<uint64_t> keys(n);
        std::vector<uint32_t> ids(n);
        std::vector<double> sxy(2 * n);
        if (oracle_build(xy.data(), n, curve, keys.data(), ids.data(), sxy.data()) != 0) {
          std::printf("build failed\n");
          return 1;
        }
        std::vector<uint64_t> off(m + 1);
        const int64_t tot = oracle_query(keys.data(), ids.data(), sxy.data(), n, q.data(),
                                         d.data(), m, curve, off.data(), nullptr, 0, 3, metric);
        std::vector<uint32_t> got(tot > 0 ? tot : 1);
        oracle_query(keys.data(), ids.data(), sxy.data(), n, q.data(), d.data(), m, curve,
                     off.data(), got.data(), tot, 3, metric);
        got.resize(tot);
        if (tot != bt || !same_csr(off, got, bo, bi)) {
          std::printf("disagreement: round %d curve %d metric %d\n", round, curve, metric);
          return 1;
        }
      }
    }
    // three dimensions
    std::vector<double> xyz(3 * n);
    for (auto& v : xyz) v = (g() % 7 == 0) ? edge(g) : u(g);
    std::vector<double> q3(3 * m);
    for (auto& v : q3) v = u(g) * 1.4 - 0.2;
    std::vector<uint64_t> bo(m + 1), off(m + 1);
    const int64_t bt = oracle_brute3(xyz.data(), n, q3.data(), d.data(), m, bo.data(), nullptr, 0, 0);
    std::vector<uint32_t> bi(bt > 0 ? bt : 1);
    oracle_brute3(xyz.data(), n, q3.data(), d.data(), m, bo.data(), bi.data(), bt, 0);
    bi.resize(bt);
    std::vector<uint64_t> keys(n);
    std::vector<uint32_t> ids(n);
    std::vector<double> sxyz(3 * n);
    if (oracle_build3(xyz.data(), n, keys.data(), ids.data(), sxyz.data()) != 0) return 1;
    const int64_t tot = oracle_query3(keys.data(), ids.data(), sxyz.data(), n, q3.data(), d.data(),
                                      m, off.data(), nullptr, 0, 2, 0);
    std::vector<uint32_t> got(tot > 0 ? tot : 1);
    oracle_query3(keys.data(), ids.data(), sxyz.data(), n, q3.data(), d.data(), m, off.data(),
                  got.data(), tot, 2, 0);
    got.resize(tot);
    if (tot != bt || !same_csr(off, got, bo, bi)) {
      std::printf("3-D disagreement: round %d\n", round);
      return 1;
    }
  }
  std::printf("ok\n");
  return 0;
}
