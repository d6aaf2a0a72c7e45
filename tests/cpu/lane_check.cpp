// Host build of the search lane of libsfc (the text the search kernel
// includes, query_lane.inc, with the helpers of query_lane.h, learned.h,
// stree.h and curve.h), for running under the address and
// undefined-behaviour sanitizers.  A C++ compiler other than the HIP one
// reads __device__ and __forceinline__ as plain inline functions, so the
// device logic runs here as host code.
//
// Reads one binary job from argv[1], writes every lane's index ranges to
// argv[2].  Job layout (little-endian, 8-byte words unless noted):
//   n, m, curve, refine, search, refine_min, ball, with_occ,
//   keys[n], q[2m] (f64), delta[m] (f64),
//   search 1 (learned): xb[4097] u32, rt[65537] u32, lp[4097] (u32 x2),
//     npieces, fk[npieces], pr[npieces] (f64 slope, i32 elo, i32 ehi),
//     ps[npieces + 1] u32, dt[2^20 + 1] u32,
//   with_occ: occ[words] u32 preceded by words.
// Output: for each query and each of its 4 lanes, (b0, e0, b1, e1) u64 and
// then nr (u32 per query) -- the same slots the kernel writes.
#include <hip/hip_runtime.h>

#include <cmath>
#include <cstdio>
#include <cstdlib>
#include <cstring>
#include <vector>

// Device builtins that the included headers name (unused by the lane code).
static inline float __fmaf_rn(float a, float b, float c) { return std::fma(a, b, c); }
static inline unsigned int __lane_id() { return 0; }

#include "query_lane.h"

using namespace sfc;

struct Slots {
  uint64_t b0, e0, b1, e1;
};

template <int CURVE, bool REFINE, int SEARCH>
void one_lane(const uint16_t* lut, const double2* q, const double* delta, uint64_t m, uint64_t j,
              int r, const uint64_t* keys, uint64_t n, const LearnedView& lv,
              const StreeView& sv, uint32_t refine_min, bool ball, const uint32_t* occ,
              Slots* out, uint32_t* nr_out) {
  const uint64_t* pairs = nullptr;
  uint64_t b0 = 0, e0 = 0, b1 = 0, e1 = 0, klo = 0, khi = 0;
  int nr = 0;
  bool bad = false;
  uint32_t fb = 0, ends = 0, pruned = 0;
  uint64_t base = 0, nn = n;
#include "query_lane.inc"
  (void)pairs;
  (void)klo;
  (void)khi;
  (void)fb;
  (void)ends;
  (void)pruned;
  if (bad) {
    std::fprintf(stderr, "invalid query %llu\n", (unsigned long long)j);
    std::exit(3);
  }
  *out = Slots{b0, e0, b1, e1};
  if (r == 0) *nr_out = (uint32_t)nr;
}

template <int CURVE, bool REFINE, int SEARCH>
void run_all(const uint16_t* lut, const double2* q, const double* delta, uint64_t m,
             const uint64_t* keys, uint64_t n, const LearnedView& lv, const StreeView& sv,
             uint32_t refine_min, bool ball, const uint32_t* occ, Slots* out, uint32_t* nr) {
  for (uint64_t j = 0; j < m; ++j)
    for (int r = 0; r < 4; ++r)
      one_lane<CURVE, REFINE, SEARCH>(lut, q, delta, m, j, r, keys, n, lv, sv, refine_min, ball,
                                      occ, &out[4 * j + r], &nr[j]);
}

template <int CURVE, bool REFINE>
void dispatch_search(int search, const uint16_t* lut, const double2* q, const double* delta,
                     uint64_t m, const uint64_t* keys, uint64_t n, const LearnedView& lv,
                     const StreeView& sv, uint32_t refine_min, bool ball, const uint32_t* occ,
                     Slots* out, uint32_t* nr) {
  if (search == 0)
    run_all<CURVE, REFINE, 0>(lut, q, delta, m, keys, n, lv, sv, refine_min, ball, occ, out, nr);
  else if (search == 1)
    run_all<CURVE, REFINE, 1>(lut, q, delta, m, keys, n, lv, sv, refine_min, ball, occ, out, nr);
  else
    run_all<CURVE, REFINE, 2>(lut, q, delta, m, keys, n, lv, sv, refine_min, ball, occ, out, nr);
}

template <typename T>
std::vector<T> take(FILE* f, uint64_t count) {
  std::vector<T> v(count);
  if (count && std::fread(v.data(), sizeof(T), count, f) != count) {
    std::fprintf(stderr, "short job file\n");
    std::exit(2);
  }
  return v;
}

int main(int argc, char** argv) {
  if (argc != 3) return 2;
  FILE* f = std::fopen(argv[1], "rb");
  if (!f) return 2;
  const std::vector<uint64_t> hdr = take<uint64_t>(f, 8);
  const uint64_t n = hdr[0], m = hdr[1];
  const int curve = (int)hdr[2], refine = (int)hdr[3], search = (int)hdr[4];
  const uint32_t refine_min = (uint32_t)hdr[5];
  const bool ball = hdr[6] != 0, with_occ = hdr[7] != 0;
  // Exactly sized arrays, so that the sanitizer sees any access past them.
  const std::vector<uint64_t> keys = take<uint64_t>(f, n);
  const std::vector<double> qv = take<double>(f, 2 * m);
  const std::vector<double> delta = take<double>(f, m);
  std::vector<double2> q(m);
  for (uint64_t j = 0; j < m; ++j) q[j] = double2{qv[2 * j], qv[2 * j + 1]};
  std::vector<uint32_t> xb, rt;
  std::vector<uint2> lp;
  std::vector<uint64_t> fk;
  std::vector<PieceRec> pr;
  std::vector<uint32_t> ps, dt;
  LearnedView lv{};
  if (search == 1) {
    xb = take<uint32_t>(f, kLeaves + 1);
    rt = take<uint32_t>(f, kRouteSlots + 1);
    lp = take<uint2>(f, kLeaves + 1);
    const uint64_t np = take<uint64_t>(f, 1)[0];
    fk = take<uint64_t>(f, np);
    pr = take<PieceRec>(f, np);
    ps = take<uint32_t>(f, np + 1);
    dt = take<uint32_t>(f, kDirectSlots + 1);
    lv = LearnedView{xb.data(), rt.data(), lp.data(), fk.data(), pr.data(), ps.data(), dt.data()};
  }
  std::vector<uint32_t> occ;
  if (with_occ) {
    const uint64_t words = take<uint64_t>(f, 1)[0];
    occ = take<uint32_t>(f, words);
  }
  std::fclose(f);
  // The static search tree: layer k+1 holds the first key of every 16-entry
  // block of layer k, up to a layer of at most 16 entries (each layer its
  // own exactly sized array).
  std::vector<std::vector<uint64_t>> layers;
  StreeView sv{};
  sv.layer[0] = keys.data();
  sv.size[0] = n;
  sv.top = 0;
  if (search == 2) {
    const std::vector<uint64_t>* below = &keys;
    layers.reserve(kStreeMaxLayers);
    while (below->size() > (size_t)kStreeFan) {
      std::vector<uint64_t> up((below->size() + kStreeFan - 1) / kStreeFan);
      for (size_t b = 0; b < up.size(); ++b) up[b] = (*below)[b * kStreeFan];
      layers.push_back(std::move(up));
      below = &layers.back();
      ++sv.top;
      sv.layer[sv.top] = below->data();
      sv.size[sv.top] = below->size();
    }
  }
  const uint16_t* lut = kHilbertLutConst.v;
  std::vector<Slots> out(4 * m);
  std::vector<uint32_t> nr(m);
  const uint32_t* occp = with_occ ? occ.data() : nullptr;
  if (curve == 0 && refine)
    dispatch_search<0, true>(search, lut, q.data(), delta.data(), m, keys.data(), n, lv, sv,
                             refine_min, ball, occp, out.data(), nr.data());
  else if (curve == 0)
    dispatch_search<0, false>(search, lut, q.data(), delta.data(), m, keys.data(), n, lv, sv,
                              refine_min, ball, occp, out.data(), nr.data());
  else if (refine)
    dispatch_search<1, true>(search, lut, q.data(), delta.data(), m, keys.data(), n, lv, sv,
                             refine_min, ball, occp, out.data(), nr.data());
  else
    dispatch_search<1, false>(search, lut, q.data(), delta.data(), m, keys.data(), n, lv, sv,
                              refine_min, ball, occp, out.data(), nr.data());
  FILE* o = std::fopen(argv[2], "wb");
  if (!o) return 2;
  std::fwrite(out.data(), sizeof(Slots), out.size(), o);
  std::fwrite(nr.data(), 4, nr.size(), o);
  std::fclose(o);
  return 0;
}
