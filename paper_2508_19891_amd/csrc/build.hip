// Construction (Sec. 2.1 "Storing P twice"; Alg. 2; Def. 3): curve keys,
// an LSD radix sort of (key, id) and the gather of the points into key order.
//
// Kernels, in launch order for n points:
//   keygen_hist    quantise, key, write keys; per-block LDS histograms of the
//                  eight 8-bit digits; zero the look-back state of the sort.
//   hist_reduce    sum the per-block histograms into one 8 x 256 table.
//   onesweep_pass  x8: one stable counting pass per digit.  Each block ranks
//                  a tile in LDS with wave64 ballots, publishes its digit
//                  counts through a decoupled look-back, and scatters the
//                  tile through LDS so that writes go out digit-contiguous.
//                  The first pass takes ids from the position (iota); the
//                  last pass also gathers the points into key order.
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

template <int CURVE>
__global__ __launch_bounds__(256) void keygen_hist(const double2* __restrict__ xy, uint64_t n,
                                                  uint64_t* __restrict__ keys,
                                                  uint32_t* __restrict__ partial,
                                                  uint32_t* __restrict__ err,
                                                  uint64_t* __restrict__ zero, uint64_t nzero) {
  __shared__ uint32_t hist[kDigits][kRadix];
  __shared__ uint16_t lut[CURVE == SFC_CURVE_HILBERT ? 1024 : 1];
  for (int i = threadIdx.x; i < kDigits * kRadix; i += blockDim.x) (&hist[0][0])[i] = 0;
  if (CURVE == SFC_CURVE_HILBERT)
    for (int i = threadIdx.x; i < 1024; i += blockDim.x) lut[i] = kHilbertLutConst.v[i];
  __syncthreads();

  const uint64_t stride = (uint64_t)gridDim.x * blockDim.x;
  bool bad = false;
  for (uint64_t i = (uint64_t)blockIdx.x * blockDim.x + threadIdx.x; i < n; i += stride) {
    const double2 p = xy[i];
    uint64_t key = 0;
    if (in_unit(p.x) && in_unit(p.y)) {
      const uint32_t ux = quantize(p.x), uy = quantize(p.y);
      key = CURVE == SFC_CURVE_HILBERT ? hilbert_key_lut(lut, ux, uy) : morton_key(ux, uy);
    } else {
      bad = true;
    }
    keys[i] = key;
#pragma unroll
    for (int d = 0; d < kDigits; ++d) atomicAdd(&hist[d][(key >> (8 * d)) & 255u], 1u);
  }
  if (__ballot(bad) != 0 && lane_id() == 0) atomicOr(err, kErrDomain);
  for (uint64_t i = (uint64_t)blockIdx.x * blockDim.x + threadIdx.x; i < nzero; i += stride)
    zero[i] = 0;
  __syncthreads();
  uint32_t* out = partial + (uint64_t)blockIdx.x * kDigits * kRadix;
  for (int i = threadIdx.x; i < kDigits * kRadix; i += blockDim.x) out[i] = (&hist[0][0])[i];
}

// hist[c] += sum over a slice of blocks of partial[b][c]; grid = (8, chunks).
__global__ __launch_bounds__(256) void hist_reduce(const uint32_t* __restrict__ partial,
                                                   uint32_t nblocks, uint32_t* __restrict__ hist) {
  const uint32_t col = blockIdx.x * 256 + threadIdx.x;   // digit position * 256 + digit
  const uint32_t chunks = gridDim.y;
  const uint32_t b0 = (uint32_t)(((uint64_t)nblocks * blockIdx.y) / chunks);
  const uint32_t b1 = (uint32_t)(((uint64_t)nblocks * (blockIdx.y + 1)) / chunks);
  uint32_t s = 0;
  for (uint32_t b = b0; b < b1; ++b) s += partial[(uint64_t)b * kDigits * kRadix + col];
  if (s) atomicAdd(&hist[col], s);
}

// Digit of an element in a pass: a byte of the key, or (SETPASS) a byte of
// the point set the element's id belongs to.  Padding (id 0xFFFFFFFF) takes
// digit 255 so that it sorts last.
template <bool SETPASS>
__device__ __forceinline__ uint32_t pass_digit(uint64_t k, uint32_t v, int shift,
                                               const uint32_t* __restrict__ set_id) {
  if (!SETPASS) return (uint32_t)(k >> shift) & 255u;
  return v == 0xFFFFFFFFu ? 255u : (set_id[v] >> shift) & 255u;
}

// One stable pass of the LSD radix sort over the digit pass_digit(...).
template <int ITEMS, bool FIRST, bool GATHER, bool SETPASS>
__global__ __launch_bounds__(kSortThreads) void onesweep_pass(
    const uint64_t* __restrict__ kin, const uint32_t* __restrict__ vin,
    uint64_t* __restrict__ kout, uint32_t* __restrict__ vout, uint64_t n, int shift,
    const uint32_t* __restrict__ hist, uint64_t* status, uint64_t* __restrict__ status_next,
    uint32_t* tile_counter, uint32_t* err, const double2* __restrict__ xy_in,
    double2* __restrict__ xy_out, const uint32_t* __restrict__ set_id) {
  constexpr int kTile = kSortThreads * ITEMS;
  __shared__ union {
    uint32_t wave_hist[kSortWaves][kRadix];
    struct {
      uint64_t k[kTile];
      uint32_t v[kTile];
    } st;
  } sm;
  __shared__ uint32_t s_local[kRadix];
  __shared__ uint32_t s_gbase[kRadix];
  __shared__ uint32_t s_tmp[kSortWaves];
  __shared__ uint32_t s_tile;

  const uint32_t tid = threadIdx.x, w = tid >> 6, l = tid & 63;
  if (tid == 0) s_tile = atomicAdd(tile_counter, 1u);
  for (uint32_t i = tid; i < kSortWaves * kRadix; i += kSortThreads) (&sm.wave_hist[0][0])[i] = 0;
  __syncthreads();
  const uint64_t tile = s_tile;
  const uint64_t base = tile * kTile;
  const uint64_t wbase = base + (uint64_t)w * (kWave * ITEMS);

  uint64_t key[ITEMS];
  uint32_t val[ITEMS];
  uint32_t rank[ITEMS];
#pragma unroll
  for (int i = 0; i < ITEMS; ++i) {
    const uint64_t idx = wbase + (uint64_t)i * kWave + l;
    if (idx < n) {
      key[i] = kin[idx];
      val[i] = FIRST ? (uint32_t)idx : vin[idx];
    } else {
      key[i] = ~0ull;   // padding sorts to the end of the last digit
      val[i] = 0xFFFFFFFFu;
    }
  }

  // Rank within the wave, in (item, lane) order: lanes holding the same digit
  // are found with eight ballots; the lowest of them bumps the wave's counter.
  volatile uint32_t* wh = sm.wave_hist[w];
  const uint64_t below_mask = lanemask_lt();
#pragma unroll
  for (int i = 0; i < ITEMS; ++i) {
    const uint32_t d = pass_digit<SETPASS>(key[i], val[i], shift, set_id);
    uint64_t match = ~0ull;
#pragma unroll
    for (int b = 0; b < 8; ++b) {
      const bool bit = (d >> b) & 1u;
      const uint64_t bal = __ballot(bit);
      match &= bit ? bal : ~bal;
    }
    const uint32_t cnt = (uint32_t)__popcll(match);
    const uint32_t below = (uint32_t)__popcll(match & below_mask);
    const uint32_t pre = wh[d];
    if (below == 0) wh[d] = pre + cnt;
    rank[i] = pre + below;
  }
  __syncthreads();

  // Thread d: tile count of digit d and per-wave exclusive bases.
  const uint32_t d = tid;
  uint32_t tot = 0;
#pragma unroll
  for (int ww = 0; ww < kSortWaves; ++ww) {
    const uint32_t c = sm.wave_hist[ww][d];
    sm.wave_hist[ww][d] = tot;
    tot += c;
  }
  if (tile > 0) st_release_agent(status + tile * kRadix + d, kFlagAggregate | tot);
  status_next[tile * kRadix + d] = 0;
  const uint32_t local = block_excl_scan256(tot, s_tmp);
  const uint32_t gstart = block_excl_scan256(hist[d], s_tmp);
  const uint64_t excl = lookback_publish(status, tile, kRadix, d, tot, err);
  s_local[d] = local;
  s_gbase[d] = gstart + (uint32_t)excl - local;
  __syncthreads();

  uint32_t lpos[ITEMS];
#pragma unroll
  for (int i = 0; i < ITEMS; ++i) {
    const uint32_t dd = pass_digit<SETPASS>(key[i], val[i], shift, set_id);
    lpos[i] = s_local[dd] + sm.wave_hist[w][dd] + rank[i];
  }
  __syncthreads();
#pragma unroll
  for (int i = 0; i < ITEMS; ++i) {
    sm.st.k[lpos[i]] = key[i];
    sm.st.v[lpos[i]] = val[i];
  }
  __syncthreads();

  const uint32_t valid = (uint32_t)((n - base) < (uint64_t)kTile ? (n - base) : (uint64_t)kTile);
  for (uint32_t j = tid; j < valid; j += kSortThreads) {
    const uint64_t k = sm.st.k[j];
    const uint32_t v = sm.st.v[j];
    const uint32_t pos = s_gbase[pass_digit<SETPASS>(k, v, shift, set_id)] + j;
    if (pos >= n || (GATHER && v >= n)) {   // cannot happen with a consistent histogram
      atomicOr(err, kErrInternal);
      continue;
    }
    kout[pos] = k;
    vout[pos] = v;
    if (GATHER) xy_out[pos] = xy_in[v];
  }
}

__global__ void gather_points(const uint32_t* __restrict__ ids, const double2* __restrict__ xy,
                              double2* __restrict__ out, uint64_t n) {
  const uint64_t i = (uint64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (i < n) out[i] = xy[ids[i]];
}

// Keys per thread of a radix pass: 8, 12 or 16.  The environment variable
// SFC_SORT_ITEMS overrides; else the autotuner's choice for this size; else 16.
int sort_items(uint64_t n) {
  static const int env = [] {
    const char* e = std::getenv("SFC_SORT_ITEMS");
    return e ? std::atoi(e) : 0;
  }();
  int k = env ? env : tuned(kTuneSortItems, n);
  return (k == 8 || k == 12) ? k : 16;
}
uint64_t sort_tile(uint64_t n) { return (uint64_t)kSortThreads * sort_items(n); }

// Set id of every input position (sets are contiguous in the input).
__global__ void fill_set_ids(const uint64_t* __restrict__ set_off, uint32_t n_sets, uint64_t n,
                             uint32_t* __restrict__ set_id) {
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

// Histograms of the set passes: hist[b][d] = points of sets whose byte b is d.
__global__ void set_histograms(const uint64_t* __restrict__ set_off, uint32_t n_sets,
                               uint32_t* __restrict__ hist) {
  const uint32_t s = blockIdx.x * blockDim.x + threadIdx.x;
  if (s >= n_sets) return;
  const uint32_t size = (uint32_t)(set_off[s + 1] - set_off[s]);
  if (size == 0) return;
  atomicAdd(&hist[s & 255u], size);
  atomicAdd(&hist[kRadix + ((s >> 8) & 255u)], size);
}

template <int ITEMS>
hipError_t launch_pass(bool first, bool gather, bool setpass, int shift, uint64_t tiles,
                       const uint64_t* kin, const uint32_t* vin, uint64_t* kout, uint32_t* vout,
                       uint64_t n, const uint32_t* hist, uint64_t* st, uint64_t* st_next,
                       uint32_t* counter, uint32_t* err, const double* xy, double* xy_out,
                       const uint32_t* set_id, hipStream_t s) {
  const dim3 g((uint32_t)tiles), b(kSortThreads);
  const double2* xi = (const double2*)xy;
  double2* xo = (double2*)xy_out;
#define SFC_PASS(F, G, S)                                                                   \
  onesweep_pass<ITEMS, F, G, S><<<g, b, 0, s>>>(kin, vin, kout, vout, n, shift, hist, st,   \
                                                st_next, counter, err, G ? xi : nullptr,    \
                                                G ? xo : nullptr, set_id)
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

}  // namespace

// Number of stable set passes after the key passes: one byte of the set
// index per pass.
int set_passes(uint32_t n_sets) { return n_sets <= 1 ? 0 : (n_sets <= 256 ? 1 : 2); }

// Device bytes of scratch needed by sort_build for n points.
size_t build_scratch_bytes(uint64_t n, uint32_t* keygen_blocks) {
  const uint64_t tiles = (n + sort_tile(n) - 1) / sort_tile(n);
  uint64_t blocks = (n + 1023) / 1024;
  if (blocks > 1024) blocks = 1024;
  if (blocks < 1) blocks = 1;
  if (keygen_blocks) *keygen_blocks = (uint32_t)blocks;
  size_t b = 0;
  b += align256(n * 8);                             // keys ping
  b += align256(n * 4);                             // ids ping
  b += align256(blocks * kDigits * kRadix * 4);     // per-block histograms
  b += align256((kDigits + 2) * kRadix * 4);        // histograms (keys, set bytes)
  b += align256(2 * tiles * kRadix * 8);            // look-back status (two buffers)
  b += align256(64);                                // counters + error word
  b += align256(n * 4);                             // set id per input point
  return b;
}

hipError_t launch_keys(const double* xy, uint64_t n, int curve, uint64_t* keys, uint32_t* err,
                       uint32_t* partial, uint32_t blocks, uint64_t* zero, uint64_t nzero,
                       hipStream_t s) {
  if (n == 0) return hipSuccess;
  ProfScope ps("keygen_hist", s);
  if (curve == SFC_CURVE_HILBERT)
    keygen_hist<SFC_CURVE_HILBERT><<<blocks, 256, 0, s>>>((const double2*)xy, n, keys, partial,
                                                          err, zero, nzero);
  else
    keygen_hist<SFC_CURVE_MORTON><<<blocks, 256, 0, s>>>((const double2*)xy, n, keys, partial,
                                                         err, zero, nzero);
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
                      hipStream_t s, const uint64_t* set_off, uint32_t n_sets) {
  if (n == 0) return hipSuccess;
  uint32_t kblocks = 0;
  build_scratch_bytes(n, &kblocks);
  const uint64_t tiles = (n + sort_tile(n) - 1) / sort_tile(n);
  char* p = (char*)scratch;
  uint64_t* keys_b = (uint64_t*)p;      p += align256(n * 8);
  uint32_t* ids_b = (uint32_t*)p;       p += align256(n * 4);
  uint32_t* partial = (uint32_t*)p;     p += align256((uint64_t)kblocks * kDigits * kRadix * 4);
  uint32_t* hist = (uint32_t*)p;        p += align256((kDigits + 2) * kRadix * 4);
  uint64_t* status = (uint64_t*)p;      p += align256(2 * tiles * kRadix * 8);
  uint32_t* counters = (uint32_t*)p;    p += align256(64);   // tile counter per pass
  uint32_t* set_id = (uint32_t*)p;

  const int sp = set_off ? set_passes(n_sets) : 0;
  const int passes = kDigits + sp;
  // Pass p writes the output buffers when passes - 1 - p is even, so that the
  // last pass lands in them; the keys are generated into the other buffer.
  auto out_is_final = [&](int pass) { return ((passes - 1 - pass) & 1) == 0; };
  uint64_t* keys_first = out_is_final(0) ? keys_b : keys_out;

  hipError_t e;
  // The first look-back buffer is zeroed by keygen_hist, the second by the
  // first pass.
  if ((e = fill_u32(hist, 0, (kDigits + 2) * kRadix, s)) != hipSuccess) return e;
  if ((e = fill_u32(counters, 0, 16, s)) != hipSuccess) return e;
  e = launch_keys(xy, n, curve, keys_first, err_host_visible, partial, kblocks, status,
                  tiles * kRadix, s);
  if (e != hipSuccess) return e;
  {
    ProfScope ps("hist_reduce", s);
    const uint32_t chunks = kblocks < 16 ? kblocks : 16;
    hist_reduce<<<dim3(kDigits, chunks), 256, 0, s>>>(partial, kblocks, hist);
    if ((e = hipGetLastError()) != hipSuccess) return e;
  }
  if (sp > 0) {
    ProfScope ps("set_prep", s);
    fill_set_ids<<<(uint32_t)((n + 255) / 256), 256, 0, s>>>(set_off, n_sets, n, set_id);
    set_histograms<<<(n_sets + 255) / 256, 256, 0, s>>>(set_off, n_sets, hist + kDigits * kRadix);
    if ((e = hipGetLastError()) != hipSuccess) return e;
  }
  const uint64_t* kin = keys_first;
  const uint32_t* vin = nullptr;
  for (int pass = 0; pass < passes; ++pass) {
    const bool fin = out_is_final(pass);
    uint64_t* kout = fin ? keys_out : keys_b;
    uint32_t* vout = fin ? ids_out : ids_b;
    uint64_t* st = status + (uint64_t)(pass & 1) * tiles * kRadix;
    uint64_t* st_next = status + (uint64_t)((pass + 1) & 1) * tiles * kRadix;
    const bool setpass = pass >= kDigits;
    const int shift = setpass ? 8 * (pass - kDigits) : 8 * pass;
    const bool gather = pass == passes - 1;
    ProfScope ps(setpass ? "set_pass" : "onesweep_pass", s);
    const uint32_t* hp = hist + pass * kRadix;
#define SFC_LAUNCH(I)                                                                          \
  launch_pass<I>(pass == 0, gather, setpass, shift, tiles, kin, vin, kout, vout, n, hp, st,   \
                 st_next, counters + pass, err_host_visible, xy, xy_out, set_id, s)
    switch (sort_items(n)) {
      case 16: e = SFC_LAUNCH(16); break;
      case 12: e = SFC_LAUNCH(12); break;
      default: e = SFC_LAUNCH(8); break;
    }
#undef SFC_LAUNCH
    if (e != hipSuccess) return e;
    kin = kout;
    vin = vout;
  }
  return hipSuccess;
}

hipError_t gather_sorted(const uint32_t* ids, const double* xy, double* out, uint64_t n,
                         hipStream_t s) {
  if (n == 0) return hipSuccess;
  ProfScope ps("gather_points", s);
  gather_points<<<(uint32_t)((n + 255) / 256), 256, 0, s>>>(ids, (const double2*)xy,
                                                             (double2*)out, n);
  return hipGetLastError();
}

}  // namespace sfc
