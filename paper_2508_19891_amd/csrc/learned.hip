// Fitting the learned index (router training and leaf fits), all on the GPU.
//
//   learned_sample   kSamples evenly spaced (key, rank) pairs of the sorted
//                    keys -> inputs x = top 24 key bits / 2^24, targets rank/n.
//   learned_train    one workgroup: quantile initialisation of the ramps, then
//                    Adam steps on the mean squared error over batches of 128
//                    samples (forward and backward written out below), with
//                    w1, W2, w3 projected onto >= 0 after every step so that
//                    the router stays monotone.
//   learned_xbounds  tabulation of the trained router: the first input X of
//   learned_radix    every leaf (a binary search over X per leaf, valid
//                    because routing is monotone) and the leaf at every
//                    2^8-th input.
//   learned_keybounds first key index of every leaf.
//   learned_piece_offsets  pieces per leaf (ceil(size / kPiece)) and their
//                    exclusive scan (one workgroup).
//   learned_pieces   one wave per piece: first key, interpolation slope and
//                    the exact window of (lower bound - prediction) over every
//                    query key the piece can receive.
#include <hip/hip_runtime.h>

#include "common.h"
#include "internal.h"
#include "learned.h"

namespace sfc {
namespace {

constexpr int kBatch = 128;
constexpr int kTrainThreads = 256;

__device__ __forceinline__ float clip01(float v) { return fminf(fmaxf(v, 0.f), 1.f); }
__device__ __forceinline__ float inside01(float v) { return (v > 0.f && v < 1.f) ? 1.f : 0.f; }

// Gradient of the batch's mean squared error, written into G (kParams, LDS),
// for parameters P (LDS).  Threads 0..cnt-1 hold one sample each (x, t);
// sh1 and sd2 are LDS scratch [kBatch][kHidden + 1].  Returns the batch loss
// in every thread.  The summation order is fixed, so the result does not
// depend on timing.
__device__ float batch_gradient(const float* P, float* G, float x, float t, int cnt,
                                float (*sh1)[kHidden + 1], float (*sd2)[kHidden + 1],
                                float* s_red) {
  const int tid = threadIdx.x;
  const bool mine = tid < cnt;
  float a1[kHidden], a2[kHidden];
  float g = 0.f, y = 0.f;
  if (mine) {
#pragma unroll
    for (int j = 0; j < kHidden; ++j) a1[j] = __fmaf_rn(P[kOffW1 + j], x, P[kOffB1 + j]);
    y = P[kOffB3];
#pragma unroll
    for (int i = 0; i < kHidden; ++i) {
      float a = P[kOffB2 + i];
#pragma unroll
      for (int j = 0; j < kHidden; ++j)
        a = __fmaf_rn(P[kOffW2 + i * kHidden + j], clip01(a1[j]), a);
      a2[i] = a;
      y = __fmaf_rn(P[kOffW3 + i], clip01(a), y);
    }
    g = 2.f * (y - t) / (float)cnt;
#pragma unroll
    for (int j = 0; j < kHidden; ++j) sh1[tid][j] = clip01(a1[j]);
#pragma unroll
    for (int i = 0; i < kHidden; ++i) sd2[tid][i] = g * P[kOffW3 + i] * inside01(a2[i]);
  }
  // Batch loss (fixed tree over LDS).
  s_red[tid] = mine ? (y - t) * (y - t) : 0.f;
  __syncthreads();
  for (int o = kTrainThreads / 2; o > 0; o >>= 1) {
    if (tid < o) s_red[tid] += s_red[tid + o];
    __syncthreads();
  }
  const float loss = s_red[0] / (float)(cnt > 0 ? cnt : 1);
  __syncthreads();

  // dW2[i][j] = sum_b d2[b][i] h1[b][j]; db2[i] = sum_b d2[b][i].
  for (int e = tid; e < kHidden * kHidden; e += kTrainThreads) {
    const int i = e / kHidden, j = e % kHidden;
    float acc = 0.f;
    for (int b = 0; b < cnt; ++b) acc = __fmaf_rn(sd2[b][i], sh1[b][j], acc);
    G[kOffW2 + e] = acc;
  }
  if (tid < kHidden) {
    float acc = 0.f;
    for (int b = 0; b < cnt; ++b) acc += sd2[b][tid];
    G[kOffB2 + tid] = acc;
  }
  __syncthreads();

  // Second phase: reuse the scratch for d1 = (W2^T d2) * clip'(a1) and
  // e = g * h2 (for dw3).
  float d1[kHidden], e3[kHidden];
  if (mine) {
#pragma unroll
    for (int j = 0; j < kHidden; ++j) d1[j] = 0.f;
#pragma unroll
    for (int i = 0; i < kHidden; ++i) {
      const float di = sd2[tid][i];
#pragma unroll
      for (int j = 0; j < kHidden; ++j) d1[j] = __fmaf_rn(di, P[kOffW2 + i * kHidden + j], d1[j]);
      e3[i] = g * clip01(a2[i]);
    }
#pragma unroll
    for (int j = 0; j < kHidden; ++j) d1[j] *= inside01(a1[j]);
  }
  __syncthreads();
  if (mine) {
#pragma unroll
    for (int j = 0; j < kHidden; ++j) {
      sh1[tid][j] = d1[j] * x;   // contribution to dw1
      sd2[tid][j] = d1[j];       // contribution to db1
    }
  }
  __syncthreads();
  if (tid < kHidden) {
    float aw = 0.f, ab = 0.f;
    for (int b = 0; b < cnt; ++b) {
      aw += sh1[b][tid];
      ab += sd2[b][tid];
    }
    G[kOffW1 + tid] = aw;
    G[kOffB1 + tid] = ab;
  }
  __syncthreads();
  if (mine) {
#pragma unroll
    for (int i = 0; i < kHidden; ++i) sh1[tid][i] = e3[i];
    sd2[tid][0] = g;
  }
  __syncthreads();
  if (tid < kHidden) {
    float acc = 0.f;
    for (int b = 0; b < cnt; ++b) acc += sh1[b][tid];
    G[kOffW3 + tid] = acc;
  }
  if (tid == kHidden) {
    float acc = 0.f;
    for (int b = 0; b < cnt; ++b) acc += sd2[b][0];
    G[kOffB3] = acc;
  }
  __syncthreads();
  return loss;
}

__global__ __launch_bounds__(kTrainThreads) void learned_grad_kernel(const float* __restrict__ p_in,
                                                                     const float* __restrict__ xs,
                                                                     const float* __restrict__ ts,
                                                                     int cnt,
                                                                     float* __restrict__ g_out,
                                                                     float* __restrict__ loss_out) {
  __shared__ float P[kParams], G[kParams];
  __shared__ float sh1[kBatch][kHidden + 1], sd2[kBatch][kHidden + 1];
  __shared__ float s_red[kTrainThreads];
  for (int i = threadIdx.x; i < kParams; i += kTrainThreads) P[i] = p_in[i];
  __syncthreads();
  const int tid = threadIdx.x;
  const float x = tid < cnt ? xs[tid] : 0.f, t = tid < cnt ? ts[tid] : 0.f;
  const float loss = batch_gradient(P, G, x, t, cnt, sh1, sd2, s_red);
  for (int i = tid; i < kParams; i += kTrainThreads) g_out[i] = G[i];
  if (tid == 0) loss_out[0] = loss;
}

__global__ __launch_bounds__(256) void learned_sample(const uint64_t* __restrict__ keys, uint64_t n,
                                                      uint32_t S, float* __restrict__ xs,
                                                      float* __restrict__ ts) {
  const uint32_t s = blockIdx.x * 256 + threadIdx.x;
  if (s >= S) return;
  const uint64_t i = (uint64_t)s * n / S;
  xs[s] = router_input(keys[i]);
  ts[s] = (float)((double)i / (double)n);
}

// Mean squared error of the router over all samples (one workgroup).
__device__ float sample_loss(const float* P, const float* __restrict__ xs,
                             const float* __restrict__ ts, uint32_t S, float* s_red) {
  float acc = 0.f;
  for (uint32_t s = threadIdx.x; s < S; s += kTrainThreads) {
    const float d = router_output(P, xs[s]) - ts[s];
    acc += d * d;
  }
  s_red[threadIdx.x] = acc;
  __syncthreads();
  for (int o = kTrainThreads / 2; o > 0; o >>= 1) {
    if ((int)threadIdx.x < o) s_red[threadIdx.x] += s_red[threadIdx.x + o];
    __syncthreads();
  }
  const float r = s_red[0] / (float)S;
  __syncthreads();
  return r;
}

__global__ __launch_bounds__(kTrainThreads) void learned_train(const float* __restrict__ xs,
                                                               const float* __restrict__ ts,
                                                               uint32_t S, uint32_t steps, float lr,
                                                               float* __restrict__ p_out,
                                                               float* __restrict__ losses) {
  __shared__ float P[kParams], G[kParams], Mo[kParams], Vo[kParams];
  __shared__ float sh1[kBatch][kHidden + 1], sd2[kBatch][kHidden + 1];
  __shared__ float s_red[kTrainThreads];
  const int tid = threadIdx.x;
  // Quantile initialisation: ramp j rises from quantile j/32 to (j+1)/32 of
  // the sample inputs; identity second layer; output = mean of the ramps.
  for (int i = tid; i < kParams; i += kTrainThreads) {
    float v = 0.f;
    if (i >= kOffW2 && i < kOffB2) {
      const int e = i - kOffW2;
      v = (e / kHidden == e % kHidden) ? 1.f : 0.f;
    } else if (i >= kOffW3 && i < kOffB3) {
      v = 1.f / (float)kHidden;
    }
    P[i] = v;
    Mo[i] = 0.f;
    Vo[i] = 0.f;
  }
  if (tid < kHidden) {
    const float q0 = xs[(uint64_t)tid * S / kHidden];
    const uint64_t i1 = (uint64_t)(tid + 1) * S / kHidden;
    const float q1 = xs[i1 < S ? i1 : S - 1];
    const float span = fmaxf(q1 - q0, 0x1p-24f);
    P[kOffW1 + tid] = 1.f / span;
    P[kOffB1 + tid] = -q0 / span;
  }
  __syncthreads();
  const float loss0 = sample_loss(P, xs, ts, S, s_red);

  const float b1 = 0.9f, b2 = 0.999f, eps = 1e-8f;
  float b1t = 1.f, b2t = 1.f;
  const uint32_t mask = S - 1;   // S is a power of two
  for (uint32_t st = 0; st < steps; ++st) {
    // Batch st: samples (odd multiplier) * (st * kBatch + tid) mod S, a
    // permutation of the samples within every pass over them.
    const int cnt = kBatch;
    float x = 0.f, t = 0.f;
    if (tid < cnt) {
      const uint32_t s = (uint32_t)(((uint64_t)st * kBatch + tid) * 2654435761ull) & mask;
      x = xs[s];
      t = ts[s];
    }
    batch_gradient(P, G, x, t, cnt, sh1, sd2, s_red);
    b1t *= b1;
    b2t *= b2;
    for (int i = tid; i < kParams; i += kTrainThreads) {
      const float gi = G[i];
      Mo[i] = b1 * Mo[i] + (1.f - b1) * gi;
      Vo[i] = b2 * Vo[i] + (1.f - b2) * gi * gi;
      const float mh = Mo[i] / (1.f - b1t), vh = Vo[i] / (1.f - b2t);
      float v = P[i] - lr * mh / (sqrtf(vh) + eps);
      const bool nonneg = (i < kOffB1) || (i >= kOffW2 && i < kOffB2) || (i >= kOffW3 && i < kOffB3);
      if (nonneg) v = fmaxf(v, 0.f);
      P[i] = v;
    }
    __syncthreads();
  }
  const float loss1 = sample_loss(P, xs, ts, S, s_red);
  for (int i = tid; i < kParams; i += kTrainThreads) p_out[i] = P[i];
  if (tid == 0) {
    losses[0] = loss0;
    losses[1] = loss1;
  }
}

__global__ __launch_bounds__(256) void learned_xbounds(const float* __restrict__ P,
                                                       uint32_t* __restrict__ xb) {
  const uint32_t l = blockIdx.x * 256 + threadIdx.x;
  if (l > (uint32_t)kLeaves) return;
  if (l == 0 || l == (uint32_t)kLeaves) {
    xb[l] = l == 0 ? 0u : (1u << kXBits);
    return;
  }
  uint32_t lo = 0, len = 1u << kXBits;   // first X with leaf(X) >= l, 2^24 if none
  while (len > 0) {
    const uint32_t h = len >> 1;
    if (router_leaf_x(P, lo + h) < l) {
      lo += h + 1;
      len -= h + 1;
    } else {
      len = h;
    }
  }
  xb[l] = lo;
}

__global__ __launch_bounds__(256) void learned_radix(const float* __restrict__ P,
                                                     uint32_t* __restrict__ rt) {
  const uint32_t t = blockIdx.x * 256 + threadIdx.x;
  if (t > kRouteSlots) return;
  const uint32_t X = t < kRouteSlots ? t << (kXBits - kRouteBits) : (1u << kXBits) - 1;
  rt[t] = router_leaf_x(P, X);
}

// lp[l].x = first index whose key routes to a leaf >= l: keys route by their
// top 24 bits, so that is the lower bound of xb[l] << 40 (lp[kLeaves].x = n).
__global__ __launch_bounds__(256) void learned_keybounds(const uint64_t* __restrict__ keys,
                                                         uint64_t n,
                                                         const uint32_t* __restrict__ xb,
                                                         uint2* __restrict__ lp) {
  const uint32_t l = blockIdx.x * 256 + threadIdx.x;
  if (l > (uint32_t)kLeaves) return;
  const uint32_t X = xb[l];
  lp[l].x = (l == (uint32_t)kLeaves || X >= (1u << kXBits))
                ? (uint32_t)n
                : (uint32_t)lower_bound_in(keys, 0, n, (uint64_t)X << (64 - kXBits));
}

// lp[l].y = first piece of leaf l (lp[kLeaves].y = number of pieces); one block.
__global__ __launch_bounds__(256) void learned_piece_offsets(uint2* __restrict__ lp) {
  constexpr int kPer = kLeaves / 256;
  __shared__ uint32_t s_w[4];
  const uint32_t tid = threadIdx.x;
  uint32_t c[kPer], sum = 0;
#pragma unroll
  for (int i = 0; i < kPer; ++i) {
    const uint32_t l = tid * kPer + i;
    const uint32_t S = lp[l].x, E = lp[l + 1].x;
    const uint32_t size = E > S ? E - S : 0u;
    c[i] = (size + kPiece - 1) / kPiece;
    sum += c[i];
  }
  uint32_t x = sum;   // inclusive scan over the wave
  for (int o = 1; o < 64; o <<= 1) {
    const uint32_t y = __shfl_up(x, o, 64);
    if ((tid & 63) >= (uint32_t)o) x += y;
  }
  if ((tid & 63) == 63) s_w[tid >> 6] = x;
  __syncthreads();
  uint32_t run = x - sum;
  for (uint32_t w = 0; w < (tid >> 6); ++w) run += s_w[w];
#pragma unroll
  for (int i = 0; i < kPer; ++i) {
    lp[tid * kPer + i].y = run;
    run += c[i];
  }
  if (tid == 255) lp[kLeaves].y = run;
}

// One wave per piece j of leaf l: keys[R..Rn), R = lb[l] + (j - po[l]) * kPiece.
// The pieces of all leaves tile the sorted keys in order, so a query key k
// picks the last piece whose first key is < k: the piece receives k in
// (keys[R], kmax] (kmax: the next piece's first key, keys[Rn], or the
// largest key for the last piece), and the lower bound lies in (R, Rn].
// For i in (R, Rn) the keys in (keys[i-1], keys[i]] have lower bound i (when
// keys[i-1] < keys[i]); the keys in (keys[Rn-1], kmax] have lower bound Rn.
// The prediction is monotone in k, so each interval's extremes of
// (bound - prediction) are at its ends.
__global__ __launch_bounds__(256) void learned_pieces(const uint64_t* __restrict__ keys,
                                                      uint64_t n, const uint2* __restrict__ lp,
                                                      uint32_t max_pieces,
                                                      uint64_t* __restrict__ fk,
                                                      PieceRec* __restrict__ pr,
                                                      uint32_t* __restrict__ ps) {
#pragma clang fp contract(off)
  const uint32_t lane = threadIdx.x & 63;
  const uint32_t j = blockIdx.x * 4 + (threadIdx.x >> 6);
  const uint32_t np = lp[kLeaves].y;
  if (j >= np || j >= max_pieces) return;
  uint32_t lo = 0, hi = kLeaves - 1;   // leaf: largest l with first piece <= j
  while (lo < hi) {
    const uint32_t mid = (lo + hi + 1) >> 1;
    if (lp[mid].y <= j) lo = mid;
    else hi = mid - 1;
  }
  const uint32_t l = lo;
  const uint64_t S = lp[l].x, E = lp[l + 1].x < n ? lp[l + 1].x : n;
  const uint64_t R = S + (uint64_t)(j - lp[l].y) * kPiece;
  if (R >= E) return;   // never: pieces cover exactly their leaf
  const uint64_t Rn = R + kPiece < E ? R + kPiece : E;
  const bool last = j + 1 >= lp[l + 1].y;
  const uint64_t f = keys[R];
  const uint64_t kmax = Rn < n ? keys[Rn] : ~0ull;
  // the slope spans the piece's own keys (to the next piece's first key
  // inside the leaf)
  const double span = !last ? (double)(kmax - f) : (double)(keys[E - 1] - f) + 1.0;
  const double sl = span > 0.0 ? (double)(Rn - R) / span : 0.0;
  int64_t emin = INT64_MAX, emax = INT64_MIN;
  for (uint64_t i = R + 1 + lane; i <= Rn; i += 64) {
    uint64_t klo, khi;   // keys with lower bound i: (klo - 1, khi]
    if (i < Rn) {
      if (keys[i - 1] == keys[i]) continue;
      klo = keys[i - 1] + 1;
      khi = keys[i];
    } else {
      if (keys[Rn - 1] >= kmax) continue;
      klo = keys[Rn - 1] + 1;
      khi = kmax;
    }
    const int64_t ii = (int64_t)i;
    emin = min(emin, ii - piece_predict(sl, f, R, Rn, khi));
    emax = max(emax, ii - piece_predict(sl, f, R, Rn, klo));
  }
  for (int o = 32; o > 0; o >>= 1) {
    emin = min(emin, (int64_t)__shfl_xor(emin, o, 64));
    emax = max(emax, (int64_t)__shfl_xor(emax, o, 64));
  }
  if (lane == 0) {
    PieceRec rec;
    rec.s = sl;
    rec.elo = emin > emax ? 0 : (int32_t)emin;
    rec.ehi = emin > emax ? 0 : (int32_t)emax;
    fk[j] = f;
    pr[j] = rec;
    ps[j] = (uint32_t)R;
  }
}

// dt[t] = the number of pieces whose first key is below t << 44 (t < 2^20),
// dt[2^20] = the number of pieces; ps[pieces] = n.
__global__ __launch_bounds__(256) void learned_direct(const uint64_t* __restrict__ fk,
                                                      const uint2* __restrict__ lp, uint64_t n,
                                                      uint32_t* __restrict__ ps,
                                                      uint32_t* __restrict__ dt) {
  const uint32_t t = blockIdx.x * 256 + threadIdx.x;
  if (t > kDirectSlots) return;
  const uint32_t np = lp[kLeaves].y;
  if (t == kDirectSlots) {
    dt[t] = np;
    ps[np] = (uint32_t)n;
    return;
  }
  dt[t] = (uint32_t)lower_bound_in(fk, 0, np, (uint64_t)t << (64 - kDirectBits));
}

hipError_t fit_pieces(const uint64_t* keys, uint64_t n, const LearnedArrays& a, uint32_t max_pieces,
                      hipStream_t s) {
  hipError_t e;
  {
    ProfScope ps("learned_bounds", s);
    learned_keybounds<<<(kLeaves + 1 + 255) / 256, 256, 0, s>>>(keys, n, a.xb, a.lp);
    if ((e = hipGetLastError()) != hipSuccess) return e;
    learned_piece_offsets<<<1, 256, 0, s>>>(a.lp);
    if ((e = hipGetLastError()) != hipSuccess) return e;
  }
  {
    ProfScope ps("learned_pieces", s);
    learned_pieces<<<(max_pieces + 3) / 4, 256, 0, s>>>(keys, n, a.lp, max_pieces, a.fk, a.pr,
                                                        a.ps);
    if ((e = hipGetLastError()) != hipSuccess) return e;
    learned_direct<<<(kDirectSlots + 1 + 255) / 256, 256, 0, s>>>(a.fk, a.lp, n, a.ps, a.dt);
    if ((e = hipGetLastError()) != hipSuccess) return e;
  }
  return hipSuccess;
}

}  // namespace

size_t learned_scratch_bytes() { return align256(kSamples * 4) * 2 + 256; }

uint32_t learned_max_pieces(uint64_t n) { return (uint32_t)(n / kPiece + kLeaves + 1); }

size_t learned_model_bytes(uint64_t n) {
  const uint64_t np = learned_max_pieces(n);
  return align256((kLeaves + 1) * 4) + align256((kRouteSlots + 1) * 4) +
         align256((kLeaves + 1) * 8) + align256(np * 8) + align256(np * sizeof(PieceRec)) +
         align256((np + 1) * 4) + align256((kDirectSlots + 1) * 4);
}

LearnedArrays learned_carve(void* base, uint64_t n) {
  const uint64_t np = learned_max_pieces(n);
  char* p = (char*)base;
  LearnedArrays a;
  a.xb = (uint32_t*)p;   p += align256((kLeaves + 1) * 4);
  a.rt = (uint32_t*)p;   p += align256((kRouteSlots + 1) * 4);
  a.lp = (uint2*)p;      p += align256((kLeaves + 1) * 8);
  a.fk = (uint64_t*)p;   p += align256(np * 8);
  a.pr = (PieceRec*)p;   p += align256(np * sizeof(PieceRec));
  a.ps = (uint32_t*)p;   p += align256((np + 1) * 4);
  a.dt = (uint32_t*)p;
  a.max_pieces = (uint32_t)np;
  return a;
}

hipError_t learned_fit(const uint64_t* keys, uint64_t n, uint32_t steps, float lr, float* params,
                       const LearnedArrays& a, void* scratch, float* losses, hipStream_t s) {
  if (n == 0) return hipErrorInvalidValue;
  uint32_t S = kSamples;
  while ((uint64_t)S > n) S >>= 1;
  char* p = (char*)scratch;
  float* xs = (float*)p;          p += align256(kSamples * 4);
  float* ts = (float*)p;
  hipError_t e;
  {
    ProfScope ps("learned_sample", s);
    learned_sample<<<(S + 255) / 256, 256, 0, s>>>(keys, n, S, xs, ts);
    if ((e = hipGetLastError()) != hipSuccess) return e;
  }
  {
    ProfScope ps("learned_train", s);
    learned_train<<<1, kTrainThreads, 0, s>>>(xs, ts, S, steps, lr, params, losses);
    if ((e = hipGetLastError()) != hipSuccess) return e;
  }
  {
    ProfScope ps("learned_tabulate", s);
    learned_xbounds<<<(kLeaves + 1 + 255) / 256, 256, 0, s>>>(params, a.xb);
    if ((e = hipGetLastError()) != hipSuccess) return e;
    learned_radix<<<(kRouteSlots + 1 + 255) / 256, 256, 0, s>>>(params, a.rt);
    if ((e = hipGetLastError()) != hipSuccess) return e;
  }
  return fit_pieces(keys, n, a, a.max_pieces, s);
}

hipError_t learned_refit_leaves(const uint64_t* keys, uint64_t n, const LearnedArrays& a,
                                hipStream_t s) {
  if (n == 0) return hipErrorInvalidValue;
  return fit_pieces(keys, n, a, a.max_pieces, s);
}

hipError_t learned_grad(const float* params, const float* xs, const float* ts, int cnt,
                        float* grad, float* loss, hipStream_t s) {
  if (cnt < 1 || cnt > kBatch) return hipErrorInvalidValue;
  learned_grad_kernel<<<1, kTrainThreads, 0, s>>>(params, xs, ts, cnt, grad, loss);
  return hipGetLastError();
}

__global__ __launch_bounds__(256) void route_both_kernel(const float* __restrict__ P,
                                                         LearnedView v,
                                                         const uint64_t* __restrict__ keys,
                                                         uint64_t count, uint32_t* __restrict__ direct,
                                                         uint32_t* __restrict__ table) {
  const uint64_t i = (uint64_t)blockIdx.x * 256 + threadIdx.x;
  if (i >= count) return;
  const uint32_t X = (uint32_t)(keys[i] >> (64 - kXBits));
  direct[i] = router_leaf_x(P, X);
  table[i] = route(v, X);
}

hipError_t learned_route_both(const float* params, const LearnedArrays& a, const uint64_t* keys,
                              uint64_t count, uint32_t* direct, uint32_t* table, hipStream_t s) {
  if (count == 0) return hipSuccess;
  route_both_kernel<<<(uint32_t)((count + 255) / 256), 256, 0, s>>>(params, a.view(), keys, count,
                                                                   direct, table);
  return hipGetLastError();
}

}  // namespace sfc
