// Fitting the learned index (router training and leaf fits), all on the GPU.
//
//   learned_sample   kSamples evenly spaced (key, rank) pairs of the sorted
//                    keys -> inputs x = top 24 key bits / 2^24, targets rank/n.
//   learned_train    one workgroup: quantile initialisation of the ramps, then
//                    Adam steps on the mean squared error over batches of 128
//                    samples (forward and backward written out below), with
//                    w1, W2, w3 projected onto >= 0 after every step so that
//                    the router stays monotone.
//   learned_bounds   first key index of every leaf: a binary search per leaf
//                    over the sorted keys, valid because routing is monotone.
//   learned_leaves   one workgroup per leaf: least-squares line of rank on
//                    key - base (FP64, centred, fixed reduction order), then
//                    the exact window of (lower bound - prediction) over every
//                    query key the leaf can receive.
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

// bounds[l] = first index whose key routes to a leaf >= l (bounds[kLeaves] = n).
__global__ __launch_bounds__(256) void learned_bounds(const uint64_t* __restrict__ keys, uint64_t n,
                                                      const float* __restrict__ P,
                                                      uint32_t* __restrict__ bounds) {
  const uint32_t l = blockIdx.x * 256 + threadIdx.x;
  if (l > (uint32_t)kLeaves) return;
  if (l == (uint32_t)kLeaves) {
    bounds[l] = (uint32_t)n;
    return;
  }
  uint64_t lo = 0, len = n;
  while (len > 0) {
    const uint64_t h = len >> 1;
    if (router_leaf(P, keys[lo + h]) < l) {
      lo += h + 1;
      len -= h + 1;
    } else {
      len = h;
    }
  }
  bounds[l] = (uint32_t)lo;
}

__device__ __forceinline__ double block_sum_f64(double v, double* s) {
  s[threadIdx.x] = v;
  __syncthreads();
  for (int o = 128; o > 0; o >>= 1) {
    if ((int)threadIdx.x < o) s[threadIdx.x] += s[threadIdx.x + o];
    __syncthreads();
  }
  const double r = s[0];
  __syncthreads();
  return r;
}

__device__ __forceinline__ int64_t block_min_i64(int64_t v, int64_t* s) {
  s[threadIdx.x] = v;
  __syncthreads();
  for (int o = 128; o > 0; o >>= 1) {
    if ((int)threadIdx.x < o) s[threadIdx.x] = min(s[threadIdx.x], s[threadIdx.x + o]);
    __syncthreads();
  }
  const int64_t r = s[0];
  __syncthreads();
  return r;
}

__device__ __forceinline__ int64_t block_max_i64(int64_t v, int64_t* s) {
  s[threadIdx.x] = v;
  __syncthreads();
  for (int o = 128; o > 0; o >>= 1) {
    if ((int)threadIdx.x < o) s[threadIdx.x] = max(s[threadIdx.x], s[threadIdx.x + o]);
    __syncthreads();
  }
  const int64_t r = s[0];
  __syncthreads();
  return r;
}

// One workgroup per leaf l: keys[S..E).
__global__ __launch_bounds__(256) void learned_leaves(const uint64_t* __restrict__ keys, uint64_t n,
                                                      const uint32_t* __restrict__ bounds,
                                                      LeafRec* __restrict__ leaves) {
#pragma clang fp contract(off)
  __shared__ double s_d[256];
  __shared__ int64_t s_i[256];
  __shared__ LeafRec s_leaf;
  const uint32_t l = blockIdx.x;
  const uint64_t S = bounds[l], E = bounds[l + 1];
  const uint32_t tid = threadIdx.x;
  if (E <= S) {
    if (tid == 0) {
      LeafRec r;
      r.base = 0;
      r.a = (double)S;
      r.b = 0.0;
      r.S = (uint32_t)S;
      r.E = (uint32_t)S;
      r.elo = 0;
      r.ehi = 0;
      leaves[l] = r;
    }
    return;
  }
  const uint64_t base = keys[S];
  const double cnt = (double)(E - S);
  // Centred least squares of r = i - S on u = key - base.
  double su = 0.0, sr = 0.0;
  for (uint64_t i = S + tid; i < E; i += 256) {
    su += (double)(keys[i] - base);
    sr += (double)(i - S);
  }
  const double mu = block_sum_f64(su, s_d) / cnt;
  const double mr = block_sum_f64(sr, s_d) / cnt;
  double cuv = 0.0, cuu = 0.0;
  for (uint64_t i = S + tid; i < E; i += 256) {
    const double du = (double)(keys[i] - base) - mu;
    const double dr = (double)(i - S) - mr;
    cuv += du * dr;
    cuu += du * du;
  }
  const double Cuv = block_sum_f64(cuv, s_d);
  const double Cuu = block_sum_f64(cuu, s_d);
  const double b = Cuu > 0.0 ? Cuv / Cuu : 0.0;
  const double a = (double)S + mr - b * mu;
  if (tid == 0) {
    s_leaf.base = base;
    s_leaf.a = a;
    s_leaf.b = b;
    s_leaf.S = (uint32_t)S;
    s_leaf.E = (uint32_t)E;
    s_leaf.elo = 0;
    s_leaf.ehi = 0;
  }
  __syncthreads();
  const LeafRec L = s_leaf;
  // Window: a query key k routed here has its lower bound LB in [S, E].  For
  // k in (keys[i-1], keys[i]] with i the first index of its key, LB = i and
  // the prediction lies between pred(keys[i-1] + 1) and pred(keys[i]); for k
  // above the leaf's last key, LB = E and the prediction lies between
  // pred(last + 1) and E.
  int64_t lo = 0, hi = 0;
  for (uint64_t i = S + tid; i < E; i += 256) {
    const uint64_t k = keys[i];
    if (i > 0 && keys[i - 1] == k) continue;
    const int64_t ii = (int64_t)i;
    lo = min(lo, ii - leaf_predict(L, k));
    const uint64_t kprev = i > 0 ? keys[i - 1] + 1 : 0;
    hi = max(hi, ii - leaf_predict(L, kprev));
  }
  if (tid == 0 && keys[E - 1] != ~0ull) hi = max(hi, (int64_t)E - leaf_predict(L, keys[E - 1] + 1));
  const int64_t elo = block_min_i64(lo, s_i);
  const int64_t ehi = block_max_i64(hi, s_i);
  if (tid == 0) {
    LeafRec r = L;
    r.elo = (int32_t)elo;
    r.ehi = (int32_t)ehi;
    leaves[l] = r;
  }
}

}  // namespace

size_t learned_scratch_bytes() { return align256(kSamples * 4) * 2 + align256((kLeaves + 1) * 4) + 256; }

hipError_t learned_fit(const uint64_t* keys, uint64_t n, uint32_t steps, float lr, float* params,
                       LeafRec* leaves, void* scratch, float* losses, hipStream_t s) {
  if (n == 0) return hipErrorInvalidValue;
  uint32_t S = kSamples;
  while ((uint64_t)S > n) S >>= 1;
  char* p = (char*)scratch;
  float* xs = (float*)p;          p += align256(kSamples * 4);
  float* ts = (float*)p;          p += align256(kSamples * 4);
  uint32_t* bounds = (uint32_t*)p;
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
    ProfScope ps("learned_bounds", s);
    learned_bounds<<<(kLeaves + 1 + 255) / 256, 256, 0, s>>>(keys, n, params, bounds);
    if ((e = hipGetLastError()) != hipSuccess) return e;
  }
  {
    ProfScope ps("learned_leaves", s);
    learned_leaves<<<kLeaves, 256, 0, s>>>(keys, n, bounds, leaves);
    if ((e = hipGetLastError()) != hipSuccess) return e;
  }
  return hipSuccess;
}

hipError_t learned_refit_leaves(const uint64_t* keys, uint64_t n, const float* params,
                                LeafRec* leaves, void* scratch, hipStream_t s) {
  if (n == 0) return hipErrorInvalidValue;
  char* p = (char*)scratch;
  p += 2 * align256(kSamples * 4);
  uint32_t* bounds = (uint32_t*)p;
  hipError_t e;
  {
    ProfScope ps("learned_bounds", s);
    learned_bounds<<<(kLeaves + 1 + 255) / 256, 256, 0, s>>>(keys, n, params, bounds);
    if ((e = hipGetLastError()) != hipSuccess) return e;
  }
  {
    ProfScope ps("learned_leaves", s);
    learned_leaves<<<kLeaves, 256, 0, s>>>(keys, n, bounds, leaves);
    if ((e = hipGetLastError()) != hipSuccess) return e;
  }
  return hipSuccess;
}

hipError_t learned_grad(const float* params, const float* xs, const float* ts, int cnt,
                        float* grad, float* loss, hipStream_t s) {
  if (cnt < 1 || cnt > kBatch) return hipErrorInvalidValue;
  learned_grad_kernel<<<1, kTrainThreads, 0, s>>>(params, xs, ts, cnt, grad, loss);
  return hipGetLastError();
}

}  // namespace sfc
