// Construction of the static search tree's upper layers (see stree.h).
#include <hip/hip_runtime.h>

#include "common.h"
#include "internal.h"
#include "stree.h"

namespace sfc {

namespace {

// layer k (1..top) entry b = keys[b * 16^k]: every upper layer straight from
// the key array, one launch for all layers.
struct StreeLayers {
  uint64_t* out[kStreeMaxLayers];
  uint64_t size[kStreeMaxLayers];
  uint64_t start[kStreeMaxLayers + 1];   // prefix of the sizes of layers 1..top
  int top;
};

__global__ __launch_bounds__(256) void stree_fill(const uint64_t* __restrict__ keys,
                                                  StreeLayers L) {
  const uint64_t total = L.start[L.top + 1];
  const uint64_t stride = (uint64_t)gridDim.x * blockDim.x;
  for (uint64_t i = (uint64_t)blockIdx.x * blockDim.x + threadIdx.x; i < total; i += stride) {
    int k = 1;
    while (i >= L.start[k + 1]) ++k;
    const uint64_t b = i - L.start[k];
    L.out[k][b] = keys[b << (4 * k)];
  }
}

}  // namespace

size_t stree_bytes(uint64_t n) {
  size_t bytes = 0;
  uint64_t sz = n;
  while (sz > (uint64_t)kStreeFan) {
    sz = (sz + kStreeFan - 1) / kStreeFan;
    bytes += align256(sz * 8);
  }
  return bytes;
}

StreeView stree_view(const uint64_t* keys, uint64_t n, void* buf) {
  StreeView v{};
  v.layer[0] = keys;
  v.size[0] = n;
  char* p = (char*)buf;
  int k = 0;
  while (v.size[k] > (uint64_t)kStreeFan) {
    const uint64_t sz = (v.size[k] + kStreeFan - 1) / kStreeFan;
    ++k;
    v.layer[k] = (const uint64_t*)p;
    v.size[k] = sz;
    p += align256(sz * 8);
  }
  v.top = k;
  return v;
}

hipError_t stree_build(const StreeView& v, hipStream_t s) {
  if (v.top == 0) return hipSuccess;
  StreeLayers L{};
  L.top = v.top;
  L.start[1] = 0;
  for (int k = 1; k <= v.top; ++k) {
    L.out[k] = const_cast<uint64_t*>(v.layer[k]);
    L.size[k] = v.size[k];
    L.start[k + 1] = L.start[k] + v.size[k];
  }
  const uint64_t total = L.start[v.top + 1];
  uint64_t blocks = (total + 255) / 256;
  if (blocks > 4096) blocks = 4096;
  ProfScope ps("stree_fill", s);
  stree_fill<<<(uint32_t)blocks, 256, 0, s>>>(v.layer[0], L);
  return hipGetLastError();
}

}  // namespace sfc
