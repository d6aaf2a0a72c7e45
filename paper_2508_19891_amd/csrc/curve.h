// Curve keys on the device: quantisation, Z-order (Alg. 2) and Hilbert
// (Sec. 2.1 "Choice of RSFC"), both as labels in the sense of Def. 3.
#pragma once

#include <hip/hip_runtime.h>

#include <cstdint>

namespace sfc {

constexpr double kTwo32 = 4294967296.0;   // 2^32

// Grid cell of a coordinate in [0,1): floor(v * 2^32).  The scaling by a
// power of two is exact, so the product is below 2^32 for every v < 1.
__host__ __device__ __forceinline__ uint32_t quantize(double v) {
  return (uint32_t)__builtin_floor(v * kTwo32);
}

__host__ __device__ __forceinline__ bool in_unit(double v) { return v >= 0.0 && v < 1.0; }

// Spreads the 32 bits of v to the even bit positions of a 64-bit word.
__host__ __device__ __forceinline__ uint64_t spread_bits(uint32_t v) {
  uint64_t x = v;
  x = (x | (x << 16)) & 0x0000FFFF0000FFFFull;
  x = (x | (x << 8)) & 0x00FF00FF00FF00FFull;
  x = (x | (x << 4)) & 0x0F0F0F0F0F0F0F0Full;
  x = (x | (x << 2)) & 0x3333333333333333ull;
  x = (x | (x << 1)) & 0x5555555555555555ull;
  return x;
}

// Z-order: x's bit i at key bit 2i, y's bit i at key bit 2i+1.
__host__ __device__ __forceinline__ uint64_t morton_key(uint32_t x, uint32_t y) {
  return spread_bits(x) | (spread_bits(y) << 1);
}

// Three dimensions (the d-dimensional Morton code of Sec. 1 / Sec. 2.1 for
// d = 3): 21 bits per axis, cell floor(v * 2^21); x's bit i at key bit 3i,
// y's at 3i+1, z's at 3i+2 (a 63-bit key).
constexpr double kTwo21 = 2097152.0;   // 2^21
constexpr uint32_t kMaxCell3 = 2097151u;

__host__ __device__ __forceinline__ uint32_t quantize3(double v) {
  return (uint32_t)__builtin_floor(v * kTwo21);
}

// Spreads the low 21 bits of v to every third bit position.
__host__ __device__ __forceinline__ uint64_t spread_bits3(uint32_t v) {
  uint64_t x = v & 0x1FFFFFu;
  x = (x | (x << 32)) & 0x001F00000000FFFFull;
  x = (x | (x << 16)) & 0x001F0000FF0000FFull;
  x = (x | (x << 8)) & 0x100F00F00F00F00Full;
  x = (x | (x << 4)) & 0x10C30C30C30C30C3ull;
  x = (x | (x << 2)) & 0x1249249249249249ull;
  return x;
}

__host__ __device__ __forceinline__ uint64_t morton3_key(uint32_t x, uint32_t y, uint32_t z) {
  return spread_bits3(x) | (spread_bits3(y) << 1) | (spread_bits3(z) << 2);
}

// Inverse of spread_bits: the even bits of x, packed.
__host__ __device__ __forceinline__ uint32_t compact_bits(uint64_t x) {
  x &= 0x5555555555555555ull;
  x = (x | (x >> 1)) & 0x3333333333333333ull;
  x = (x | (x >> 2)) & 0x0F0F0F0F0F0F0F0Full;
  x = (x | (x >> 4)) & 0x00FF00FF00FF00FFull;
  x = (x | (x >> 8)) & 0x0000FFFF0000FFFFull;
  x = (x | (x >> 16)) & 0x00000000FFFFFFFFull;
  return (uint32_t)x;
}

// Inverse of spread_bits3: every third bit of x, packed (21 bits).
__host__ __device__ __forceinline__ uint32_t compact_bits3(uint64_t x) {
  x &= 0x1249249249249249ull;
  x = (x | (x >> 2)) & 0x10C30C30C30C30C3ull;
  x = (x | (x >> 4)) & 0x100F00F00F00F00Full;
  x = (x | (x >> 8)) & 0x001F0000FF0000FFull;
  x = (x | (x >> 16)) & 0x001F00000000FFFFull;
  x = (x | (x >> 32)) & 0x00000000001FFFFFull;
  return (uint32_t)x;
}

// The grid cell (x, y) whose Hilbert label is key: the levels from the
// bottom up, each undoing the frame the cell's quadrant imposed (the inverse
// of the quadrant-rotation construction, whose orientation hilbert_key_lut
// follows).
__host__ __device__ __forceinline__ void hilbert_decode(uint64_t key, uint32_t& x, uint32_t& y) {
  uint32_t cx = 0, cy = 0;
  uint64_t t = key;
  for (int b = 0; b < 32; ++b) {
    const uint32_t s = 1u << b;
    const uint32_t rx = (uint32_t)(t >> 1) & 1u;
    const uint32_t ry = (uint32_t)(t ^ rx) & 1u;
    if (ry == 0) {
      if (rx == 1) {
        cx = s - 1 - cx;
        cy = s - 1 - cy;
      }
      const uint32_t tmp = cx;
      cx = cy;
      cy = tmp;
    }
    cx += s * rx;
    cy += s * ry;
    t >>= 2;
  }
  x = cx;
  y = cy;
}

// Packed grid cell (as pack_cell2 / pack_cell3) of the point whose key is
// `key` on `curve`: the key holds the cell exactly.
__host__ __device__ __forceinline__ uint64_t cell_of_key(int curve, uint64_t key) {
  if (curve == 2)   // SFC_CURVE_MORTON3
    return (uint64_t)compact_bits3(key) | ((uint64_t)compact_bits3(key >> 1) << 21) |
           ((uint64_t)compact_bits3(key >> 2) << 42);
  uint32_t x, y;
  if (curve == 1) {   // SFC_CURVE_HILBERT
    hilbert_decode(key, x, y);
  } else {
    x = compact_bits(key);
    y = compact_bits(key >> 1);
  }
  return (uint64_t)x | ((uint64_t)y << 32);
}

// Grid cells of a point packed in one word: x | y << 32 in the plane,
// x | y << 21 | z << 42 in three dimensions (coordinates in [0,1)).
__host__ __device__ __forceinline__ uint64_t pack_cell2(double x, double y) {
  return (uint64_t)quantize(x) | ((uint64_t)quantize(y) << 32);
}
__host__ __device__ __forceinline__ uint64_t pack_cell3(double x, double y, double z) {
  return (uint64_t)quantize3(x) | ((uint64_t)quantize3(y) << 21) |
         ((uint64_t)quantize3(z) << 42);
}

// Hilbert order.  The frame of a sub-square is one of four symmetries of the
// square, kept as two bits: bit 0 = x and y exchanged, bit 1 = both
// complemented.  At each level the pair of coordinate bits is mapped into the
// frame, giving (x', y'); the sub-square's rank is 2x' + (x' xor y') (the
// order (0,0), (0,1), (1,1), (1,0)); a lower-left child (y' = 0, x' = 0)
// exchanges the axes of its frame and a lower-right child (y' = 0, x' = 1)
// exchanges and complements them.  The four symmetries commute, so frames
// compose by xor.  kHilbertLut applies four levels at once: index
// (frame << 8) | (4 x bits << 4) | (4 y bits), entry (frame' << 8) | 8 key
// bits.
struct HilbertLut {
  uint16_t v[4 * 256];
};

constexpr HilbertLut make_hilbert_lut() {
  HilbertLut t{};
  for (int f0 = 0; f0 < 4; ++f0) {
    for (int xn = 0; xn < 16; ++xn) {
      for (int yn = 0; yn < 16; ++yn) {
        int f = f0;
        int digits = 0;
        for (int b = 3; b >= 0; --b) {
          const int xb = (xn >> b) & 1;
          const int yb = (yn >> b) & 1;
          const int sw = f & 1;
          const int cp = (f >> 1) & 1;
          const int xp = (sw ? yb : xb) ^ cp;
          const int yp = (sw ? xb : yb) ^ cp;
          digits = (digits << 2) | ((xp << 1) | (xp ^ yp));
          const int low = yp == 0 ? 1 : 0;
          f ^= low | ((low & xp) << 1);
        }
        t.v[(f0 << 8) | (xn << 4) | yn] = (uint16_t)((f << 8) | digits);
      }
    }
  }
  return t;
}

// The table in constant memory (one copy per translation unit).
namespace {
__constant__ HilbertLut kHilbertLutConst = make_hilbert_lut();
}  // namespace

// Hilbert key through a lookup table (in LDS or constant memory): eight
// steps of four levels, most significant first, starting in the identity
// frame.
__host__ __device__ __forceinline__ uint64_t hilbert_key_lut(const uint16_t* lut, uint32_t x,
                                                    uint32_t y) {
  uint64_t key = 0;
  uint32_t f = 0;
#pragma unroll
  for (int s = 28; s >= 0; s -= 4) {
    const uint32_t idx = (f << 8) | (((x >> s) & 15u) << 4) | ((y >> s) & 15u);
    const uint32_t e = lut[idx];
    key = (key << 8) | (e & 0xFFu);
    f = e >> 8;
  }
  return key;
}

// The inverse table: index (frame << 8) | 8 key bits, entry
// (frame' << 8) | (4 x bits << 4) | (4 y bits) (the forward table is a
// bijection of the 256 (x, y) nibble pairs onto the 256 digit bytes in
// every frame).
constexpr HilbertLut make_hilbert_inv_lut() {
  const HilbertLut fwd = make_hilbert_lut();
  HilbertLut t{};
  for (int f0 = 0; f0 < 4; ++f0)
    for (int xy = 0; xy < 256; ++xy) {
      const int e = fwd.v[(f0 << 8) | xy];
      t.v[(f0 << 8) | (e & 0xFF)] = (uint16_t)((e & 0x300) | xy);
    }
  return t;
}

namespace {
__constant__ HilbertLut kHilbertInvLutConst = make_hilbert_inv_lut();
}  // namespace

// cell_of_key with the Hilbert labels decoded through the inverse table.
__host__ __device__ __forceinline__ void hilbert_decode_lut(const uint16_t* inv, uint64_t key,
                                                            uint32_t& x, uint32_t& y);
__host__ __device__ __forceinline__ uint64_t cell_of_key_lut(int curve, uint64_t key,
                                                             const uint16_t* inv) {
  if (curve != 1) return cell_of_key(curve, key);   // not SFC_CURVE_HILBERT
  uint32_t x, y;
  hilbert_decode_lut(inv, key, x, y);
  return (uint64_t)x | ((uint64_t)y << 32);
}

// hilbert_decode through the inverse table: eight steps of four levels,
// most significant first, starting in the identity frame.
__host__ __device__ __forceinline__ void hilbert_decode_lut(const uint16_t* inv, uint64_t key,
                                                            uint32_t& x, uint32_t& y) {
  uint32_t f = 0, cx = 0, cy = 0;
#pragma unroll
  for (int s = 56; s >= 0; s -= 8) {
    const uint32_t e = inv[(f << 8) | ((uint32_t)(key >> s) & 0xFFu)];
    cx = (cx << 4) | ((e >> 4) & 15u);
    cy = (cy << 4) | (e & 15u);
    f = e >> 8;
  }
  x = cx;
  y = cy;
}

}  // namespace sfc
