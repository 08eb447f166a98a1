// Halo rows as 16-byte pieces when the rows are only 4-byte aligned (every cloth at least 4 wide,
// widths or offsets not multiples of 4): the piece of columns col .. col + 3 is loaded from
// b = min(col, W - 4), inside the row, and staged at col like any other. In a tile that crosses
// the right edge of the grid (e = W - c0 its first off-grid column, relative to the tile), only
// the piece holding column e - 1 is out of place: it starts at 4 qs, qs = (e - 1) / 4, and holds
// global columns W - 4 .. W - 1, sh = 4 qs + 4 - e places right of where they belong. After
// staging, shift_piece_lds moves element min(k + sh, 3) to k, so that column 4 qs + k holds
// min(c0 + 4 qs + k, W - 1), the clamped value; with sh = 0 the piece is in place and column e
// takes a copy of column e - 1 (the only off-grid column a node's taps read).
#pragma once
#include <hip/hip_runtime.h>

namespace pecnn {

// 16 bytes from a float address that is only 4-byte aligned: the copy states the true alignment,
// and the target's code generator chooses the access (one 16-byte load on gfx950).
__device__ __forceinline__ float4 gld4_dword(const float* __restrict__ base, unsigned idx) {
  float4 v;
  __builtin_memcpy(&v, reinterpret_cast<const char*>(base) + idx * (unsigned)sizeof(float), sizeof(float4));
  return v;
}

// p: the first of the piece's four columns in one LDS row (the row continues past it), sh in 0..3.
// In ascending k each read is at or right of the write, so one thread shifts a row in place.
template <typename T>
__device__ __forceinline__ void shift_piece_lds(T* p, int sh) {
  if (sh == 0) {
    p[4] = p[3];
  } else {
#pragma unroll
    for (int k = 0; k < 4; ++k) p[k] = p[min(k + sh, 3)];
  }
}

// Smallest width of a plan's cloths (host arrays).
inline int plan_min_width(const int32_t* W, int n) {
  int m = W[0];
  for (int b = 1; b < n; ++b) m = W[b] < m ? W[b] : m;
  return m;
}

}  // namespace pecnn
