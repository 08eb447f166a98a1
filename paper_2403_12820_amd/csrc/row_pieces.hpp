// Halo rows as 16-byte pieces when the rows are only 4-byte aligned (every cloth at least 4 wide,
// widths or offsets not multiples of 4): a piece that would cross the right edge of the grid is
// loaded at W - 4, inside the row, and its values are moved into place in registers.
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

// Element k of the result is element min(k + sh, 3) of p (sh >= 0). For the piece of columns
// col .. col + 3 loaded from b = min(col, W - 4), sh = col - b puts column min(col + k, W - 1) at k.
__device__ __forceinline__ float4 shift_clamped(float4 p, int sh) {
  float4 r;
  r.x = sh == 0 ? p.x : (sh == 1 ? p.y : (sh == 2 ? p.z : p.w));
  r.y = sh == 0 ? p.y : (sh == 1 ? p.z : p.w);
  r.z = sh == 0 ? p.z : p.w;
  r.w = p.w;
  return r;
}

// Smallest width of a plan's cloths (host arrays).
inline int plan_min_width(const int32_t* W, int n) {
  int m = W[0];
  for (int b = 1; b < n; ++b) m = W[b] < m ? W[b] : m;
  return m;
}

}  // namespace pecnn
