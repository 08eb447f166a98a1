// The node-blocked table that the reverse pass of the CNN frame writes and its gather kernel
// reads: per node the adjoints of the im2col entries of U(S^k) (through both U(S^k) and
// U(S^k - S^{k-1})) and of U(S^k - S^{k-1}), 54 rows each in tap order c * 9 + o, then
// gdv = dLoss/d(dv) (3 rows). 32 consecutive nodes form one block of rows x 32 floats, so a row
// of a block is one 128-byte line.
#pragma once
#include <cstdint>

namespace pecnn {

constexpr int kBtRows = 111, kBtGus = 0, kBtGud = 54, kBtGdv = 108;
__host__ __device__ inline int64_t bt_node(int64_t q) { return (q >> 5) * (int64_t)kBtRows * 32 + (q & 31); }
__host__ __device__ inline int64_t bt_floats(int64_t n) { return (n + 31) / 32 * 32 * (int64_t)kBtRows; }

}  // namespace pecnn
