// Shared pieces of the CNN-cell kernels: MFMA operand types, the lane-slot maps that assign
// conv taps and channels to lanes, the parameter layout and the weight loaders.
#pragma once
#include "common.hpp"

namespace pecnn {

typedef __bf16 bf16x8 __attribute__((ext_vector_type(8)));
typedef float f32x4 __attribute__((ext_vector_type(4)));

// Tap of conv slot s (0..15) in lane group g: returns K column (c*9 + o) or -1 for padding, and
// the LDS offset (channel plane, row, column) relative to the node's centre cell.
__device__ __forceinline__ int slot_tap(int g, int s, int PL, int HX, int& lds_off) {
  int c, o;
  if (s < 8) {
    if (g >= 3) { lds_off = 0; return -1; }
    c = g;
    o = s + (s >= 4 ? 1 : 0);
  } else {
    const int idx = 8 * g + (s - 8);
    if (idx >= 27) { lds_off = 0; return -1; }
    c = 3 + idx / 9;
    o = idx % 9;
  }
  const int dy = o / 3 - 1, dx = o % 3 - 1;
  lds_off = c * PL + dy * HX + dx;
  return c * 9 + o;
}

// Channel held in D-layout slot e (0..Ch/4-1) by lane group g.
__device__ __forceinline__ int slot_channel(int g, int e) { return 16 * (e >> 2) + 4 * g + (e & 3); }

__device__ __forceinline__ float isru(float z, float alpha) {
  return z * __builtin_amdgcn_rsqf(__builtin_fmaf(alpha * z, z, 1.f));
}

template <int CH, bool BF>
struct CnnWeights;

// bf16 operands: one 16x16x32 MFMA consumes 8 slots per lane.
template <int CH>
struct CnnWeights<CH, true> {
  static constexpr int MB = CH / 16, CPL = CH / 4, NHK = (3 * CPL + 7) / 8;
  bf16x8 conv[MB][2];
  bf16x8 mix[2 * MB];
  bf16x8 head[NHK];
};
// FP32 operands: one 16x16x4 MFMA consumes 1 slot per lane.
template <int CH>
struct CnnWeights<CH, false> {
  static constexpr int MB = CH / 16, CPL = CH / 4, NHK = 3 * CPL;
  float conv[MB][16];
  float mix[2 * MB][CPL];
  float head[NHK];
};

struct ThetaOff {
  int K, A, B, WL, WN, WD, bL;
};
__host__ __device__ inline ThetaOff theta_off(int ch) {
  ThetaOff o;
  o.K = 0;
  o.A = ch * 54;
  o.B = o.A + ch * ch;
  o.WL = o.B + ch * ch;
  o.WN = o.WL + 3 * ch;
  o.WD = o.WN + 3 * ch;
  o.bL = o.WD + 3 * ch;
  return o;
}

// Head weight of slot q for output row i (< 3) in lane group g.
// REP: rows 4k+i (i < 3) of every 4-row group repeat output i, so that each lane group holds the
// whole head output of its column.
template <int CH, bool REP = false>
__device__ __forceinline__ float head_weight(const float* __restrict__ th, const ThetaOff& O, int i, int g, int q) {
  constexpr int CPL = CH / 4;
  if (REP) i &= 3;
  if (i >= 3 || q >= 3 * CPL) return 0.f;
  const int br = q / CPL, e = q % CPL;
  const int base = br == 0 ? O.WL : (br == 1 ? O.WN : O.WD);
  return th[base + i * CH + slot_channel(g, e)];
}

template <int CH>
__device__ __forceinline__ float mix_weight(const float* __restrict__ th, const ThetaOff& O, int row, int g, int e) {
  // rows 0..CH-1: A, rows CH..2CH-1: B
  const int base = row < CH ? O.A + row * CH : O.B + (row - CH) * CH;
  return th[base + slot_channel(g, e)];
}

template <int CH, bool REP = false>
__device__ void load_weights(CnnWeights<CH, true>& w, const float* __restrict__ th, int li, int g, int PL, int HX) {
  constexpr int MB = CH / 16, CPL = CH / 4, NHK = (3 * CPL + 7) / 8;
  const ThetaOff O = theta_off(CH);
#pragma unroll
  for (int mb = 0; mb < MB; ++mb)
#pragma unroll
    for (int ks = 0; ks < 2; ++ks)
#pragma unroll
      for (int e = 0; e < 8; ++e) {
        int lo;
        const int t = slot_tap(g, 8 * ks + e, PL, HX, lo);
        w.conv[mb][ks][e] = (__bf16)(t >= 0 ? th[O.K + (16 * mb + li) * 54 + t] : 0.f);
      }
#pragma unroll
  for (int mb = 0; mb < 2 * MB; ++mb)
#pragma unroll
    for (int e = 0; e < 8; ++e)
      w.mix[mb][e] = (__bf16)(e < CPL ? mix_weight<CH>(th, O, 16 * mb + li, g, e) : 0.f);
#pragma unroll
  for (int k = 0; k < NHK; ++k)
#pragma unroll
    for (int e = 0; e < 8; ++e) w.head[k][e] = (__bf16)head_weight<CH, REP>(th, O, li, g, 8 * k + e);
}

template <int CH>
__device__ void load_weights(CnnWeights<CH, false>& w, const float* __restrict__ th, int li, int g, int PL, int HX) {
  constexpr int MB = CH / 16, CPL = CH / 4, NHK = 3 * CPL;
  const ThetaOff O = theta_off(CH);
#pragma unroll
  for (int mb = 0; mb < MB; ++mb)
#pragma unroll
    for (int s = 0; s < 16; ++s) {
      int lo;
      const int t = slot_tap(g, s, PL, HX, lo);
      w.conv[mb][s] = t >= 0 ? th[O.K + (16 * mb + li) * 54 + t] : 0.f;
    }
#pragma unroll
  for (int mb = 0; mb < 2 * MB; ++mb)
#pragma unroll
    for (int e = 0; e < CPL; ++e) w.mix[mb][e] = mix_weight<CH>(th, O, 16 * mb + li, g, e);
#pragma unroll
  for (int q = 0; q < NHK; ++q) w.head[q] = head_weight<CH>(th, O, li, g, q);
}

// ---- products of one 16-node segment; all 64 lanes take part.
// conv: acc[mb] += K-block * U^T with the lane's 16 slot values u[].
template <int CH>
__device__ __forceinline__ void conv_mfma(const CnnWeights<CH, true>& w, const float* u, f32x4* acc) {
  bf16x8 b0, b1;
#pragma unroll
  for (int e = 0; e < 8; ++e) { b0[e] = (__bf16)u[e]; b1[e] = (__bf16)u[8 + e]; }
#pragma unroll
  for (int mb = 0; mb < CH / 16; ++mb) {
    acc[mb] = __builtin_amdgcn_mfma_f32_16x16x32_bf16(w.conv[mb][0], b0, acc[mb], 0, 0, 0);
    acc[mb] = __builtin_amdgcn_mfma_f32_16x16x32_bf16(w.conv[mb][1], b1, acc[mb], 0, 0, 0);
  }
}
template <int CH>
__device__ __forceinline__ void conv_mfma(const CnnWeights<CH, false>& w, const float* u, f32x4* acc) {
#pragma unroll
  for (int mb = 0; mb < CH / 16; ++mb)
#pragma unroll
    for (int s = 0; s < 16; ++s) acc[mb] = __builtin_amdgcn_mfma_f32_16x16x4f32(w.conv[mb][s], u[s], acc[mb], 0, 0, 0);
}

// mix: out[mb'] = [A; B] block * phi^T, phi given as the lane's CH/4 slot values.
template <int CH>
__device__ __forceinline__ void mix_mfma(const CnnWeights<CH, true>& w, const float* phi, f32x4* out) {
  constexpr int CPL = CH / 4;
  bf16x8 b;
#pragma unroll
  for (int e = 0; e < 8; ++e) b[e] = (__bf16)(e < CPL ? phi[e] : 0.f);
#pragma unroll
  for (int mb = 0; mb < 2 * (CH / 16); ++mb) {
    out[mb] = f32x4{0.f, 0.f, 0.f, 0.f};
    out[mb] = __builtin_amdgcn_mfma_f32_16x16x32_bf16(w.mix[mb], b, out[mb], 0, 0, 0);
  }
}
template <int CH>
__device__ __forceinline__ void mix_mfma(const CnnWeights<CH, false>& w, const float* phi, f32x4* out) {
  constexpr int CPL = CH / 4;
#pragma unroll
  for (int mb = 0; mb < 2 * (CH / 16); ++mb) {
    out[mb] = f32x4{0.f, 0.f, 0.f, 0.f};
#pragma unroll
    for (int e = 0; e < CPL; ++e) out[mb] = __builtin_amdgcn_mfma_f32_16x16x4f32(w.mix[mb][e], phi[e], out[mb], 0, 0, 0);
  }
}

// head: dv^T = W_head * F^T, F given as the lane's 3*CH/4 slot values [phi | n | d].
template <int CH>
__device__ __forceinline__ f32x4 head_mfma(const CnnWeights<CH, true>& w, const float* F) {
  constexpr int NQ = 3 * (CH / 4), NHK = (NQ + 7) / 8;
  f32x4 acc = {0.f, 0.f, 0.f, 0.f};
#pragma unroll
  for (int k = 0; k < NHK; ++k) {
    bf16x8 b;
#pragma unroll
    for (int e = 0; e < 8; ++e) b[e] = (__bf16)(8 * k + e < NQ ? F[8 * k + e] : 0.f);
    acc = __builtin_amdgcn_mfma_f32_16x16x32_bf16(w.head[k], b, acc, 0, 0, 0);
  }
  return acc;
}
template <int CH>
__device__ __forceinline__ f32x4 head_mfma(const CnnWeights<CH, false>& w, const float* F) {
  constexpr int NQ = 3 * (CH / 4);
  f32x4 acc = {0.f, 0.f, 0.f, 0.f};
#pragma unroll
  for (int q = 0; q < NQ; ++q) acc = __builtin_amdgcn_mfma_f32_16x16x4f32(w.head[q], F[q], acc, 0, 0, 0);
  return acc;
}

}  // namespace pecnn
