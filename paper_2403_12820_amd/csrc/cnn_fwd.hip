// Physics-embedded CNN cell, forward (section 3.2, eqs. 6 and 7, then eq. 5 as in Fig. 2).
//
// Implicit GEMM on the gfx950 matrix cores, computed transposed so that every product's
// output is already in the layout the next product consumes (no LDS transposes):
//
//   phi^T [Ch x 16 nodes] = K [Ch x 64 taps]      * U(S^k)^T [64 x 16]       (eq. 6)
//   xi^T  [Ch x 16]       = K                     * U(S^k - S^{k-1})^T
//   [a; b]^T [2Ch x 16]   = [A; B] [2Ch x Ch]     * phi^T                   (nonlinear branch)
//   dv^T  [16 x 16]       = [W_L W_N W_D] (rows 0..2) * [phi; sigma(a b); xi sigma(phi)]^T
//
// A 16x16 MFMA output gives lane l (column l%16 = node, group g = l/16) the rows 4g..4g+3 of
// each 16-row block. Feeding that register set straight back as the B operand assigns to lane
// group g the contraction slots of those rows; the weights (A operand) are loaded with the same
// slot-to-row map, so each channel is contracted exactly once whatever order the hardware uses
// inside a lane group. The same trick fixes which conv taps each lane builds: slots 0..7 of
// group g < 3 are the 8 off-centre taps of position channel g (the centre tap of a position
// channel is identically zero), slots 8..15 hold the 27 velocity taps spread over the groups.
//
// Operands are bf16 (v_mfma_f32_16x16x32_bf16, RNE conversion, FP32 accumulation) or FP32
// (v_mfma_f32_16x16x4_f32). Position taps are differenced against the centre in FP32 before
// the cast, so bf16 sees spacings of order h rather than absolute positions.
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
  return z * __builtin_amdgcn_rsqf(1.f + alpha * z * z);
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
template <int CH>
__device__ __forceinline__ float head_weight(const float* __restrict__ th, const ThetaOff& O, int i, int g, int q) {
  constexpr int CPL = CH / 4;
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

template <int CH>
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
    for (int e = 0; e < 8; ++e) w.head[k][e] = (__bf16)head_weight<CH>(th, O, li, g, 8 * k + e);
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

template <int CH, bool BF, int TX, int TY>
__global__ __launch_bounds__(256) void cnn_fwd_kernel(
    const InstDev* __restrict__ inst, const int32_t* __restrict__ prefix, int n_inst, int n_tiles,
    const uint8_t* __restrict__ pin, const float* __restrict__ s_prev, const float* __restrict__ s_cur,
    float* __restrict__ s_next, int64_t N, const float* __restrict__ theta, float dt, float alpha,
    const int32_t* __restrict__ skip) {
  constexpr int HX = TX + 2, HY = TY + 2, PL = HX * HY;
  constexpr int MB = CH / 16, CPL = CH / 4;
  constexpr int SEGX = TX / 16, NSEG = SEGX * TY;
  __shared__ float tS[6 * PL];
  __shared__ float tD[6 * PL];

  const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
  const int li = lane & 15, g = lane >> 4;

  CnnWeights<CH, BF> w;
  load_weights<CH>(w, theta, li, g, PL, HX);
  const ThetaOff O = theta_off(CH);
  const float bias0 = theta[O.bL + 0], bias1 = theta[O.bL + 1], bias2 = theta[O.bL + 2];
  int off[16];
#pragma unroll
  for (int s = 0; s < 16; ++s) slot_tap(g, s, PL, HX, off[s]);
  const int ctr_plane = (g < 3 ? g : 0) * PL;

  int first, stride, count;
  xcd_tile_range(n_tiles, first, stride, count);
  for (int it = 0; it < count; ++it) {
    const int t = first + it * stride;
    const int b = find_instance(prefix, n_inst, t);
    if (skip != nullptr && skip[b] != 0) continue;  // uniform over the workgroup
    const InstDev I = inst[b];
    const int lt = t - prefix[b];
    const int tiles_x = (I.W + TX - 1) / TX;
    const int r0 = (lt / tiles_x) * TY, c0 = (lt % tiles_x) * TX;

    // Stage S^k and S^k - S^{k-1} over the tile plus a one-node halo, clamped to the grid
    // (the clamp-to-edge padding of the convolution).
    for (int e = threadIdx.x; e < 6 * PL; e += 256) {
      const int c = e / PL;
      const int rem = e - c * PL;
      const int rr = rem / HX, cc = rem - (rem / HX) * HX;
      const int gi = min(max(r0 + rr - 1, 0), I.H - 1);
      const int gj = min(max(c0 + cc - 1, 0), I.W - 1);
      const int64_t q = (int64_t)c * N + I.off + (int64_t)gi * I.W + gj;
      const float sk = s_cur[q];
      tS[e] = sk;
      tD[e] = sk - s_prev[q];
    }
    __syncthreads();

    for (int seg = wave; seg < NSEG; seg += 4) {
      const int ly = seg / SEGX, lx = (seg % SEGX) * 16 + li;
      const int base = (ly + 1) * HX + (lx + 1);
      // im2col of this lane's 16 slots: FP32 differences with the centre for position taps
      float uS[16], uD[16];
      const float cS = tS[ctr_plane + base], cD = tD[ctr_plane + base];
#pragma unroll
      for (int s = 0; s < 16; ++s) {
        const float vs = tS[base + off[s]], vd = tD[base + off[s]];
        uS[s] = s < 8 ? vs - cS : vs;
        uD[s] = s < 8 ? vd - cD : vd;
      }
      f32x4 accP[MB], accX[MB];
#pragma unroll
      for (int mb = 0; mb < MB; ++mb) {
        accP[mb] = f32x4{0.f, 0.f, 0.f, 0.f};
        accX[mb] = f32x4{0.f, 0.f, 0.f, 0.f};
      }
      conv_mfma<CH>(w, uS, accP);
      conv_mfma<CH>(w, uD, accX);

      float phi[CPL], xi[CPL];
#pragma unroll
      for (int e = 0; e < CPL; ++e) {
        phi[e] = accP[e >> 2][e & 3];
        xi[e] = accX[e >> 2][e & 3];
      }
      f32x4 ab[2 * MB];
      mix_mfma<CH>(w, phi, ab);
      float F[3 * CPL];
#pragma unroll
      for (int e = 0; e < CPL; ++e) {
        const float a = ab[e >> 2][e & 3], bb = ab[MB + (e >> 2)][e & 3];
        const float gs = isru(phi[e], alpha);
        F[e] = phi[e];
        F[CPL + e] = isru(a * bb, alpha);
        F[2 * CPL + e] = xi[e] * gs;
      }
      const f32x4 dv = head_mfma<CH>(w, F);

      // eq. (5) inside the frame, in lane group 0 (rows 0..2 of the head output)
      const int i = r0 + ly, j = c0 + lx;
      if (g == 0 && i < I.H && j < I.W) {
        const int64_t p = I.off + (int64_t)i * I.W + j;
        const float vx = tS[3 * PL + base], vy = tS[4 * PL + base], vz = tS[5 * PL + base];
        float nx = vx + dv[0] + bias0 + dt * I.ax;
        float ny = vy + dv[1] + bias1 + dt * I.ay;
        float nz = vz + dv[2] + bias2 + dt * I.az;
        if (pin[p]) nx = ny = nz = 0.f;
        s_next[3 * N + p] = nx;
        s_next[4 * N + p] = ny;
        s_next[5 * N + p] = nz;
        s_next[0 * N + p] = tS[base] + dt * nx;
        s_next[1 * N + p] = tS[PL + base] + dt * ny;
        s_next[2 * N + p] = tS[2 * PL + base] + dt * nz;
      }
    }
    __syncthreads();
  }
}

template <int CH, bool BF, int TX, int TY>
static void launch_cnn(const pecnn_plan* plan, int slot, const float* sp, const float* sc, float* sn,
                       const float* theta, float dt, float alpha, const int32_t* skip, hipStream_t st) {
  const int n_tiles = plan->n_tiles[slot];
  int grid = num_cus() * 4;
  const int need = ((n_tiles + 7) / 8) * 8;
  if (need < grid) grid = need;
  if (grid < 8) grid = 8;
  hipLaunchKernelGGL((cnn_fwd_kernel<CH, BF, TX, TY>), dim3(grid), dim3(256), 0, st, plan->d_inst,
                     plan->d_prefix[slot], plan->n, n_tiles, plan->pin, sp, sc, sn, plan->total, theta, dt,
                     alpha, skip);
}

template <int CH, bool BF>
static int dispatch_cfg(const pecnn_plan* plan, int cfg, const float* sp, const float* sc, float* sn,
                        const float* theta, float dt, float alpha, const int32_t* skip, hipStream_t st) {
  const int slot = cnn_cfg_slot(cfg);
  switch (cfg) {
    case 0: launch_cnn<CH, BF, 64, 4>(plan, slot, sp, sc, sn, theta, dt, alpha, skip, st); break;
    case 1: launch_cnn<CH, BF, 32, 8>(plan, slot, sp, sc, sn, theta, dt, alpha, skip, st); break;
    case 2: launch_cnn<CH, BF, 16, 16>(plan, slot, sp, sc, sn, theta, dt, alpha, skip, st); break;
    default: return PECNN_E_INVALID;
  }
  return PECNN_OK;
}

int cnn_forward_launch(const pecnn_plan* plan, int cfg, const pecnn_model* m, const float* sp,
                       const float* sc, float* sn, const int32_t* skip, hipStream_t st) {
  int rc;
  if (m->ch == 16)
    rc = m->precision == PECNN_BF16 ? dispatch_cfg<16, true>(plan, cfg, sp, sc, sn, m->theta, m->dt, m->isru_alpha, skip, st)
                                    : dispatch_cfg<16, false>(plan, cfg, sp, sc, sn, m->theta, m->dt, m->isru_alpha, skip, st);
  else
    rc = m->precision == PECNN_BF16 ? dispatch_cfg<32, true>(plan, cfg, sp, sc, sn, m->theta, m->dt, m->isru_alpha, skip, st)
                                    : dispatch_cfg<32, false>(plan, cfg, sp, sc, sn, m->theta, m->dt, m->isru_alpha, skip, st);
  if (rc != PECNN_OK) return rc;
  PECNN_LAUNCH_CHECK("cnn_fwd_kernel");
  return PECNN_OK;
}

}  // namespace pecnn
