// Reverse mode of the CNN frame on the matrix cores (section 3.2.1: the parameters w, b are
// optimised by gradient backpropagation through eqs. 5-7). FP32 operands throughout
// (v_mfma_f32_16x16x4_f32), in the transposed channel x node layout of the forward kernels.
//
// One persistent pass over tiles of 64 x 4 nodes, four waves, each wave one 16-node segment at a
// time:
//   * the frame is recomputed from S^k and S^k - S^{k-1}, staged with a one-node halo;
//   * the adjoint of eq. (5) gives gdv = dLoss/d(dv); the head adjoint, the ISRU and product
//     adjoints and the [A;B] adjoint follow (matrix cores for the products, FP32 VALU for the rest);
//   * the adjoint of the im2col entries, K^T [dLoss/dphi ; dLoss/dxi], goes to a compact
//     node-blocked table (54 + 54 rows and gdv) that the gather kernel turns into the input
//     gradients (the clamped stencil is read from the neighbours' side);
//   * the parameter gradients are products with the node axis as the contraction. Each wave moves
//     one segment's factors through its own LDS scratch into the node-major operand layout and
//     accumulates 16 x 16 tiles in registers over all its segments; at the end the four waves add
//     their sums in LDS and the workgroup writes one row of partial sums.
// Deterministic: every wave owns fixed segments and sums them in order, the waves are added in
// order, and the rows are summed in order by the final kernel.
#include "cnn_bwd_table.hpp"
#include "cnn_common.hpp"

namespace pecnn {

template <int CH>
struct BtLds {
  static constexpr int MB = CH / 16, CPL = CH / 4;
  static constexpr int TX = 64, TY = 4, HX = TX + 2, HY = TY + 2, PL = HX * HY;
  // per-lane operand tables: entry (table row r, lane l, u) at ((r * 64 + l) * 4 + u)
  static constexpr int CONV_R = MB * 4;           // conv A operands, slots s = 4 sq + u
  static constexpr int MIX_R = 2 * MB * CPL / 4;   // [A;B] A operands
  static constexpr int MIXT_R = MB * 2 * CPL / 4;  // [A^T | B^T] A operands
  static constexpr int KT_R = 4 * CPL / 4;         // K^T A operands, four 16-slot row blocks
  static constexpr int SR = (CH + 64 > 3 * CH ? CH + 64 : 3 * CH);  // scratch rows per wave
  static constexpr int oS = 0, oD = 6 * PL, oCONV = 12 * PL, oMIX = oCONV + CONV_R * 256,
                       oMIXT = oMIX + MIX_R * 256, oKT = oMIXT + MIXT_R * 256, oSCR = oKT + KT_R * 256,
                       TOTAL = oSCR + 4 * SR * 16;
};

__device__ __forceinline__ f32x4 lds4(const float* __restrict__ t, int row, int lane) {
  return *reinterpret_cast<const f32x4*>(&t[(row * 64 + lane) * 4]);
}

// LDS writes of this wave are complete and ordered before what follows (the scratch is private to
// the wave; its lanes exchange values through it).
__device__ __forceinline__ void wave_lds_sync() { asm volatile("s_waitcnt lgkmcnt(0)" ::: "memory"); }

// The per-lane operand tables, (table row r, lane l, u) at (r * 64 + l) * 4 + u: conv A operands
// K (slots s = 4 sq + u), [A;B] A operands, [A^T | B^T] A operands and K^T A operands (row
// kappa = 4 s + g' of the conv's K dimension). Loops of fixed trip count, so that the parameter
// loads of a thread are all in flight together.
template <int CH>
__device__ __forceinline__ void fill_tables(float* lds, const float* __restrict__ theta, int tid) {
  using Lc = BtLds<CH>;
  constexpr int CPL = Lc::CPL, PL = Lc::PL, HX = Lc::HX;
  const ThetaOff O = theta_off(CH);
#pragma unroll
  for (int k = 0; k < Lc::CONV_R; ++k) {
    const int e = tid + 256 * k;
    const int r = e >> 8, l = (e >> 2) & 63, u = e & 3;
    const int mb = r / 4, s = 4 * (r % 4) + u, lli = l & 15, lg = l >> 4;
    int lo;
    const int t = slot_tap(lg, s, PL, HX, lo);
    lds[Lc::oCONV + e] = t >= 0 ? theta[O.K + (16 * mb + lli) * 54 + t] : 0.f;
  }
#pragma unroll
  for (int k = 0; k < Lc::MIX_R; ++k) {
    const int e = tid + 256 * k;
    const int r = e >> 8, l = (e >> 2) & 63, u = e & 3;
    const int mbp = r / (CPL / 4), ee = 4 * (r % (CPL / 4)) + u, lli = l & 15, lg = l >> 4;
    lds[Lc::oMIX + e] = mix_weight<CH>(theta, O, 16 * mbp + lli, lg, ee);
  }
#pragma unroll
  for (int k = 0; k < Lc::MIXT_R; ++k) {
    const int e = tid + 256 * k;
    const int r = e >> 8, l = (e >> 2) & 63, u = e & 3;
    const int mb = r / (2 * CPL / 4), jj = 4 * (r % (2 * CPL / 4)) + u, lli = l & 15, lg = l >> 4;
    const int base = jj < CPL ? O.A : O.B;
    const int c = slot_channel(lg, jj < CPL ? jj : jj - CPL);
    lds[Lc::oMIXT + e] = theta[base + c * CH + 16 * mb + lli];
  }
#pragma unroll
  for (int k = 0; k < Lc::KT_R; ++k) {
    const int e = tid + 256 * k;
    const int r = e >> 8, l = (e >> 2) & 63, u = e & 3;
    const int rb = r / (CPL / 4), ee = 4 * (r % (CPL / 4)) + u, lli = l & 15, lg = l >> 4;
    const int kap = 16 * rb + lli;
    int lo;
    const int t = slot_tap(kap & 3, kap >> 2, PL, HX, lo);
    lds[Lc::oKT + e] = t >= 0 ? theta[O.K + slot_channel(lg, ee) * 54 + t] : 0.f;
  }
}

template <int CH>
__global__ __launch_bounds__(256) __attribute__((amdgpu_waves_per_eu(2, 2))) void bwd_tile_kernel(
    const InstDev* __restrict__ inst, const int32_t* __restrict__ prefix, int n_inst, int n_tiles,
    const uint8_t* __restrict__ pin, const float* __restrict__ s_prev, const float* __restrict__ s_cur,
    const float* __restrict__ g_next, int64_t N, const float* __restrict__ theta, float dt, float alpha,
    float* __restrict__ tab, float* __restrict__ partial) {
  using Lc = BtLds<CH>;
  constexpr int MB = Lc::MB, CPL = Lc::CPL, TX = Lc::TX, TY = Lc::TY, HX = Lc::HX, HY = Lc::HY, PL = Lc::PL;
  constexpr int SEGX = TX / 16, NSEG = SEGX * TY;
  constexpr int P = CH * 54 + 2 * CH * CH + 9 * CH + 3;
  __shared__ __align__(16) float lds[Lc::TOTAL];
  float* tS = lds + Lc::oS;
  float* tD = lds + Lc::oD;

  const int tid = threadIdx.x, lane = tid & 63, wave = tid >> 6;
  const int li = lane & 15, g = lane >> 4;
  const ThetaOff O = theta_off(CH);

  fill_tables<CH>(lds, theta, tid);
  __syncthreads();

  // LDS offsets of the im2col slots relative to the node's centre cell: the position slots
  // (s < 8) of lane group g are the 8 off-centre taps of channel g, at compile-time offsets from
  // its plane (group 3's are padding: they read plane 0 and meet zero weights); the velocity
  // slots depend on the group
  const int ctr_plane = (g < 3 ? g : 0) * PL;
  int voff[8];
#pragma unroll
  for (int s = 0; s < 8; ++s) slot_tap(g, 8 + s, PL, HX, voff[s]);
  const int pm = (li & 3) * 4 + (li >> 2);  // scratch column of this lane's node
  float* X = lds + Lc::oSCR + wave * Lc::SR * 16;

  f32x4 accK[MB][4], accA[MB][MB], accB[MB][MB], accW[3][MB];
#pragma unroll
  for (int mb = 0; mb < MB; ++mb) {
#pragma unroll
    for (int tb = 0; tb < 4; ++tb) accK[mb][tb] = f32x4{0.f, 0.f, 0.f, 0.f};
#pragma unroll
    for (int m2 = 0; m2 < MB; ++m2) accA[mb][m2] = accB[mb][m2] = f32x4{0.f, 0.f, 0.f, 0.f};
#pragma unroll
    for (int h = 0; h < 3; ++h) accW[h][mb] = f32x4{0.f, 0.f, 0.f, 0.f};
  }
  float db0 = 0.f, db1 = 0.f, db2 = 0.f;

  int first, stride, count;
  xcd_tile_range(n_tiles, first, stride, count);
  for (int it = 0; it < count; ++it) {
    const int t = first + it * stride;
    const int b = find_instance(prefix, n_inst, t);
    const InstDev I = inst[b];
    const int lt = t - prefix[b];
    const int tiles_x = (I.W + TX - 1) / TX;
    const int r0 = (lt / tiles_x) * TY, c0 = (lt % tiles_x) * TX;
    for (int e = tid; e < 6 * PL; e += 256) {
      const int c = e / PL, rem = e - c * PL;
      const int rr = rem / HX, cc = rem - (rem / HX) * HX;
      const int gi = min(max(r0 + rr - 1, 0), I.H - 1), gj = min(max(c0 + cc - 1, 0), I.W - 1);
      const int64_t q = (int64_t)c * N + I.off + (int64_t)gi * I.W + gj;
      const float sk = s_cur[q];
      tS[e] = sk;
      tD[e] = sk - s_prev[q];
    }
    __syncthreads();

    for (int seg = wave; seg < NSEG; seg += 4) {
      const int ly = seg / SEGX, lx = (seg % SEGX) * 16 + li;
      const int base = (ly + 1) * HX + (lx + 1);
      const int i = r0 + ly, j = c0 + lx;
      const bool valid = i < I.H && j < I.W;
      const int64_t p = I.off + (int64_t)(valid ? i : 0) * I.W + (valid ? j : 0);

      // ---- forward recompute: im2col, phi and xi (eq. 6), [a; b] = [A; B] phi
      float uS[16], uD[16];  // consumed by the conv products below
      const float cS = tS[ctr_plane + base], cD = tD[ctr_plane + base];
#pragma unroll
      for (int s = 0; s < 8; ++s) {
        const int o = s + (s >= 4 ? 1 : 0);
        const int d = ctr_plane + (o / 3 - 1) * HX + (o % 3 - 1);
        uS[s] = tS[base + d] - cS;
        uD[s] = tD[base + d] - cD;
        uS[8 + s] = tS[base + voff[s]];
        uD[8 + s] = tD[base + voff[s]];
      }
      f32x4 accP[MB], accX[MB];
#pragma unroll
      for (int mb = 0; mb < MB; ++mb) {
        accP[mb] = accX[mb] = f32x4{0.f, 0.f, 0.f, 0.f};
#pragma unroll
        for (int sq = 0; sq < 4; ++sq) {
          const f32x4 w = lds4(lds + Lc::oCONV, mb * 4 + sq, lane);
#pragma unroll
          for (int u = 0; u < 4; ++u) {
            accP[mb] = __builtin_amdgcn_mfma_f32_16x16x4f32(w[u], uS[4 * sq + u], accP[mb], 0, 0, 0);
            accX[mb] = __builtin_amdgcn_mfma_f32_16x16x4f32(w[u], uD[4 * sq + u], accX[mb], 0, 0, 0);
          }
        }
      }
      float phi[CPL], xi[CPL];
#pragma unroll
      for (int e = 0; e < CPL; ++e) {
        phi[e] = accP[e >> 2][e & 3];
        xi[e] = accX[e >> 2][e & 3];
      }
      f32x4 ab[2 * MB];
#pragma unroll
      for (int mbp = 0; mbp < 2 * MB; ++mbp) {
        ab[mbp] = f32x4{0.f, 0.f, 0.f, 0.f};
#pragma unroll
        for (int eq = 0; eq < CPL / 4; ++eq) {
          const f32x4 w = lds4(lds + Lc::oMIX, mbp * (CPL / 4) + eq, lane);
#pragma unroll
          for (int u = 0; u < 4; ++u)
            ab[mbp] = __builtin_amdgcn_mfma_f32_16x16x4f32(w[u], phi[4 * eq + u], ab[mbp], 0, 0, 0);
        }
      }

      // ---- adjoint of eq. (5): gdv = C^T (g_v' + dt g_x') (zero for pinned and off-grid nodes)
      float gd0 = 0.f, gd1 = 0.f, gd2 = 0.f;
      if (valid && pin[p] == 0) {
        gd0 = __builtin_fmaf(dt, g_next[p], g_next[3 * N + p]);
        gd1 = __builtin_fmaf(dt, g_next[N + p], g_next[4 * N + p]);
        gd2 = __builtin_fmaf(dt, g_next[2 * N + p], g_next[5 * N + p]);
      }
      const float bg = g == 0 ? gd0 : (g == 1 ? gd1 : (g == 2 ? gd2 : 0.f));
      // head adjoints: dLoss/dphi (W_L part), dLoss/dn, dLoss/dd
      // (A operands W_h^T: rows = channels, K = the three outputs with a zero pad; read from the
      // cached parameters rather than held in registers)
      f32x4 gH[3][MB];
#pragma unroll
      for (int h = 0; h < 3; ++h)
#pragma unroll
        for (int mb = 0; mb < MB; ++mb) {
          const int hb = h == 0 ? O.WL : (h == 1 ? O.WN : O.WD);
          const float w = g < 3 ? theta[hb + g * CH + 16 * mb + li] : 0.f;
          gH[h][mb] = __builtin_amdgcn_mfma_f32_16x16x4f32(w, bg, f32x4{0.f, 0.f, 0.f, 0.f}, 0, 0, 0);
        }

      // ---- eq. (7) elementwise adjoints (ISRU sigma(z) = z (1 + alpha z^2)^(-1/2), sigma' = r^3)
      float ga[CPL], gb[CPL], gxi[CPL], nn[CPL], dd[CPL];
      f32x4 gp[MB];
#pragma unroll
      for (int e = 0; e < CPL; ++e) {
        const float ph = phi[e], x = xi[e];
        const float a = ab[e >> 2][e & 3], bb = ab[MB + (e >> 2)][e & 3];
        const float r1 = __builtin_amdgcn_rsqf(__builtin_fmaf(alpha * ph, ph, 1.f));
        const float gs = ph * r1, dgs = r1 * r1 * r1;
        const float z = a * bb;
        const float r2 = __builtin_amdgcn_rsqf(__builtin_fmaf(alpha * z, z, 1.f));
        const float gz = gH[1][e >> 2][e & 3] * (r2 * r2 * r2);
        const float gdd = gH[2][e >> 2][e & 3];
        nn[e] = z * r2;
        dd[e] = x * gs;
        ga[e] = gz * bb;
        gb[e] = gz * a;
        gp[e >> 2][e & 3] = __builtin_fmaf(gdd * x, dgs, gH[0][e >> 2][e & 3]);
        gxi[e] = gdd * gs;
      }
      // ---- parameter gradients: products over the segment's 16 nodes (K = node), operands moved
      // to the node-major layout through this wave's scratch (row r, column pm = node slot); the
      // phases run in the order that frees registers soonest
      // dW_L += gdv phi^T, dW_N += gdv n^T, dW_D += gdv d^T (rows 0..2 of the 16-row operand are
      // gdv; the others are left as they are and only feed output rows that are dropped)
      {
        if (g == 0) {
          X[0 * 16 + pm] = gd0;
          X[1 * 16 + pm] = gd1;
          X[2 * 16 + pm] = gd2;
        }
#pragma unroll
        for (int e = 0; e < CPL; ++e) {
          const int r = slot_channel(g, e);
          X[(16 + r) * 16 + pm] = phi[e];
          X[(16 + CH + r) * 16 + pm] = nn[e];
        }
        wave_lds_sync();
        const f32x4 Gd = *reinterpret_cast<const f32x4*>(&X[li * 16 + 4 * g]);
        f32x4 F0[MB], F1[MB];
#pragma unroll
        for (int mb = 0; mb < MB; ++mb) {
          F0[mb] = *reinterpret_cast<const f32x4*>(&X[(16 + 16 * mb + li) * 16 + 4 * g]);
          F1[mb] = *reinterpret_cast<const f32x4*>(&X[(16 + CH + 16 * mb + li) * 16 + 4 * g]);
        }
        wave_lds_sync();
#pragma unroll
        for (int e = 0; e < CPL; ++e) X[(16 + slot_channel(g, e)) * 16 + pm] = dd[e];
        wave_lds_sync();
        f32x4 F2[MB];
#pragma unroll
        for (int mb = 0; mb < MB; ++mb) F2[mb] = *reinterpret_cast<const f32x4*>(&X[(16 + 16 * mb + li) * 16 + 4 * g]);
        wave_lds_sync();
#pragma unroll
        for (int q = 0; q < 4; ++q)
#pragma unroll
          for (int mb = 0; mb < MB; ++mb) {
            accW[0][mb] = __builtin_amdgcn_mfma_f32_16x16x4f32(Gd[q], F0[mb][q], accW[0][mb], 0, 0, 0);
            accW[1][mb] = __builtin_amdgcn_mfma_f32_16x16x4f32(Gd[q], F1[mb][q], accW[1][mb], 0, 0, 0);
            accW[2][mb] = __builtin_amdgcn_mfma_f32_16x16x4f32(Gd[q], F2[mb][q], accW[2][mb], 0, 0, 0);
          }
      }
      // dLoss/dphi += A^T dLoss/da + B^T dLoss/db
#pragma unroll
      for (int mb = 0; mb < MB; ++mb)
#pragma unroll
        for (int jq = 0; jq < 2 * CPL / 4; ++jq) {
          const f32x4 w = lds4(lds + Lc::oMIXT, mb * (2 * CPL / 4) + jq, lane);
#pragma unroll
          for (int u = 0; u < 4; ++u) {
            const int jj = 4 * jq + u;
            gp[mb] = __builtin_amdgcn_mfma_f32_16x16x4f32(w[u], jj < CPL ? ga[jj] : gb[jj - CPL], gp[mb], 0, 0, 0);
          }
        }
      float gphi[CPL];
#pragma unroll
      for (int e = 0; e < CPL; ++e) gphi[e] = gp[e >> 2][e & 3];

      // dA += dLoss/da phi^T, dB += dLoss/db phi^T
      {
#pragma unroll
        for (int e = 0; e < CPL; ++e) {
          const int r = slot_channel(g, e);
          X[r * 16 + pm] = ga[e];
          X[(CH + r) * 16 + pm] = gb[e];
          X[(2 * CH + r) * 16 + pm] = phi[e];
        }
        wave_lds_sync();
        f32x4 Aa[MB], Bb[MB], Ph[MB];
#pragma unroll
        for (int mb = 0; mb < MB; ++mb) {
          Aa[mb] = *reinterpret_cast<const f32x4*>(&X[(16 * mb + li) * 16 + 4 * g]);
          Bb[mb] = *reinterpret_cast<const f32x4*>(&X[(CH + 16 * mb + li) * 16 + 4 * g]);
          Ph[mb] = *reinterpret_cast<const f32x4*>(&X[(2 * CH + 16 * mb + li) * 16 + 4 * g]);
        }
        wave_lds_sync();
#pragma unroll
        for (int q = 0; q < 4; ++q)
#pragma unroll
          for (int m1 = 0; m1 < MB; ++m1)
#pragma unroll
            for (int m2 = 0; m2 < MB; ++m2) {
              accA[m1][m2] = __builtin_amdgcn_mfma_f32_16x16x4f32(Aa[m1][q], Ph[m2][q], accA[m1][m2], 0, 0, 0);
              accB[m1][m2] = __builtin_amdgcn_mfma_f32_16x16x4f32(Bb[m1][q], Ph[m2][q], accB[m1][m2], 0, 0, 0);
            }
      }
      // ---- adjoint of the im2col entries: K^T dLoss/dphi and K^T dLoss/dxi (slot order)
      f32x4 gUS[4], gUD[4];
#pragma unroll
      for (int rb = 0; rb < 4; ++rb) {
        gUS[rb] = gUD[rb] = f32x4{0.f, 0.f, 0.f, 0.f};
#pragma unroll
        for (int eq = 0; eq < CPL / 4; ++eq) {
          const f32x4 w = lds4(lds + Lc::oKT, rb * (CPL / 4) + eq, lane);
#pragma unroll
          for (int u = 0; u < 4; ++u) {
            gUS[rb] = __builtin_amdgcn_mfma_f32_16x16x4f32(w[u], gphi[4 * eq + u], gUS[rb], 0, 0, 0);
            gUD[rb] = __builtin_amdgcn_mfma_f32_16x16x4f32(w[u], gxi[4 * eq + u], gUD[rb], 0, 0, 0);
          }
        }
      }
      if (valid) {
        float* __restrict__ F = tab + bt_node(p);
#pragma unroll
        for (int rb = 0; rb < 4; ++rb)
#pragma unroll
          for (int v = 0; v < 4; ++v) {
            // this lane's output row 16 rb + 4 g + v is conv slot s = 4 rb + g of lane group v
            const int sl = 4 * rb + g;
            const int vi = 8 * v + sl - 8;
            const int tp = rb < 2 ? (v < 3 ? v * 9 + sl + (sl >= 4 ? 1 : 0) : -1) : (vi < 27 ? 27 + vi : -1);
            if (tp >= 0) {
              F[(kBtGus + tp) * 32] = gUS[rb][v] + gUD[rb][v];  // S^k enters U(S^k) and U(S^k - S^{k-1})
              F[(kBtGud + tp) * 32] = gUD[rb][v];
            }
          }
        if (g == 0) {
          // the centre taps of the position channels multiply identical zeros: no adjoint
#pragma unroll
          for (int c = 0; c < 3; ++c) {
            F[(kBtGus + c * 9 + 4) * 32] = 0.f;
            F[(kBtGud + c * 9 + 4) * 32] = 0.f;
          }
          F[(kBtGdv + 0) * 32] = gd0;
          F[(kBtGdv + 1) * 32] = gd1;
          F[(kBtGdv + 2) * 32] = gd2;
          db0 += gd0;
          db1 += gd1;
          db2 += gd2;
        }
      }

      // dK (slot order) += dLoss/dphi U(S)^T, then dLoss/dxi U(S - S_prev)^T; the im2col entries
      // are read again from the staged tile rather than kept in registers
#pragma unroll
      for (int half = 0; half < 2; ++half) {
        const float* __restrict__ T = half == 0 ? tS : tD;
        const float ct = T[ctr_plane + base];
#pragma unroll
        for (int e = 0; e < CPL; ++e) X[slot_channel(g, e) * 16 + pm] = half == 0 ? gphi[e] : gxi[e];
#pragma unroll
        for (int s = 0; s < 8; ++s) {
          const int o = s + (s >= 4 ? 1 : 0);
          X[(CH + 4 * s + g) * 16 + pm] = T[base + ctr_plane + (o / 3 - 1) * HX + (o % 3 - 1)] - ct;
          X[(CH + 4 * (8 + s) + g) * 16 + pm] = T[base + voff[s]];
        }
        wave_lds_sync();
        f32x4 Ga[MB], Ub[4];
#pragma unroll
        for (int mb = 0; mb < MB; ++mb) Ga[mb] = *reinterpret_cast<const f32x4*>(&X[(16 * mb + li) * 16 + 4 * g]);
#pragma unroll
        for (int tb = 0; tb < 4; ++tb) Ub[tb] = *reinterpret_cast<const f32x4*>(&X[(CH + 16 * tb + li) * 16 + 4 * g]);
        wave_lds_sync();
#pragma unroll
        for (int q = 0; q < 4; ++q)
#pragma unroll
          for (int mb = 0; mb < MB; ++mb)
#pragma unroll
            for (int tb = 0; tb < 4; ++tb)
              accK[mb][tb] = __builtin_amdgcn_mfma_f32_16x16x4f32(Ga[mb][q], Ub[tb][q], accK[mb][tb], 0, 0, 0);
      }
    }
    __syncthreads();  // the staged tile is reused by the next one
  }

  // ---- the parameter gradients of this workgroup, one row in the flat parameter layout: each
  // wave writes its sums to LDS (the tile stage is free now), then the four rows are added in
  // wave order
  // (the loop ends on a barrier: no wave reads the tile stage or the operand tables any more)
  static_assert(4 * P <= Lc::TOTAL, "LDS holds four partial rows");
  float* __restrict__ out = lds + wave * P;
#pragma unroll
  for (int mb = 0; mb < MB; ++mb)
#pragma unroll
    for (int tb = 0; tb < 4; ++tb) {
      const int kap = 16 * tb + li;
      int lo;
      const int tp = slot_tap(kap & 3, kap >> 2, PL, HX, lo);
      if (tp >= 0)
#pragma unroll
        for (int v = 0; v < 4; ++v) out[O.K + (16 * mb + 4 * g + v) * 54 + tp] = accK[mb][tb][v];
    }
  for (int e = lane; e < 3 * CH; e += 64) out[O.K + (e / 3) * 54 + (e % 3) * 9 + 4] = 0.f;
#pragma unroll
  for (int m1 = 0; m1 < MB; ++m1)
#pragma unroll
    for (int m2 = 0; m2 < MB; ++m2)
#pragma unroll
      for (int v = 0; v < 4; ++v) {
        out[O.A + (16 * m1 + 4 * g + v) * CH + 16 * m2 + li] = accA[m1][m2][v];
        out[O.B + (16 * m1 + 4 * g + v) * CH + 16 * m2 + li] = accB[m1][m2][v];
      }
#pragma unroll
  for (int h = 0; h < 3; ++h) {
    const int base = h == 0 ? O.WL : (h == 1 ? O.WN : O.WD);
#pragma unroll
    for (int mb = 0; mb < MB; ++mb)
#pragma unroll
      for (int v = 0; v < 4; ++v)
        if (4 * g + v < 3) out[base + (4 * g + v) * CH + 16 * mb + li] = accW[h][mb][v];
  }
  // b_L: the wave's lanes hold per-node sums of gdv; an xor tree in a fixed order
#pragma unroll
  for (int o = 32; o > 0; o >>= 1) {
    db0 += __shfl_xor(db0, o, 64);
    db1 += __shfl_xor(db1, o, 64);
    db2 += __shfl_xor(db2, o, 64);
  }
  if (lane == 0) {
    out[O.bL + 0] = db0;
    out[O.bL + 1] = db1;
    out[O.bL + 2] = db2;
  }
  __syncthreads();
  float* __restrict__ row = partial + (int64_t)blockIdx.x * P;
  for (int e = tid; e < P; e += 256) row[e] = ((lds[e] + lds[P + e]) + lds[2 * P + e]) + lds[3 * P + e];
}

// ------------------------------------------------------------------ host side
// Two workgroups per CU (the LDS and register budget of the kernel), never more than the tiles:
// every workgroup writes one row of partial sums.
int bwd_tile_grid(const pecnn_plan* plan) {
  const int nt = plan->n_tiles[cnn_cfg_slot(0)];
  const int g = num_cus() * 2;
  return nt < g ? (nt > 0 ? nt : 1) : g;
}

size_t bwd_tile_ws_bytes(const pecnn_plan* plan, int ch) {
  const size_t tab = (size_t)bt_floats(plan->total) * sizeof(float);
  const size_t P = (size_t)ch * 54 + 2 * (size_t)ch * ch + 9 * (size_t)ch + 3;
  return ((tab + 255) / 256) * 256 + (size_t)bwd_tile_grid(plan) * P * sizeof(float);
}

int bwd_tile_launch(const pecnn_plan* plan, const pecnn_model* m, const float* sp, const float* sc, const float* gn,
                    float* tab, float* partial, hipStream_t st) {
  const int slot = cnn_cfg_slot(0);  // tiles of 64 x 4 nodes
  const int grid = bwd_tile_grid(plan);
  if (m->ch == 16)
    hipLaunchKernelGGL(bwd_tile_kernel<16>, dim3(grid), dim3(256), 0, st, plan->d_inst, plan->d_prefix[slot], plan->n,
                       plan->n_tiles[slot], plan->pin, sp, sc, gn, plan->total, m->theta, m->dt, m->isru_alpha, tab,
                       partial);
  else
    hipLaunchKernelGGL(bwd_tile_kernel<32>, dim3(grid), dim3(256), 0, st, plan->d_inst, plan->d_prefix[slot], plan->n,
                       plan->n_tiles[slot], plan->pin, sp, sc, gn, plan->total, m->theta, m->dt, m->isru_alpha, tab,
                       partial);
  PECNN_LAUNCH_CHECK("bwd_tile_kernel");
  return PECNN_OK;
}

}  // namespace pecnn
