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
#include "cnn_common.hpp"

namespace pecnn {

template <int CH, bool BF, int TX, int TY>
__global__ __launch_bounds__(256) void cnn_fwd_kernel(
    const InstDev* __restrict__ inst, const int32_t* __restrict__ prefix, int n_inst, int n_tiles,
    const uint8_t* __restrict__ pin, const float* __restrict__ s_prev, const float* __restrict__ s_cur,
    float* __restrict__ s_next, int64_t N, const float* __restrict__ theta, float dt, float alpha,
    const int32_t* __restrict__ skip, const float* __restrict__ sphere) {
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
    // (the clamp-to-edge padding of the convolution); every load of a thread is issued before
    // its first store.
    constexpr int NST = (6 * PL + 255) / 256;
    float vs[NST], vp[NST];
#pragma unroll
    for (int k = 0; k < NST; ++k) {
      const int e = (int)threadIdx.x + 256 * k;
      vs[k] = vp[k] = 0.f;
      if (e < 6 * PL) {
        const int c = e / PL;
        const int rem = e - c * PL;
        const int rr = rem / HX, cc = rem - (rem / HX) * HX;
        const int gi = min(max(r0 + rr - 1, 0), I.H - 1);
        const int gj = min(max(c0 + cc - 1, 0), I.W - 1);
        const int64_t q = (int64_t)c * N + I.off + (int64_t)gi * I.W + gj;
        vs[k] = s_cur[q];
        vp[k] = s_prev[q];
      }
    }
#pragma unroll
    for (int k = 0; k < NST; ++k) {
      const int e = (int)threadIdx.x + 256 * k;
      if (e < 6 * PL) {
        tS[e] = vs[k];
        tD[e] = vs[k] - vp[k];
      }
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
        float nx = (vx + dv[0]) + __builtin_fmaf(dt, I.ax, bias0);
        float ny = (vy + dv[1]) + __builtin_fmaf(dt, I.ay, bias1);
        float nz = (vz + dv[2]) + __builtin_fmaf(dt, I.az, bias2);
        if (I.pres != 0.f) {  // eq. (3) at S^k, a known external force (uniform over the workgroup)
          const int nb[4] = {1, HX, -1, -HX};  // right, down, left, up
          float d[4][3];
#pragma unroll
          for (int q = 0; q < 4; ++q)
#pragma unroll
            for (int c = 0; c < 3; ++c) d[q][c] = tS[c * PL + base + nb[q]] - tS[c * PL + base];
          const bool has[4] = {j + 1 < I.W, i + 1 < I.H, j > 0, i > 0};
          float p0, p1, p2;
          pressure_pairs(d, has, p0, p1, p2);
          const float cp = dt * I.pres / I.mass;
          nx = __builtin_fmaf(cp, p0, nx);
          ny = __builtin_fmaf(cp, p1, ny);
          nz = __builtin_fmaf(cp, p2, nz);
        }
        const bool pinned = pin[p] != 0;
        if (pinned) nx = ny = nz = 0.f;
        float y0 = __builtin_fmaf(dt, nx, tS[base]), y1 = __builtin_fmaf(dt, ny, tS[PL + base]),
              y2 = __builtin_fmaf(dt, nz, tS[2 * PL + base]);
        if (!pinned)  // the constraint of eq. (5) with the instance's sphere, if it has one
          sphere_update(sphere + b * kSphereStride, dt, tS[base], tS[PL + base], tS[2 * PL + base], nx, ny, nz, y0,
                        y1, y2);
        s_next[3 * N + p] = nx;
        s_next[4 * N + p] = ny;
        s_next[5 * N + p] = nz;
        s_next[0 * N + p] = y0;
        s_next[1 * N + p] = y1;
        s_next[2 * N + p] = y2;
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
                     alpha, skip, plan->d_sphere);
}

template <int CH, bool BF>
static int dispatch_cfg(const pecnn_plan* plan, int cfg, const float* sp, const float* sc, float* sn,
                        const float* theta, float dt, float alpha, const int32_t* skip, hipStream_t st) {
  const int slot = cnn_cfg_slot(cfg);
  switch (cfg) {
    case 0: launch_cnn<CH, BF, 64, 4>(plan, slot, sp, sc, sn, theta, dt, alpha, skip, st); break;
    case 1: launch_cnn<CH, BF, 32, 8>(plan, slot, sp, sc, sn, theta, dt, alpha, skip, st); break;
    case 2: launch_cnn<CH, BF, 16, 16>(plan, slot, sp, sc, sn, theta, dt, alpha, skip, st); break;
    case 3: launch_cnn<CH, BF, 64, 8>(plan, slot, sp, sc, sn, theta, dt, alpha, skip, st); break;
    default: return PECNN_E_INVALID;
  }
  return PECNN_OK;
}

int cnn_forward_bf16_launch(const pecnn_plan*, int, const pecnn_model*, const float*, const float*, float*,
                            const int32_t*, hipStream_t);
int pair_forward_launch(const pecnn_plan*, const pecnn_model*, const float*, float*, const int32_t*, hipStream_t);

int cnn_forward_launch(const pecnn_plan* plan, int cfg, const pecnn_model* m, const float* sp,
                       const float* sc, float* sn, const int32_t* skip, hipStream_t st) {
  if (m->cell == PECNN_CELL_PAIR) return pair_forward_launch(plan, m, sc, sn, skip, st);
  if (m->precision == PECNN_BF16) return cnn_forward_bf16_launch(plan, cfg, m, sp, sc, sn, skip, st);
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
