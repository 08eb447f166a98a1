// bf16 CNN frame (section 3.2, eqs. 6-7, then eq. 5; Fig. 2), the inference hot path.
//
// Same products and lane-slot maps as the generic kernel (cnn_fwd.hip), organised for
// throughput on gfx950:
//  * persistent workgroups walk the batch's tile list; while a tile is computed, the halo of
//    the next tile (S^k, S^{k-1} and the pin flags) is already in flight into registers, as
//    16-byte loads where the rows allow it;
//  * the halo is staged once per tile: FP32 S^k (all six planes), FP32 S^k - S^{k-1} for the
//    position planes, and bf16 copies of both velocity planes, so that velocity taps are plain
//    16-bit LDS reads and only position taps need the FP32 difference with the centre;
//  * every LDS offset of a tap is a lane constant plus a compile-time segment offset;
//  * each wave owns whole rows of the tile and works in quads of four 16-node segments; the
//    head rows repeat the three outputs in every 4-row group, so lane group g finishes segment
//    g of the quad and a quad's 64 results leave as full-row stores.
#include "cnn_common.hpp"
#include "row_pieces.hpp"

namespace pecnn {

typedef __bf16 bf16x4 __attribute__((ext_vector_type(4)));


// WPE: waves per SIMD the register allocation is held to (3 fits the tiles up to 256 nodes).
// VEC: how the halo rows load. 1: every plane row starts 16-byte aligned (W and the instance
// offsets are multiples of 4), so as aligned 16-byte pieces. 2: every instance is at least 4
// wide, so as 16-byte pieces at 4-byte alignment, the piece that would cross the right edge of
// the grid taken at W - 4 and its values moved into place in LDS after staging. 0: as single
// floats.
// EXT: some instance of the batch has a pressure (eq. 3), added as a known external force, or a
// sphere in the constraint of eq. (5); the others skip both uniformly.
template <int CH, int TX, int TY, bool A1, int WPE, int VEC, bool EXT>
__global__ __launch_bounds__(256) __attribute__((amdgpu_waves_per_eu(WPE, WPE))) void cnn_fwd_bf16_kernel(
    const InstDev* __restrict__ inst, const int32_t* __restrict__ prefix, int n_inst, int n_tiles,
    const uint8_t* __restrict__ pin, const float* __restrict__ s_prev, const float* __restrict__ s_cur,
    float* __restrict__ s_next, int64_t N, const float* __restrict__ theta, float dt, float alpha,
    const int32_t* __restrict__ skip, const float* __restrict__ sphere) {
  constexpr int RS = TX + 8;  // LDS row stride: tile column j at 4 + j, halo columns at 3 and 4 + TX
  constexpr int HY = TY + 2;
  constexpr int PLN = HY * RS;
  constexpr int MB = CH / 16, CPL = CH / 4;
  constexpr int SEGX = TX / 16, NSEG = SEGX * TY, SPW = NSEG / 4, RPW = SPW / SEGX;
  static_assert(SPW % 4 == 0 && SPW % SEGX == 0, "tile shape");
  constexpr int QV = TX / 4;
  constexpr int NROW = 6 * HY;
  constexpr int NV = NROW * QV, NVT = (NV + 255) / 256;
  constexpr int NH = NROW * 2, NHT = (NH + 255) / 256;
  constexpr int NP = TX * TY, NPT = (NP + 255) / 256;

  __shared__ __align__(16) float tS[6 * PLN];
  __shared__ __align__(16) float tD[3 * PLN];
  __shared__ __align__(16) __bf16 tV[6 * PLN];  // velocity planes of S^k, then of S^k - S^{k-1}
  __shared__ uint8_t tP[NP];

  const int tid = threadIdx.x;
  const int lane = tid & 63, wave = tid >> 6;
  const int li = lane & 15, g = lane >> 4;

  CnnWeights<CH, true> w;
  load_weights<CH, true>(w, theta, li, g, PLN, RS);
  const ThetaOff O = theta_off(CH);
  const float bias0 = theta[O.bL + 0], bias1 = theta[O.bL + 1], bias2 = theta[O.bL + 2];

  // Lane constants: LDS index of the top-left neighbour of this lane's node in the wave's first
  // segment, so that every tap offset below is a non-negative compile-time immediate.
  const unsigned tl0 = (unsigned)((wave * RPW) * RS + 3 + li);
  const unsigned pos_base = (unsigned)((g < 3 ? g : 2) * PLN) + tl0;
  unsigned vbase[8];
#pragma unroll
  for (int s = 0; s < 8; ++s) {
    const int idx = 8 * g + s;
    int o = RS + 1;  // padding slots read the centre (weight zero)
    if (idx < 27) {
      const int c = idx / 9, oo = idx % 9;
      o = c * PLN + (oo / 3) * RS + (oo % 3);
    }
    vbase[s] = tl0 + (unsigned)o;
  }

  float4 pS[NVT], pP[NVT];
  float hS[NHT], hP[NHT];
  uint8_t pp[NPT];
  const int N32 = (int)N;  // validated: 24 N < 2^32

  int first, stride, count;
  xcd_tile_range(n_tiles, first, stride, count);

  TileCursor tcur;
  cursor_init(tcur);
  // coordinates of tile number it of this workgroup; false when its instance is skipped
  // This workgroup's tiles are first, first + stride, ... below t_end. Tiles of skipped
  // instances are passed over whole: the cursor jumps to the first tile of the sequence beyond
  // the instance, so they cost no loads, staging or compute.
  const int t_end = first + count * stride;
  auto next_tile = [&](int t) -> int {
    while (t < t_end) {
      cursor_seek(tcur, inst, prefix, n_inst, t, skip);
      if (tcur.flag == 0) return t;
      t = first + ((tcur.end - first + stride - 1) / stride) * stride;
    }
    return -1;
  };
  // coordinates of tile t, whose instance the cursor holds
  int ib = 0;  // instance of the tile in I
  auto coords = [&](int t, InstDev& I, int& r0, int& c0) {
    I = tcur.I;
    ib = tcur.b;
    const int lt = t - tcur.start;
    const int tiles_x = (I.W + TX - 1) / TX;
    r0 = (lt / tiles_x) * TY;
    c0 = (lt % tiles_x) * TX;
  };

  // Per-thread item coordinates do not depend on the tile: float4 item i of this thread is
  // channel c, halo row rr, column group q.
  int it_cq[NVT], it_rr[NVT];
#pragma unroll
  for (int i = 0; i < NVT; ++i) {
    const int j = tid + 256 * i;
    const int row = j / QV, q = j - (j / QV) * QV;
    const int c = row / HY;
    it_rr[i] = row - c * HY;
    it_cq[i] = c * N32 + 4 * q;
  }

  // Issue the halo loads of a tile into registers (they stay in flight during compute). Rows
  // and columns are clamped to the grid in the addresses; every load has one code path, so
  // that it writes its final register and nothing waits for it before the tile is staged.
  auto issue = [&](const InstDev& I, int r0, int c0) {
    const int off32 = (int)I.off;
#pragma unroll
    for (int i = 0; i < NVT; ++i) {
      const int j = tid + 256 * i;
      if (NV % 256 == 0 || j < NV) {
        const int q = (j - (j / QV) * QV);
        const int c = (j / QV) / HY;
        const int gi = min(max(r0 + it_rr[i] - 1, 0), I.H - 1);
        const int col = c0 + 4 * q;
        const unsigned rb = (unsigned)(c * N32 + off32 + gi * I.W);
        if constexpr (VEC == 1) {
          // a piece right of the grid loads the last in-grid piece; staging keeps its last column
          const unsigned a = rb + (unsigned)min(col, I.W - 4);
          pS[i] = gld(reinterpret_cast<const float4*>(s_cur), a);
          pP[i] = gld(reinterpret_cast<const float4*>(s_prev), a);
        } else if constexpr (VEC == 2) {
          // the four columns from min(col, W - 4): inside the row for every W >= 4
          const unsigned a = rb + (unsigned)min(col, I.W - 4);
          pS[i] = gld4_dword(s_cur, a);
          pP[i] = gld4_dword(s_prev, a);
        } else {
          const unsigned j0 = rb + min(col, I.W - 1), j1 = rb + min(col + 1, I.W - 1),
                         j2 = rb + min(col + 2, I.W - 1), j3 = rb + min(col + 3, I.W - 1);
          pS[i] = make_float4(gld(s_cur, j0), gld(s_cur, j1), gld(s_cur, j2), gld(s_cur, j3));
          pP[i] = make_float4(gld(s_prev, j0), gld(s_prev, j1), gld(s_prev, j2), gld(s_prev, j3));
        }
      }
    }
#pragma unroll
    for (int i = 0; i < NHT; ++i) {
      const int j = tid + 256 * i;
      if (j < NH) {
        const int row = j >> 1, side = j & 1;
        const int c = row / HY, rr = row - (row / HY) * HY;
        const int gi = min(max(r0 + rr - 1, 0), I.H - 1);
        const int cj = side ? min(c0 + TX, I.W - 1) : max(c0 - 1, 0);
        const unsigned a = (unsigned)(c * N32 + off32 + gi * I.W + cj);
        hS[i] = gld(s_cur, a);
        hP[i] = gld(s_prev, a);
      }
    }
#pragma unroll
    for (int i = 0; i < NPT; ++i) {
      const int j = tid + 256 * i;
      if (NP % 256 == 0 || j < NP) {
        const int ly = j / TX, lx = j - (j / TX) * TX;
        const int gi = min(r0 + ly, I.H - 1), gj = min(c0 + lx, I.W - 1);
        pp[i] = pin[(unsigned)(off32 + gi * I.W + gj)];  // nodes off the grid are never stored
      }
    }
  };

  // Registers -> LDS: FP32 S^k, FP32 position differences in time, bf16 velocity planes.
  auto stage = [&]() {
#pragma unroll
    for (int i = 0; i < NVT; ++i) {
      const int j = tid + 256 * i;
      if (NV % 256 == 0 || j < NV) {
        const int row = j / QV, q = j - (j / QV) * QV;
        const int c = row / HY, rr = row - (row / HY) * HY;
        const int e = rr * RS + 4 + 4 * q;

        *reinterpret_cast<float4*>(&tS[c * PLN + e]) = pS[i];
        const float4 d = make_float4(pS[i].x - pP[i].x, pS[i].y - pP[i].y, pS[i].z - pP[i].z, pS[i].w - pP[i].w);
        if (c < 3) {
          *reinterpret_cast<float4*>(&tD[c * PLN + e]) = d;
        } else {
          bf16x4 vs = {(__bf16)pS[i].x, (__bf16)pS[i].y, (__bf16)pS[i].z, (__bf16)pS[i].w};
          bf16x4 vd = {(__bf16)d.x, (__bf16)d.y, (__bf16)d.z, (__bf16)d.w};
          *reinterpret_cast<bf16x4*>(&tV[(c - 3) * PLN + e]) = vs;
          *reinterpret_cast<bf16x4*>(&tV[c * PLN + e]) = vd;
        }
      }
    }
#pragma unroll
    for (int i = 0; i < NHT; ++i) {
      const int j = tid + 256 * i;
      if (j < NH) {
        const int row = j >> 1, side = j & 1;
        const int c = row / HY, rr = row - (row / HY) * HY;
        const int e = rr * RS + (side ? 4 + TX : 3);
        tS[c * PLN + e] = hS[i];
        const float d = hS[i] - hP[i];
        if (c < 3) {
          tD[c * PLN + e] = d;
        } else {
          tV[(c - 3) * PLN + e] = (__bf16)hS[i];
          tV[c * PLN + e] = (__bf16)d;
        }
      }
    }
#pragma unroll
    for (int i = 0; i < NPT; ++i) {
      const int j = tid + 256 * i;
      if (NP % 256 == 0 || j < NP) tP[j] = pp[i];
    }
  };

  int t = next_tile(first);
  if (t < 0) return;  // uniform over the workgroup
  InstDev I;
  int r0 = 0, c0 = 0;
  coords(t, I, r0, c0);
  issue(I, r0, c0);

  for (;;) {
    const InstDev Ic = I;
    const int ibc = ib;
    const int rc0 = r0, cc0 = c0;
    // every prefetched register is consumed here on every path, so the next loads that reuse
    // them never wait on older stores
    stage();
    __syncthreads();
    if (VEC == 1 && cc0 + TX > Ic.W) {
      // a tile crossing the right edge of the grid: its 16-byte pieces right of the edge hold
      // the last in-grid piece, but the taps of the last column read the clamped copy of it
      // one column further; write that column (the only one off the grid that a node reads)
      const int dst = 4 + (Ic.W - cc0);
      for (int e = tid; e < 15 * HY; e += 256) {
        const int pl = e / HY, rr = e - (e / HY) * HY;
        const int o = rr * RS + dst;
        if (pl < 6) tS[pl * PLN + o] = tS[pl * PLN + o - 1];
        else if (pl < 9) tD[(pl - 6) * PLN + o] = tD[(pl - 6) * PLN + o - 1];
        else tV[(pl - 9) * PLN + o] = tV[(pl - 9) * PLN + o - 1];
      }
      __syncthreads();
    }
    if (VEC == 2 && cc0 + TX > Ic.W) {
      // a tile crossing the right edge of the grid, its pieces loaded from min(col, W - 4): the
      // piece holding the last in-grid column sits sh columns right of its source (row_pieces.hpp)
      const int e = Ic.W - cc0, qs = (e - 1) >> 2, sh = 4 * qs + 4 - e;
      for (int it = tid; it < 15 * HY; it += 256) {
        const int pl = it / HY, rr = it - (it / HY) * HY;
        const int o = rr * RS + 4 + 4 * qs;
        if (pl < 6) shift_piece_lds(&tS[pl * PLN + o], sh);
        else if (pl < 9) shift_piece_lds(&tD[(pl - 6) * PLN + o], sh);
        else shift_piece_lds(&tV[(pl - 9) * PLN + o], sh);
      }
      __syncthreads();
    }
    // prefetch the next tile while this one is computed (after the last tile, a reload of this
    // one: every iteration issues the same loads, with no branch around them)
    const int tn = next_tile(t + stride);
    if (tn >= 0) coords(tn, I, r0, c0);
    issue(I, r0, c0);

    {
      // per-instance constant part of eq. (5): b_L + dt a_ext
      const float cx = __builtin_fmaf(dt, Ic.ax, bias0), cy = __builtin_fmaf(dt, Ic.ay, bias1),
                  cz = __builtin_fmaf(dt, Ic.az, bias2);
      float e0 = 0.f, e1 = 0.f, e2 = 0.f;  // head output of the segment this lane group finishes
#pragma unroll
      for (int k = 0; k < SPW; ++k) {
        constexpr int C0 = RS + 1;  // centre relative to the top-left neighbour
        const unsigned so = (unsigned)((k / SEGX) * RS + (k % SEGX) * 16);
        // im2col: position taps of channel g as FP32 differences with the centre, bf16 velocity taps
        bf16x8 bS0, bD0, bS1, bD1;
        const float cs = tS[pos_base + so + C0], cd = tD[pos_base + so + C0];
#pragma unroll
        for (int s = 0; s < 8; ++s) {
          const int o = s + (s >= 4 ? 1 : 0);
          const unsigned d = (unsigned)((o / 3) * RS + (o % 3));
          bS0[s] = (__bf16)(tS[pos_base + so + d] - cs);
          bD0[s] = (__bf16)(tD[pos_base + so + d] - cd);
        }
#pragma unroll
        for (int s = 0; s < 8; ++s) {
          bS1[s] = tV[vbase[s] + so];
          bD1[s] = tV[vbase[s] + so + 3 * PLN];
        }
        f32x4 accP[MB], accX[MB];
#pragma unroll
        for (int mb = 0; mb < MB; ++mb) {
          accP[mb] = __builtin_amdgcn_mfma_f32_16x16x32_bf16(w.conv[mb][0], bS0, f32x4{0.f, 0.f, 0.f, 0.f}, 0, 0, 0);
          accX[mb] = __builtin_amdgcn_mfma_f32_16x16x32_bf16(w.conv[mb][0], bD0, f32x4{0.f, 0.f, 0.f, 0.f}, 0, 0, 0);
        }
#pragma unroll
        for (int mb = 0; mb < MB; ++mb) {
          accP[mb] = __builtin_amdgcn_mfma_f32_16x16x32_bf16(w.conv[mb][1], bS1, accP[mb], 0, 0, 0);
          accX[mb] = __builtin_amdgcn_mfma_f32_16x16x32_bf16(w.conv[mb][1], bD1, accX[mb], 0, 0, 0);
        }
        // nonlinear branch: [a; b] = [A; B] phi
        bf16x8 bphi;
#pragma unroll
        for (int e = 0; e < 8; ++e) bphi[e] = (__bf16)(e < CPL ? accP[(e & 7) >> 2][e & 3] : 0.f);
        f32x4 ab[2 * MB];
#pragma unroll
        for (int mb = 0; mb < 2 * MB; ++mb)
          ab[mb] = __builtin_amdgcn_mfma_f32_16x16x32_bf16(w.mix[mb], bphi, f32x4{0.f, 0.f, 0.f, 0.f}, 0, 0, 0);
        // ISRU branches and the derivative product (FP32)
        float F[3 * CPL];
#pragma unroll
        for (int e = 0; e < CPL; ++e) {
          const float ph = accP[e >> 2][e & 3];
          const float z = ab[e >> 2][e & 3] * ab[MB + (e >> 2)][e & 3];
          const float t1 = A1 ? __builtin_fmaf(ph, ph, 1.f) : __builtin_fmaf(alpha * ph, ph, 1.f);
          const float t2 = A1 ? __builtin_fmaf(z, z, 1.f) : __builtin_fmaf(alpha * z, z, 1.f);
          const float gs = ph * __builtin_amdgcn_rsqf(t1);
          F[e] = ph;
          F[CPL + e] = z * __builtin_amdgcn_rsqf(t2);
          F[2 * CPL + e] = accX[e >> 2][e & 3] * gs;
        }
        f32x4 hv;
        if constexpr (CH == 32) {
          bf16x8 bn, bd;
#pragma unroll
          for (int e = 0; e < 8; ++e) {
            bn[e] = (__bf16)F[CPL + e];
            bd[e] = (__bf16)F[2 * CPL + e];
          }
          hv = __builtin_amdgcn_mfma_f32_16x16x32_bf16(w.head[0], bphi, f32x4{0.f, 0.f, 0.f, 0.f}, 0, 0, 0);
          hv = __builtin_amdgcn_mfma_f32_16x16x32_bf16(w.head[1], bn, hv, 0, 0, 0);
          hv = __builtin_amdgcn_mfma_f32_16x16x32_bf16(w.head[2], bd, hv, 0, 0, 0);
        } else {
          hv = head_mfma<CH>(w, F);
        }
        // every lane group holds the three outputs; group (k & 3) keeps this segment's
        if (g == (k & 3)) {
          e0 = hv[0];
          e1 = hv[1];
          e2 = hv[2];
        }

        if ((k & 3) == 3) {
          // quad epilogue: lane group g finishes segment (k - 3 + g); eq. (5) with pins and wind
          const int kk = k - 3 + g;
          const int sy = wave * RPW + kk / SEGX, sx = (kk % SEGX) * 16 + li;
          const int i = rc0 + sy, j = cc0 + sx;
          const int cell = (sy + 1) * RS + 4 + sx;
          if (i < Ic.H && j < Ic.W) {
            const unsigned p = (unsigned)((int)Ic.off + i * Ic.W + j);
            float nx = (tS[3 * PLN + cell] + e0) + cx;
            float ny = (tS[4 * PLN + cell] + e1) + cy;
            float nz = (tS[5 * PLN + cell] + e2) + cz;
            if constexpr (EXT) {
              if (Ic.pres != 0.f) {  // eq. (3) at S^k, uniform over the workgroup
                const int nb[4] = {1, RS, -1, -RS};  // right, down, left, up
                float d[4][3];
#pragma unroll
                for (int q = 0; q < 4; ++q)
#pragma unroll
                  for (int c = 0; c < 3; ++c) d[q][c] = tS[c * PLN + cell + nb[q]] - tS[c * PLN + cell];
                const bool has[4] = {j + 1 < Ic.W, i + 1 < Ic.H, j > 0, i > 0};
                float p0, p1, p2;
                pressure_pairs(d, has, p0, p1, p2);
                const float cp = dt * Ic.pres / Ic.mass;
                nx = __builtin_fmaf(cp, p0, nx);
                ny = __builtin_fmaf(cp, p1, ny);
                nz = __builtin_fmaf(cp, p2, nz);
              }
            }
            const bool pinned = tP[sy * TX + sx] != 0;
            if (pinned) nx = ny = nz = 0.f;
            float y0, y1, y2;
            if constexpr (EXT) {
              if (!pinned) {
                sphere_update(sphere + ibc * kSphereStride, dt, tS[cell], tS[PLN + cell], tS[2 * PLN + cell], nx, ny,
                              nz, y0, y1, y2);
              } else {
                y0 = tS[cell];
                y1 = tS[PLN + cell];
                y2 = tS[2 * PLN + cell];
              }
            } else {
              y0 = __builtin_fmaf(dt, nx, tS[cell]);
              y1 = __builtin_fmaf(dt, ny, tS[PLN + cell]);
              y2 = __builtin_fmaf(dt, nz, tS[2 * PLN + cell]);
            }
            gst(s_next, 3 * N32 + p, nx);
            gst(s_next, 4 * N32 + p, ny);
            gst(s_next, 5 * N32 + p, nz);
            gst(s_next, p, y0);
            gst(s_next, N32 + p, y1);
            gst(s_next, 2 * N32 + p, y2);
          }
        }
      }
    }
    __syncthreads();
    if (tn < 0) break;  // uniform
    t = tn;
  }
}

template <int CH, int TX, int TY, bool A1, int WPE, int VEC, bool EXT>
static void launch_bf16(const pecnn_plan* plan, int slot, const float* sp, const float* sc, float* sn,
                        const float* theta, float dt, float alpha, const int32_t* skip, hipStream_t st) {
  const int n_tiles = plan->n_tiles[slot];
  static int per_cu = 0;  // resident workgroups per CU of this instantiation
  if (per_cu == 0) {
    int v = 0;
    if (hipOccupancyMaxActiveBlocksPerMultiprocessor(&v, cnn_fwd_bf16_kernel<CH, TX, TY, A1, WPE, VEC, EXT>, 256, 0) !=
            hipSuccess ||
        v < 1)
      v = 2;
    per_cu = v;
  }
  int grid = num_cus() * per_cu;
  const int need = ((n_tiles + 7) / 8) * 8;
  if (need < grid) grid = need;
  if (grid < 8) grid = 8;
  hipLaunchKernelGGL((cnn_fwd_bf16_kernel<CH, TX, TY, A1, WPE, VEC, EXT>), dim3(grid), dim3(256), 0, st, plan->d_inst,
                     plan->d_prefix[slot], plan->n, n_tiles, plan->pin, sp, sc, sn, plan->total, theta, dt, alpha,
                     skip, plan->d_sphere);
}

template <int CH, bool A1, int VEC, bool EXT>
static int bf16_cfg_v(const pecnn_plan* plan, int cfg, const float* sp, const float* sc, float* sn,
                      const float* theta, float dt, float alpha, const int32_t* skip, hipStream_t st) {
  const int slot = cnn_cfg_slot(cfg);
  switch (cfg) {
    case 0: launch_bf16<CH, 64, 4, A1, 3, VEC, EXT>(plan, slot, sp, sc, sn, theta, dt, alpha, skip, st); break;
    case 1: launch_bf16<CH, 32, 8, A1, 3, VEC, EXT>(plan, slot, sp, sc, sn, theta, dt, alpha, skip, st); break;
    case 2: launch_bf16<CH, 16, 16, A1, 3, VEC, EXT>(plan, slot, sp, sc, sn, theta, dt, alpha, skip, st); break;
    case 3: launch_bf16<CH, 64, 8, A1, 2, VEC, EXT>(plan, slot, sp, sc, sn, theta, dt, alpha, skip, st); break;
    default: return PECNN_E_INVALID;
  }
  return PECNN_OK;
}

template <int CH, bool A1>
static int bf16_cfg(const pecnn_plan* plan, int cfg, const float* sp, const float* sc, float* sn,
                    const float* theta, float dt, float alpha, const int32_t* skip, hipStream_t st) {
  const int min_w = plan_min_width(plan->W, plan->n);
  if (plan->has_pressure || plan->has_sphere) {
    if (plan->vec4) return bf16_cfg_v<CH, A1, 1, true>(plan, cfg, sp, sc, sn, theta, dt, alpha, skip, st);
    if (min_w >= 4) return bf16_cfg_v<CH, A1, 2, true>(plan, cfg, sp, sc, sn, theta, dt, alpha, skip, st);
    return bf16_cfg_v<CH, A1, 0, true>(plan, cfg, sp, sc, sn, theta, dt, alpha, skip, st);
  }
  if (plan->vec4) return bf16_cfg_v<CH, A1, 1, false>(plan, cfg, sp, sc, sn, theta, dt, alpha, skip, st);
  if (min_w >= 4) return bf16_cfg_v<CH, A1, 2, false>(plan, cfg, sp, sc, sn, theta, dt, alpha, skip, st);
  return bf16_cfg_v<CH, A1, 0, false>(plan, cfg, sp, sc, sn, theta, dt, alpha, skip, st);
}

int cnn_forward_bf16_launch(const pecnn_plan* plan, int cfg, const pecnn_model* m, const float* sp,
                            const float* sc, float* sn, const int32_t* skip, hipStream_t st) {
  const bool a1 = m->isru_alpha == 1.0f;
  int rc;
  if (m->ch == 16)
    rc = a1 ? bf16_cfg<16, true>(plan, cfg, sp, sc, sn, m->theta, m->dt, m->isru_alpha, skip, st)
            : bf16_cfg<16, false>(plan, cfg, sp, sc, sn, m->theta, m->dt, m->isru_alpha, skip, st);
  else
    rc = a1 ? bf16_cfg<32, true>(plan, cfg, sp, sc, sn, m->theta, m->dt, m->isru_alpha, skip, st)
            : bf16_cfg<32, false>(plan, cfg, sp, sc, sn, m->theta, m->dt, m->isru_alpha, skip, st);
  if (rc != PECNN_OK) return rc;
  PECNN_LAUNCH_CHECK("cnn_fwd_bf16_kernel");
  return PECNN_OK;
}

}  // namespace pecnn
