// Mass-spring cloth step (section 3.1, eqs. 1, 2, 4, 5) on gfx950.
//
// One workgroup owns a TX x TY tile of one instance; the six state planes of the tile plus a
// two-node halo (the stencil radius of the bending springs) are staged in LDS, then each thread
// integrates RY nodes. Workgroups are persistent over the batch's tile list: the next tile's
// loads (16-byte where the rows allow it, plus its pin flags) are issued into registers before
// the current tile is computed, so HBM latency hides behind the spring arithmetic. Each XCD
// walks a contiguous tile range, so halo rows shared by neighbouring tiles meet in one L2.
#include "common.hpp"
#include "row_pieces.hpp"

#include <type_traits>

namespace pecnn {

// The 12 springs of a node: (row offset, column offset, family).
// Family 0 structural (rest h), 1 shear (rest sqrt(2) h), 2 bend (rest 2h).
struct Spring { int dy, dx, fam; };
__device__ constexpr Spring kSprings[12] = {
    {0, 1, 0}, {0, -1, 0}, {1, 0, 0}, {-1, 0, 0},
    {1, 1, 1}, {1, -1, 1}, {-1, 1, 1}, {-1, -1, 1},
    {0, 2, 2}, {0, -2, 2}, {2, 0, 2}, {-2, 0, 2}};

// VEC: how the tile rows load. 1: every plane row starts 16-byte aligned (W and the instance
// offsets are multiples of 4), so as aligned 16-byte pieces. 2: every cloth is at least 4 wide,
// so as 16-byte pieces at 4-byte alignment, the piece that would cross the right edge taken at
// W - 4 and shifted into place in LDS after staging. 0: as single floats.
// EXT: some instance of the batch has a pressure (eq. 3) or a sphere in its constraint; the
// others skip both uniformly.
// PAIR: instead of the springs, one frame of the paper's own cell read literally (section 3.2):
// twelve channels, one per stencil neighbour j, phi_c = s_c (x_j - x), xi_c = s_c (v_j - v) with
// the same frozen two-point filter on each axis (eq. 6; zero when j is off the grid), then per axis
// dv = sum_c [wL_c phi_c + wN_c sigma(phi_c) + wD_c xi_c sigma(phi_c)] + b_L (eq. 7) and eq. (5)
// with pins, wind and pressure. It has the springs' stencil, so it shares their tiles and halo.
struct PairArgs {
  const float* theta;    // s[12] | wL[12] | wN[12] | wD[12] | bL[3]
  float alpha, dt;       // ISRU parameter, frame time step
  const int32_t* skip;   // instances to leave alone (fallen back), or null
};

template <int TX, int TY, int RY, int VEC, bool EXT, bool PAIR = false>
__global__ __launch_bounds__(TX*(TY / RY)) void ms_step_kernel(
    const InstDev* __restrict__ inst, const int32_t* __restrict__ prefix, int n_inst, int n_tiles,
    const uint8_t* __restrict__ pin, const float* __restrict__ s_in, float* __restrict__ s_out,
    int64_t N, MsParamsDev P, const uint8_t* __restrict__ active, PairArgs pa, const float* __restrict__ sphere) {
  constexpr int NT = TX * (TY / RY);
  constexpr int RS = TX + 8;  // LDS row stride: tile column j at 4 + j, halo columns 2, 3 and 4+TX, 5+TX
  constexpr int HY = TY + 4;
  constexpr int PLN = HY * RS;
  constexpr int QV = TX / 4;
  constexpr int NROW = 6 * HY;
  constexpr int NV = NROW * QV, NVT = (NV + NT - 1) / NT;
  constexpr int NH = NROW * 4, NHT = (NH + NT - 1) / NT;
  constexpr int NP = TX * TY, NPT = (NP + NT - 1) / NT;
  __shared__ __align__(16) float lds[6 * PLN];
  __shared__ uint8_t tP[NP];

  const int tid = threadIdx.x;
  const int tx = tid % TX;
  const int ty0 = (tid / TX) * RY;
  float4 pv[NVT];
  float ph[NHT];
  uint8_t pp[NPT];

  int first, stride, count;
  xcd_tile_range(n_tiles, first, stride, count);

  TileCursor tcur;
  cursor_init(tcur);
  // coordinates of tile number it of this workgroup; false when its instance is inactive
  // This workgroup's tiles are first, first + stride, ... below t_end. Tiles of skipped
  // instances are passed over whole: the cursor jumps to the first tile of the sequence beyond
  // the instance, so they cost no loads, staging or compute.
  const int t_end = first + count * stride;
  auto next_tile = [&](int t) -> int {
    while (t < t_end) {
      if constexpr (PAIR) {
        cursor_seek(tcur, inst, prefix, n_inst, t, pa.skip);
        if (tcur.flag == 0) return t;
      } else {
        cursor_seek(tcur, inst, prefix, n_inst, t, active);
        if ((active == nullptr || tcur.flag != 0)) return t;
      }
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
  // Issue the loads of a tile and its two-node halo (rows and columns clamped to the grid; the
  // clamped copies are never used as springs, whose ends are checked against the grid). Every
  // load has one code path, so that it writes its final register and nothing waits for it
  // before the tile is staged.
  auto issue = [&](const InstDev& I, int r0, int c0) {
#pragma unroll
    for (int i = 0; i < NVT; ++i) {
      const int j = tid + NT * i;
      if (NV % NT == 0 || j < NV) {
        const int row = j / QV, q = j - (j / QV) * QV;
        const int c = row / HY, rr = row - (row / HY) * HY;
        const int gi = min(max(r0 + rr - 2, 0), I.H - 1);
        const int col = c0 + 4 * q;
        const unsigned rb = (unsigned)(c * (int)N + (int)I.off + gi * I.W);
        if constexpr (VEC == 1) {
          // a piece right of the grid loads the last in-grid piece (never a spring end)
          pv[i] = gld(reinterpret_cast<const float4*>(s_in), rb + (unsigned)min(col, I.W - 4));
        } else if constexpr (VEC == 2) {
          // the four columns from min(col, W - 4): inside the row for every W >= 4
          pv[i] = gld4_dword(s_in, rb + (unsigned)min(col, I.W - 4));
        } else {
          pv[i] = make_float4(gld(s_in, rb + min(col, I.W - 1)), gld(s_in, rb + min(col + 1, I.W - 1)),
                              gld(s_in, rb + min(col + 2, I.W - 1)), gld(s_in, rb + min(col + 3, I.W - 1)));
        }
      }
    }
#pragma unroll
    for (int i = 0; i < NHT; ++i) {
      const int j = tid + NT * i;
      if (NH % NT == 0 || j < NH) {
        const int row = j >> 2, side = j & 3;  // columns c0-2, c0-1, c0+TX, c0+TX+1
        const int c = row / HY, rr = row - (row / HY) * HY;
        const int gi = min(max(r0 + rr - 2, 0), I.H - 1);
        const int gj = min(max(side < 2 ? c0 - 2 + side : c0 + TX + side - 2, 0), I.W - 1);
        ph[i] = gld(s_in, (unsigned)(c * (int)N + (int)I.off + gi * I.W + gj));
      }
    }
#pragma unroll
    for (int i = 0; i < NPT; ++i) {
      const int j = tid + NT * i;
      if (NP % NT == 0 || j < NP) {
        const int ly = j / TX, lx = j - (j / TX) * TX;
        const int gi = min(r0 + ly, I.H - 1), gj = min(c0 + lx, I.W - 1);
        pp[i] = pin[(unsigned)((int)I.off + gi * I.W + gj)];  // nodes off the grid are never stored
      }
    }
  };
  auto stage = [&]() {
#pragma unroll
    for (int i = 0; i < NVT; ++i) {
      const int j = tid + NT * i;
      if (NV % NT == 0 || j < NV) {
        const int row = j / QV, q = j - (j / QV) * QV;
        const int c = row / HY, rr = row - (row / HY) * HY;
        *reinterpret_cast<float4*>(&lds[c * PLN + rr * RS + 4 + 4 * q]) = pv[i];
      }
    }
#pragma unroll
    for (int i = 0; i < NHT; ++i) {
      const int j = tid + NT * i;
      if (NH % NT == 0 || j < NH) {
        const int row = j >> 2, side = j & 3;
        const int c = row / HY, rr = row - (row / HY) * HY;
        lds[c * PLN + rr * RS + (side < 2 ? 2 + side : 2 + TX + side)] = ph[i];
      }
    }
#pragma unroll
    for (int i = 0; i < NPT; ++i) {
      const int j = tid + NT * i;
      if (NP % NT == 0 || j < NP) tP[j] = pp[i];
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
    if (VEC == 2 && cc0 + TX > Ic.W) {
      // a tile crossing the right edge of the grid, its pieces loaded from min(col, W - 4): the
      // piece holding the last in-grid column sits sh columns right of its source (row_pieces.hpp)
      const int e = Ic.W - cc0, qs = (e - 1) >> 2, sh = 4 * qs + 4 - e;
      for (int it = tid; it < 6 * HY; it += NT) {
        const int pl = it / HY, rr = it - (it / HY) * HY;
        shift_piece_lds(&lds[pl * PLN + rr * RS + 4 + 4 * qs], sh);
      }
      __syncthreads();
    }
    // prefetch the next tile (after the last tile, a reload of this one: no branch around it)
    const int tn = next_tile(t + stride);
    if (tn >= 0) coords(tn, I, r0, c0);
    issue(I, r0, c0);

    {
      const float L[3] = {Ic.h, Ic.h * 1.41421356237309515f, 2.f * Ic.h};
      const float tiny = 1e-24f * Ic.h * Ic.h;
      const float sc = P.dt / Ic.mass;
      const float nmu = -P.mu;
      // eq. (4) plus the wind, constant part: m (g + a_ext)
      const float g0 = Ic.mass * (P.g[0] + Ic.ax), g1 = Ic.mass * (P.g[1] + Ic.ay), g2 = Ic.mass * (P.g[2] + Ic.az);
#pragma unroll
      for (int ry = 0; ry < RY; ++ry) {
        const int ly = ty0 + ry;
        const int i = rc0 + ly, j = cc0 + tx;
        if (i < Ic.H && j < Ic.W) {
          const unsigned p = (unsigned)((int)Ic.off + i * Ic.W + j);
          const int e = (ly + 2) * RS + 4 + tx;
          const float x0 = lds[e], x1 = lds[PLN + e], x2 = lds[2 * PLN + e];
          const float v0 = lds[3 * PLN + e], v1 = lds[4 * PLN + e], v2 = lds[5 * PLN + e];
          float n0 = 0.f, n1 = 0.f, n2 = 0.f;
          if constexpr (PAIR) {
            if (!tP[ly * TX + tx]) {
              float acc[3] = {pa.theta[48], pa.theta[49], pa.theta[50]};  // b_L
              const float xv[6] = {x0, x1, x2, v0, v1, v2};
#pragma unroll
              for (int q = 0; q < 12; ++q) {
                const Spring S = kSprings[q];
                const int ii = i + S.dy, jj = j + S.dx;
                if (ii < 0 || ii >= Ic.H || jj < 0 || jj >= Ic.W) continue;  // no channel off the grid
                const int en = e + S.dy * RS + S.dx;
                const float sq = pa.theta[q], wl = pa.theta[12 + q], wn = pa.theta[24 + q], wd = pa.theta[36 + q];
#pragma unroll
                for (int a = 0; a < 3; ++a) {
                  const float phi = sq * (lds[a * PLN + en] - xv[a]);
                  const float xi = sq * (lds[(3 + a) * PLN + en] - xv[3 + a]);
                  const float sg = phi * __builtin_amdgcn_rsqf(__builtin_fmaf(pa.alpha * phi, phi, 1.f));
                  acc[a] = __builtin_fmaf(wl, phi, acc[a]);
                  acc[a] = __builtin_fmaf(wn, sg, acc[a]);
                  acc[a] = __builtin_fmaf(wd * xi, sg, acc[a]);
                }
              }
              n0 = (v0 + acc[0]) + pa.dt * Ic.ax;
              n1 = (v1 + acc[1]) + pa.dt * Ic.ay;
              n2 = (v2 + acc[2]) + pa.dt * Ic.az;
              if constexpr (EXT) {
                if (Ic.pres != 0.f) {  // eq. (3) at S^k, a known external force
                  const int nb[4] = {1, RS, -1, -RS};  // right, down, left, up
                  float d[4][3];
#pragma unroll
                  for (int k = 0; k < 4; ++k)
#pragma unroll
                    for (int a = 0; a < 3; ++a) d[k][a] = lds[a * PLN + e + nb[k]] - xv[a];
                  const bool has[4] = {j + 1 < Ic.W, i + 1 < Ic.H, j > 0, i > 0};
                  float p0, p1, p2;
                  pressure_pairs(d, has, p0, p1, p2);
                  const float cp = pa.dt * Ic.pres / Ic.mass;
                  n0 = __builtin_fmaf(cp, p0, n0);
                  n1 = __builtin_fmaf(cp, p1, n1);
                  n2 = __builtin_fmaf(cp, p2, n2);
                }
              }
            }
          } else if (!tP[ly * TX + tx]) {
            float f0 = __builtin_fmaf(-P.drag, v0, g0);
            float f1 = __builtin_fmaf(-P.drag, v1, g1);
            float f2 = __builtin_fmaf(-P.drag, v2, g2);
            // One spring loop, two instances. Tiles whose springs all have both ends on the grid take
            // every spring as it is. Edge tiles take the same loop and zero the coefficient of a
            // spring whose far end is off the grid: that end reads a clamped copy in the halo, so
            // every value stays finite, and a zero coefficient adds nothing to the force. Eight
            // comparisons per node and one select per spring replace a branch per spring. A
            // degenerate spring (r ~ 0) contributes nothing either: with ir = 0 both coefficients
            // vanish.
            auto springs = [&](auto masked) {
              bool u1 = true, u2 = true, d1 = true, d2 = true, l1 = true, l2 = true, r1 = true, r2 = true;
              if constexpr (decltype(masked)::value) {
                u1 = i >= 1;
                u2 = i >= 2;
                d1 = i + 1 < Ic.H;
                d2 = i + 2 < Ic.H;
                l1 = j >= 1;
                l2 = j >= 2;
                r1 = j + 1 < Ic.W;
                r2 = j + 2 < Ic.W;
              }
#pragma unroll
              for (int q = 0; q < 12; ++q) {
                const Spring S = kSprings[q];
                const int en = e + S.dy * RS + S.dx;
                const float d0 = x0 - lds[en], d1_ = x1 - lds[PLN + en], d2_ = x2 - lds[2 * PLN + en];
                const float w0 = v0 - lds[3 * PLN + en], w1 = v1 - lds[4 * PLN + en], w2 = v2 - lds[5 * PLN + en];
                const float rr = __builtin_fmaf(d2_, d2_, __builtin_fmaf(d1_, d1_, d0 * d0));
                const float ir = rr > tiny ? __builtin_amdgcn_rsqf(rr) : 0.f;
                const float r = rr * ir;
                const float ce = (P.k[S.fam] * (L[S.fam] - r)) * ir;  // eq. (1): -k (r - L) / r
                const float vx = __builtin_fmaf(w2, d2_, __builtin_fmaf(w1, d1_, w0 * d0));
                float cf = __builtin_fmaf((nmu * ir) * ir, vx, ce);   // eq. (2): -mu (v.x) / r^2
                if constexpr (decltype(masked)::value) {
                  const bool rok = S.dy == 0 ? true : S.dy == 1 ? d1 : S.dy == 2 ? d2 : S.dy == -1 ? u1 : u2;
                  const bool cok = S.dx == 0 ? true : S.dx == 1 ? r1 : S.dx == 2 ? r2 : S.dx == -1 ? l1 : l2;
                  cf = (rok && cok) ? cf : 0.f;
                }
                f0 = __builtin_fmaf(cf, d0, f0);
                f1 = __builtin_fmaf(cf, d1_, f1);
                f2 = __builtin_fmaf(cf, d2_, f2);
                // compiler fence: each spring's LDS reads stay next to their use instead of all 72
                // being hoisted, which would cost occupancy
                asm volatile("" ::: "memory");
              }
            };
            // workgroup-uniform: every spring of every node of the tile has both ends on the grid
            const bool interior = rc0 >= 2 && cc0 >= 2 && rc0 + TY + 2 <= Ic.H && cc0 + TX + 2 <= Ic.W;
            if (interior) springs(std::false_type{});
            else springs(std::true_type{});
            if constexpr (EXT) {
              if (Ic.pres != 0.f) {  // eq. (3), uniform over the workgroup
                const int nb[4] = {1, RS, -1, -RS};  // right, down, left, up
                float d[4][3];
#pragma unroll
                for (int k = 0; k < 4; ++k) {
                  d[k][0] = lds[e + nb[k]] - x0;
                  d[k][1] = lds[PLN + e + nb[k]] - x1;
                  d[k][2] = lds[2 * PLN + e + nb[k]] - x2;
                }
                const bool has[4] = {j + 1 < Ic.W, i + 1 < Ic.H, j > 0, i > 0};
                float s0, s1, s2;
                pressure_pairs(d, has, s0, s1, s2);
                f0 = __builtin_fmaf(Ic.pres, s0, f0);
                f1 = __builtin_fmaf(Ic.pres, s1, f1);
                f2 = __builtin_fmaf(Ic.pres, s2, f2);
              }
            }
            // eq. (5): semi-implicit Euler
            n0 = __builtin_fmaf(sc, f0, v0);
            n1 = __builtin_fmaf(sc, f1, v1);
            n2 = __builtin_fmaf(sc, f2, v2);
          }
          const int N32 = (int)N;
          const float dto = PAIR ? pa.dt : P.dt;
          float y0, y1, y2;
          if constexpr (EXT) {
            if (!tP[ly * TX + tx]) {
              sphere_update(sphere + ibc * kSphereStride, dto, x0, x1, x2, n0, n1, n2, y0, y1, y2);
            } else {
              y0 = __builtin_fmaf(dto, n0, x0);
              y1 = __builtin_fmaf(dto, n1, x1);
              y2 = __builtin_fmaf(dto, n2, x2);
            }
          } else {
            y0 = __builtin_fmaf(dto, n0, x0);
            y1 = __builtin_fmaf(dto, n1, x1);
            y2 = __builtin_fmaf(dto, n2, x2);
          }
          gst(s_out, 3 * N32 + p, n0);
          gst(s_out, 4 * N32 + p, n1);
          gst(s_out, 5 * N32 + p, n2);
          gst(s_out, p, y0);
          gst(s_out, N32 + p, y1);
          gst(s_out, 2 * N32 + p, y2);
        }
      }
    }
    __syncthreads();
    if (tn < 0) break;  // uniform
    t = tn;
  }
}

static int grid_for(int n_tiles, int per_cu) {
  int g = num_cus() * per_cu;
  int need = ((n_tiles + 7) / 8) * 8;
  if (need < g) g = need;
  if (g < 8) g = 8;
  return g;
}

template <int TX, int TY, int RY>
static void launch_ms(const pecnn_plan* plan, int slot, const MsParamsDev& P, const float* in,
                      float* out, const uint8_t* active, hipStream_t st) {
  const int n_tiles = plan->n_tiles[slot];
  const int grid = grid_for(n_tiles, 8);
  auto go = [&](auto kernel) {
    hipLaunchKernelGGL(kernel, dim3(grid), dim3(TX * (TY / RY)), 0, st, plan->d_inst, plan->d_prefix[slot], plan->n,
                       n_tiles, plan->pin, in, out, plan->total, P, active, PairArgs{}, plan->d_sphere);
  };
  const int vec = plan->vec4 ? 1 : (plan_min_width(plan->W, plan->n) >= 4 ? 2 : 0);
  if (plan->has_pressure || plan->has_sphere) {
    if (vec == 1) go(ms_step_kernel<TX, TY, RY, 1, true>);
    else if (vec == 2) go(ms_step_kernel<TX, TY, RY, 2, true>);
    else go(ms_step_kernel<TX, TY, RY, 0, true>);
  } else {
    if (vec == 1) go(ms_step_kernel<TX, TY, RY, 1, false>);
    else if (vec == 2) go(ms_step_kernel<TX, TY, RY, 2, false>);
    else go(ms_step_kernel<TX, TY, RY, 0, false>);
  }
}

template <int TX, int TY, int RY>
static void launch_pair(const pecnn_plan* plan, int slot, const PairArgs& pa, const float* in, float* out,
                        hipStream_t st) {
  const int n_tiles = plan->n_tiles[slot];
  const int grid = grid_for(n_tiles, 8);
  const MsParamsDev P{};
  auto go = [&](auto kernel) {
    hipLaunchKernelGGL(kernel, dim3(grid), dim3(TX * (TY / RY)), 0, st, plan->d_inst, plan->d_prefix[slot], plan->n,
                       n_tiles, plan->pin, in, out, plan->total, P, (const uint8_t*)nullptr, pa, plan->d_sphere);
  };
  const int vec = plan->vec4 ? 1 : (plan_min_width(plan->W, plan->n) >= 4 ? 2 : 0);
  if (plan->has_pressure || plan->has_sphere) {
    if (vec == 1) go(ms_step_kernel<TX, TY, RY, 1, true, true>);
    else if (vec == 2) go(ms_step_kernel<TX, TY, RY, 2, true, true>);
    else go(ms_step_kernel<TX, TY, RY, 0, true, true>);
  } else {
    if (vec == 1) go(ms_step_kernel<TX, TY, RY, 1, false, true>);
    else if (vec == 2) go(ms_step_kernel<TX, TY, RY, 2, false, true>);
    else go(ms_step_kernel<TX, TY, RY, 0, false, true>);
  }
}

// One frame of the pair cell on the simulator's tiles (configuration plan->ms_cfg).
int pair_forward_launch(const pecnn_plan* plan, const pecnn_model* m, const float* sc, float* sn,
                        const int32_t* skip, hipStream_t st) {
  const int cfg = plan->ms_cfg;
  const int slot = ms_cfg_slot(cfg);
  const PairArgs pa{m->theta, m->isru_alpha, m->dt, skip};
  switch (cfg) {
    case 0: launch_pair<32, 8, 1>(plan, slot, pa, sc, sn, st); break;
    case 1: launch_pair<64, 4, 1>(plan, slot, pa, sc, sn, st); break;
    case 2: launch_pair<16, 16, 1>(plan, slot, pa, sc, sn, st); break;
    case 3: launch_pair<32, 16, 2>(plan, slot, pa, sc, sn, st); break;
    case 4: launch_pair<64, 8, 2>(plan, slot, pa, sc, sn, st); break;
    default: return PECNN_E_INVALID;
  }
  PECNN_LAUNCH_CHECK("ms_step_kernel (pair cell)");
  return PECNN_OK;
}

MsParamsDev ms_params_dev(const cloth_ms_params* p) {
  MsParamsDev d;
  d.k[0] = p->k_struct;
  d.k[1] = p->k_shear;
  d.k[2] = p->k_bend;
  d.mu = p->mu;
  d.drag = p->drag;
  d.g[0] = p->g[0];
  d.g[1] = p->g[1];
  d.g[2] = p->g[2];
  d.dt = p->dt;
  return d;
}

// One step with tile configuration cfg (no validation: callers validate).
int ms_step_once(const pecnn_plan* plan, int cfg, const MsParamsDev& P, const float* in, float* out,
                 const uint8_t* active, hipStream_t st) {
  const int slot = ms_cfg_slot(cfg);
  switch (cfg) {
    case 0: launch_ms<32, 8, 1>(plan, slot, P, in, out, active, st); break;
    case 1: launch_ms<64, 4, 1>(plan, slot, P, in, out, active, st); break;
    case 2: launch_ms<16, 16, 1>(plan, slot, P, in, out, active, st); break;
    case 3: launch_ms<32, 16, 2>(plan, slot, P, in, out, active, st); break;
    case 4: launch_ms<64, 8, 2>(plan, slot, P, in, out, active, st); break;
    default: return PECNN_E_INVALID;
  }
  PECNN_LAUNCH_CHECK("ms_step_kernel");
  return PECNN_OK;
}

// n_steps with ping-pong through ws; the last step lands in out.
int ms_step_run(const pecnn_plan* plan, int cfg, const MsParamsDev& P, const float* in, float* out,
                float* tmp, int n_steps, const uint8_t* active, hipStream_t st) {
  const float* src = in;
  for (int k = 0; k < n_steps; ++k) {
    float* dst = ((n_steps - 1 - k) % 2 == 0) ? out : tmp;
    int rc = ms_step_once(plan, cfg, P, src, dst, active, st);
    if (rc != PECNN_OK) return rc;
    src = dst;
  }
  return PECNN_OK;
}

}  // namespace pecnn
