// Mass-spring cloth step (section 3.1, eqs. 1, 2, 4, 5) on gfx950.
//
// One workgroup owns a TX x TY tile of one instance; the six state planes of the tile plus a
// two-node halo (the stencil radius of the bending springs) are staged in LDS with coalesced
// row loads, then each thread integrates RY nodes. Workgroups are persistent over the batch's
// tile list, with a contiguous tile range per XCD so that halo rows shared by neighbouring
// tiles are served by one L2.
#include "common.hpp"

namespace pecnn {

// The 12 springs of a node: (row offset, column offset, family).
// Family 0 structural (rest h), 1 shear (rest sqrt(2) h), 2 bend (rest 2h).
struct Spring { int dy, dx, fam; };
__device__ constexpr Spring kSprings[12] = {
    {0, 1, 0}, {0, -1, 0}, {1, 0, 0}, {-1, 0, 0},
    {1, 1, 1}, {1, -1, 1}, {-1, 1, 1}, {-1, -1, 1},
    {0, 2, 2}, {0, -2, 2}, {2, 0, 2}, {-2, 0, 2}};

template <int TX, int TY, int RY>
__global__ __launch_bounds__(TX*(TY / RY)) void ms_step_kernel(
    const InstDev* __restrict__ inst, const int32_t* __restrict__ prefix, int n_inst, int n_tiles,
    const uint8_t* __restrict__ pin, const float* __restrict__ s_in, float* __restrict__ s_out,
    int64_t N, MsParamsDev P, const uint8_t* __restrict__ active) {
  constexpr int HX = TX + 4, HY = TY + 4;
  constexpr int NT = TX * (TY / RY);
  __shared__ float lds[6][HY][HX];

  int first, stride, count;
  xcd_tile_range(n_tiles, first, stride, count);
  const int tx = threadIdx.x % TX;
  const int ty0 = (threadIdx.x / TX) * RY;

  for (int it = 0; it < count; ++it) {
    const int t = first + it * stride;
    const int b = find_instance(prefix, n_inst, t);
    if (active != nullptr && active[b] == 0) continue;  // uniform over the workgroup
    const InstDev I = inst[b];
    const int lt = t - prefix[b];
    const int tiles_x = (I.W + TX - 1) / TX;
    const int r0 = (lt / tiles_x) * TY;
    const int c0 = (lt % tiles_x) * TX;
    const float* __restrict__ src = s_in + I.off;

    for (int e = threadIdx.x; e < 6 * HY * HX; e += NT) {
      const int c = e / (HY * HX);
      const int rem = e - c * (HY * HX);
      const int rr = rem / HX;
      const int cc = rem - rr * HX;
      const int gi = r0 + rr - 2, gj = c0 + cc - 2;
      float v = 0.f;
      if (gi >= 0 && gi < I.H && gj >= 0 && gj < I.W) v = src[c * N + (int64_t)gi * I.W + gj];
      lds[c][rr][cc] = v;
    }
    __syncthreads();

    const float L[3] = {I.h, I.h * 1.41421356237309515f, 2.f * I.h};
    const float tiny = 1e-24f * I.h * I.h;
    const float inv_m = 1.f / I.mass;
#pragma unroll
    for (int ry = 0; ry < RY; ++ry) {
      const int ly = ty0 + ry;
      const int i = r0 + ly, j = c0 + tx;
      if (i < I.H && j < I.W) {
        const int64_t p = I.off + (int64_t)i * I.W + j;
        const int hy = ly + 2, hx = tx + 2;
        const float x0 = lds[0][hy][hx], x1 = lds[1][hy][hx], x2 = lds[2][hy][hx];
        const float v0 = lds[3][hy][hx], v1 = lds[4][hy][hx], v2 = lds[5][hy][hx];
        float n0, n1, n2;
        if (pin[p]) {
          n0 = n1 = n2 = 0.f;
        } else {
          // eq. (4) plus the wind: m (g + a_ext) - d v
          float f0 = I.mass * (P.g[0] + I.ax) - P.drag * v0;
          float f1 = I.mass * (P.g[1] + I.ay) - P.drag * v1;
          float f2 = I.mass * (P.g[2] + I.az) - P.drag * v2;
#pragma unroll
          for (int q = 0; q < 12; ++q) {
            const Spring S = kSprings[q];
            const int ii = i + S.dy, jj = j + S.dx;
            if (ii < 0 || ii >= I.H || jj < 0 || jj >= I.W) continue;
            const int ny = hy + S.dy, nx = hx + S.dx;
            const float d0 = x0 - lds[0][ny][nx], d1 = x1 - lds[1][ny][nx], d2 = x2 - lds[2][ny][nx];
            const float w0 = v0 - lds[3][ny][nx], w1 = v1 - lds[4][ny][nx], w2 = v2 - lds[5][ny][nx];
            const float r2 = d0 * d0 + d1 * d1 + d2 * d2;
            if (!(r2 > tiny)) continue;
            const float ir = __builtin_amdgcn_rsqf(r2);
            const float r = r2 * ir;
            const float ce = -P.k[S.fam] * (r - L[S.fam]) * ir;            // eq. (1)
            const float cd = -P.mu * (w0 * d0 + w1 * d1 + w2 * d2) * ir * ir;  // eq. (2)
            const float cf = ce + cd;
            f0 += cf * d0;
            f1 += cf * d1;
            f2 += cf * d2;
          }
          // eq. (5): semi-implicit Euler
          const float s = P.dt * inv_m;
          n0 = v0 + s * f0;
          n1 = v1 + s * f1;
          n2 = v2 + s * f2;
        }
        s_out[3 * N + p] = n0;
        s_out[4 * N + p] = n1;
        s_out[5 * N + p] = n2;
        s_out[0 * N + p] = x0 + P.dt * n0;
        s_out[1 * N + p] = x1 + P.dt * n1;
        s_out[2 * N + p] = x2 + P.dt * n2;
      }
    }
    __syncthreads();
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
  hipLaunchKernelGGL((ms_step_kernel<TX, TY, RY>), dim3(grid), dim3(TX * (TY / RY)), 0, st,
                     plan->d_inst, plan->d_prefix[slot], plan->n, n_tiles, plan->pin, in, out,
                     plan->total, P, active);
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
