// Reverse mode of the CNN frame (section 3.2.1: the parameters w, b are optimised by gradient
// backpropagation through eqs. 5-7), FP32, deterministic. Three steps in two launches:
//
//  1. bwd_tile (cnn_bwd_tile.hip): on the matrix cores, per tile of 64 x 4 nodes: recomputes the
//     cell, pulls the adjoint of eq. (5) back through the heads, the ISRU branches and the two
//     Ch x Ch maps, writes the adjoints of the im2col entries (and gdv) to a compact table, and
//     accumulates the parameter gradients in registers (one partial row per workgroup).
//  2. bwd_gather: one thread per node: the adjoint of the clamped im2col, written as a gather
//     over the (neighbour, tap) pairs that read this node, plus the direct terms of eq. (5).
//     Accumulates into g_cur and g_prev.
//  3. wgrad_final: a fixed-order sum of the partial rows into g_theta, in the same launch as 2.
// The pair cell (section 3.2 read literally) and the sphere's reverse mode follow below.
#include "cnn_bwd_table.hpp"
#include "cnn_common.hpp"

namespace pecnn {

__host__ __device__ inline int64_t theta_count(int ch) { return (int64_t)ch * 54 + 2 * ch * ch + 9 * ch + 3; }

__device__ __forceinline__ int clampi(int v, int lo, int hi) { return v < lo ? lo : (v > hi ? hi : v); }

// Node kernels walk the batch in chunks of kChunk nodes; chunk t belongs to instance
// chunk_inst[t] and starts at its node (t - prefix[b]) kChunk.
// Node indices inside an instance fit 32 bits (the batch size limit), so the row / column split
// is a 32-bit division.
__device__ __forceinline__ bool chunk_node(const InstDev* inst, const int32_t* prefix, const int32_t* chunk_inst,
                                           int t, int& b, int& local) {
  b = chunk_inst[t];
  local = (t - prefix[b]) * kChunk + (int)threadIdx.x;
  return local < inst[b].H * inst[b].W;
}

// For node q: g_cur/g_prev += direct terms of eq. (5) + adjoint of the clamped, centre-differenced
// im2col: a tap (c, o) of node p read S_c(clamp(p + o)) (and, for positions, -S_c(p)); plus, with a
// pressure, the adjoint of the eq. (3) term of q and of its four neighbours, which read x_q.
__device__ __forceinline__ void bwd_gather_chunk(
    int t, const InstDev* __restrict__ inst, const int32_t* __restrict__ prefix, const int32_t* __restrict__ chunk_inst,
    const uint8_t* __restrict__ pin, const float* __restrict__ s_cur, const float* __restrict__ g_next, int64_t N,
    float dt, const float* __restrict__ tab, float* __restrict__ g_cur, float* __restrict__ g_prev) {
  int b;
  int local;
  if (!chunk_node(inst, prefix, chunk_inst, t, b, local)) return;
  const InstDev I = inst[b];
  const int qi = local / I.W, qj = local - (local / I.W) * I.W;
  const int64_t q = I.off + local;
  const float* __restrict__ gus = tab + kBtGus * 32;
  const float* __restrict__ gud = tab + kBtGud * 32;
  const bool pinned = pin[q] != 0;
  float accC[6], accP[6];
#pragma unroll
  for (int c = 0; c < 6; ++c) { accC[c] = 0.f; accP[c] = 0.f; }
  // taps of neighbours p whose clamped offset lands on q
#pragma unroll
  for (int dy = -1; dy <= 1; ++dy)
#pragma unroll
    for (int dx = -1; dx <= 1; ++dx) {
      const int o = (dy + 1) * 3 + (dx + 1);
      for (int pi = qi - dy - 1; pi <= qi - dy + 1; ++pi) {
        if (pi < 0 || pi >= I.H || clampi(pi + dy, 0, I.H - 1) != qi) continue;
        for (int pj = qj - dx - 1; pj <= qj - dx + 1; ++pj) {
          if (pj < 0 || pj >= I.W || clampi(pj + dx, 0, I.W - 1) != qj) continue;
          const int64_t pp = I.off + (int64_t)pi * I.W + pj;
#pragma unroll
          for (int c = 0; c < 6; ++c) {
            accC[c] += gus[bt_node(pp) + (c * 9 + o) * 32];
            accP[c] -= gud[bt_node(pp) + (c * 9 + o) * 32];
          }
        }
      }
    }
  // centre term of the position taps of q itself
#pragma unroll
  for (int c = 0; c < 3; ++c)
#pragma unroll
    for (int o = 0; o < 9; ++o) {
      accC[c] -= gus[bt_node(q) + (c * 9 + o) * 32];
      accP[c] += gud[bt_node(q) + (c * 9 + o) * 32];
    }
  if (I.pres != 0.f) {  // eq. (3): the pressure terms that read x_q (dLoss/dv' of P from the table)
    float acc[3] = {0.f, 0.f, 0.f};
    auto gdv = [&](int64_t P, float (&l)[3]) {
      for (int k = 0; k < 3; ++k) l[k] = tab[bt_node(P) + (kBtGdv + k) * 32];
    };
    pressure_adjoint_gather(I.H, I.W, I.off, qi, qj, dt * I.pres / I.mass, s_cur, N, gdv, acc);
    for (int k = 0; k < 3; ++k) accC[k] += acc[k];
  }
  // eq. (5): x' = x + dt v', v' = C(v + dv + dt a)
#pragma unroll
  for (int k = 0; k < 3; ++k) {
    accC[k] += g_next[k * N + q];
    if (!pinned) accC[3 + k] += g_next[(3 + k) * N + q] + dt * g_next[k * N + q];
  }
  if (g_cur)
#pragma unroll
    for (int c = 0; c < 6; ++c) g_cur[c * N + q] += accC[c];
  if (g_prev)
#pragma unroll
    for (int c = 0; c < 6; ++c) g_prev[c * N + q] += accP[c];
}

// g_theta[e] += sum over the partial rows, one block of 256 threads for kWfParams parameters: each
// of kWfGroups threads per parameter sums a fixed stride of rows, then a fixed-order combine in LDS
// (deterministic). The loads of eight rows are issued before their adds.
constexpr int kWfParams = 32, kWfGroups = 8;
static_assert(kWfParams * kWfGroups == 256, "one 256-thread block per parameter group");
__device__ __forceinline__ void wgrad_final_block(int blk, const float* __restrict__ partial, int n_rows, int P,
                                                  float* __restrict__ g_theta) {
  __shared__ double sh[kWfGroups][kWfParams + 1];
  const int pl = threadIdx.x % kWfParams, r0 = threadIdx.x / kWfParams;
  const int e = blk * kWfParams + pl;
  double s = 0.0;
  if (e < P) {
#pragma unroll 8
    for (int r = r0; r < n_rows; r += kWfGroups) s += (double)partial[(int64_t)r * P + e];
  }
  sh[r0][pl] = s;
  __syncthreads();
  if (r0 == 0 && e < P) {
    double u = 0.0;
#pragma unroll
    for (int k = 0; k < kWfGroups; ++k) u += sh[k][pl];
    g_theta[e] += (float)u;
  }
}

__host__ __device__ inline int wgrad_final_blocks(int P) { return (P + kWfParams - 1) / kWfParams; }

__global__ __launch_bounds__(256) void wgrad_final_kernel(const float* __restrict__ partial, int n_rows, int P,
                                                          float* __restrict__ g_theta) {
  wgrad_final_block(blockIdx.x, partial, n_rows, P, g_theta);
}

// The gather and the parameter sum read disjoint outputs of bwd_tile and write disjoint arrays, so
// one launch runs both: the first nw blocks sum parameters (dispatched first, they overlap the
// gather), the rest gather one chunk each.
__global__ __launch_bounds__(256) void bwd_gather_final_kernel(
    int nw, const float* __restrict__ partial, int n_rows, int P, float* __restrict__ g_theta,
    const InstDev* __restrict__ inst, const int32_t* __restrict__ prefix, const int32_t* __restrict__ chunk_inst,
    const uint8_t* __restrict__ pin, const float* __restrict__ s_cur, const float* __restrict__ g_next, int64_t N,
    float dt, const float* __restrict__ tab, float* __restrict__ g_cur, float* __restrict__ g_prev) {
  if ((int)blockIdx.x < nw)
    wgrad_final_block(blockIdx.x, partial, n_rows, P, g_theta);
  else
    bwd_gather_chunk((int)blockIdx.x - nw, inst, prefix, chunk_inst, pin, s_cur, g_next, N, dt, tab, g_cur, g_prev);
}

// ---------------------------------------------------------------- the pair cell
// Reverse mode of the pair-cell frame (section 3.2 read literally; the PAIR mode of the stencil
// kernel). For node P with l = dLoss/dv' (zero when P is pinned), a channel c whose neighbour j
// is on the grid, and an axis a, with d = x_j - x_P, e = v_j - v_P, phi = s_c d, xi = s_c e:
//   dLoss/dphi = l_a (wL_c + (wN_c + wD_c xi) sigma'(phi)),  dLoss/dxi = l_a wD_c sigma(phi);
//   x_j gets + s_c dLoss/dphi and x_P gets - s_c dLoss/dphi (v likewise with dLoss/dxi);
//   wL_c += l_a phi, wN_c += l_a sigma(phi), wD_c += l_a xi sigma(phi),
//   s_c += dLoss/dphi d + dLoss/dxi e, b_L += l.
// Two kernels: state gradients as a gather (each node collects the terms that read it), and
// per-chunk parameter sums in fixed order, finished by wgrad_final_kernel. S^{k-1} is not read.
constexpr int kPairP = 51;
__device__ constexpr int kPairNb[12][2] = {{0, 1}, {0, -1}, {1, 0}, {-1, 0}, {1, 1}, {1, -1},
                                           {-1, 1}, {-1, -1}, {0, 2}, {0, -2}, {2, 0}, {-2, 0}};

__device__ __forceinline__ void pair_terms(const float* __restrict__ th, int c, float alpha, float d, float e, float l,
                                           float& gphi, float& gxi, float& phi, float& xi, float& sg) {
  const float sq = th[c], wl = th[12 + c], wn = th[24 + c], wd = th[36 + c];
  phi = sq * d;
  xi = sq * e;
  const float r = __builtin_amdgcn_rsqf(__builtin_fmaf(alpha * phi, phi, 1.f));
  sg = phi * r;
  gphi = l * __builtin_fmaf(__builtin_fmaf(wd, xi, wn), r * r * r, wl);
  gxi = l * (wd * sg);
}

__device__ __forceinline__ void pair_gdv(const uint8_t* __restrict__ pin, const float* __restrict__ g_next, int64_t N,
                                         float dt, int64_t P, float (&l)[3]) {
  const bool pinned = pin[P] != 0;
#pragma unroll
  for (int k = 0; k < 3; ++k) l[k] = pinned ? 0.f : g_next[(3 + k) * N + P] + dt * g_next[k * N + P];
}

__global__ __launch_bounds__(256) void pair_gather_kernel(
    const InstDev* __restrict__ inst, const int32_t* __restrict__ prefix, const int32_t* __restrict__ chunk_inst,
    const uint8_t* __restrict__ pin, const float* __restrict__ s_cur, const float* __restrict__ g_next, int64_t N,
    const float* __restrict__ theta, float alpha, float dt, float* __restrict__ g_cur) {
  int b, local;
  if (!chunk_node(inst, prefix, chunk_inst, blockIdx.x, b, local)) return;
  const InstDev I = inst[b];
  const int qi = local / I.W, qj = local - (local / I.W) * I.W;
  const int64_t q = I.off + local;
  float acc[6];
  float lq[3];
  pair_gdv(pin, g_next, N, dt, q, lq);
#pragma unroll
  for (int k = 0; k < 3; ++k) {  // eq. (5): x' = x + dt v', v' = C(v + dv + dt a)
    acc[k] = g_next[k * N + q];
    acc[3 + k] = lq[k];
  }
  float gphi, gxi, phi, xi, sg;
  for (int c = 0; c < 12; ++c) {
    // q as the centre of its channel c
    const int ii = qi + kPairNb[c][0], jj = qj + kPairNb[c][1];
    if (ii >= 0 && ii < I.H && jj >= 0 && jj < I.W) {
      const int64_t j = I.off + (int64_t)ii * I.W + jj;
#pragma unroll
      for (int a = 0; a < 3; ++a) {
        pair_terms(theta, c, alpha, s_cur[a * N + j] - s_cur[a * N + q], s_cur[(3 + a) * N + j] - s_cur[(3 + a) * N + q],
                   lq[a], gphi, gxi, phi, xi, sg);
        acc[a] -= theta[c] * gphi;
        acc[3 + a] -= theta[c] * gxi;
      }
    }
    // q as the channel-c neighbour of node P = q - o_c
    const int pi = qi - kPairNb[c][0], pj = qj - kPairNb[c][1];
    if (pi >= 0 && pi < I.H && pj >= 0 && pj < I.W) {
      const int64_t P = I.off + (int64_t)pi * I.W + pj;
      float lp[3];
      pair_gdv(pin, g_next, N, dt, P, lp);
#pragma unroll
      for (int a = 0; a < 3; ++a) {
        pair_terms(theta, c, alpha, s_cur[a * N + q] - s_cur[a * N + P], s_cur[(3 + a) * N + q] - s_cur[(3 + a) * N + P],
                   lp[a], gphi, gxi, phi, xi, sg);
        acc[a] += theta[c] * gphi;
        acc[3 + a] += theta[c] * gxi;
      }
    }
  }
  if (I.pres != 0.f) {  // eq. (3): the pressure terms that read x_q
    float ap[3] = {0.f, 0.f, 0.f};
    auto gdv = [&](int64_t P, float (&l)[3]) { pair_gdv(pin, g_next, N, dt, P, l); };
    pressure_adjoint_gather(I.H, I.W, I.off, qi, qj, dt * I.pres / I.mass, s_cur, N, gdv, ap);
    for (int k = 0; k < 3; ++k) acc[k] += ap[k];
  }
#pragma unroll
  for (int c = 0; c < 6; ++c) g_cur[c * N + q] += acc[c];
}

__global__ __launch_bounds__(256) void pair_wgrad_kernel(
    const InstDev* __restrict__ inst, const int32_t* __restrict__ prefix, const int32_t* __restrict__ chunk_inst,
    const uint8_t* __restrict__ pin, const float* __restrict__ s_cur, const float* __restrict__ g_next, int64_t N,
    const float* __restrict__ theta, float alpha, float dt, float* __restrict__ partial) {
  __shared__ float sh[kPairP][4];
  float g[kPairP];
#pragma unroll
  for (int k = 0; k < kPairP; ++k) g[k] = 0.f;
  int b, local;
  if (chunk_node(inst, prefix, chunk_inst, blockIdx.x, b, local)) {  // every thread joins the sums below
    const InstDev I = inst[b];
    const int qi = local / I.W, qj = local - (local / I.W) * I.W;
    const int64_t q = I.off + local;
    float l[3];
    pair_gdv(pin, g_next, N, dt, q, l);
    g[48] = l[0];
    g[49] = l[1];
    g[50] = l[2];
#pragma unroll
    for (int c = 0; c < 12; ++c) {
      const int ii = qi + kPairNb[c][0], jj = qj + kPairNb[c][1];
      if (ii < 0 || ii >= I.H || jj < 0 || jj >= I.W) continue;
      const int64_t j = I.off + (int64_t)ii * I.W + jj;
#pragma unroll
      for (int a = 0; a < 3; ++a) {
        const float d = s_cur[a * N + j] - s_cur[a * N + q], e = s_cur[(3 + a) * N + j] - s_cur[(3 + a) * N + q];
        float gphi, gxi, phi, xi, sg;
        pair_terms(theta, c, alpha, d, e, l[a], gphi, gxi, phi, xi, sg);
        g[c] = __builtin_fmaf(gxi, e, __builtin_fmaf(gphi, d, g[c]));
        g[12 + c] = __builtin_fmaf(l[a], phi, g[12 + c]);
        g[24 + c] = __builtin_fmaf(l[a], sg, g[24 + c]);
        g[36 + c] = __builtin_fmaf(l[a], xi * sg, g[36 + c]);
      }
    }
  }
  // fixed-order block sums: butterfly within each wave, then the four wave sums
  const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
#pragma unroll
  for (int k = 0; k < kPairP; ++k) {
    float v = g[k];
#pragma unroll
    for (int o = 32; o > 0; o >>= 1) v += __shfl_xor(v, o);
    if (lane == 0) sh[k][wave] = v;
  }
  __syncthreads();
  if (threadIdx.x < kPairP) {
    const int k = threadIdx.x;
    partial[(int64_t)blockIdx.x * kPairP + k] = ((sh[k][0] + sh[k][1]) + sh[k][2]) + sh[k][3];
  }
}

size_t pair_backward_ws_bytes(const pecnn_plan* plan) {
  return (size_t)plan->n_tiles[kCfgChunk] * kPairP * sizeof(float);
}

int pair_backward_launch(const pecnn_plan* plan, const pecnn_model* m, const float* sc, const float* gn, float* gc,
                         float* gth, void* ws, hipStream_t st) {
  const int nt = plan->n_tiles[kCfgChunk];
  const int32_t* pre = plan->d_prefix[kCfgChunk];
  float* partial = (float*)ws;
  if (gc) {
    hipLaunchKernelGGL(pair_gather_kernel, dim3(nt), dim3(256), 0, st, plan->d_inst, pre, plan->d_chunk_inst, plan->pin,
                       sc, gn, plan->total, m->theta, m->isru_alpha, m->dt, gc);
    PECNN_LAUNCH_CHECK("pair_gather_kernel");
  }
  hipLaunchKernelGGL(pair_wgrad_kernel, dim3(nt), dim3(256), 0, st, plan->d_inst, pre, plan->d_chunk_inst, plan->pin, sc,
                     gn, plan->total, m->theta, m->isru_alpha, m->dt, partial);
  PECNN_LAUNCH_CHECK("pair_wgrad_kernel");
  hipLaunchKernelGGL(wgrad_final_kernel, dim3(wgrad_final_blocks(kPairP)), dim3(256), 0, st, partial, nt, kPairP, gth);
  PECNN_LAUNCH_CHECK("wgrad_final_kernel");
  return PECNN_OK;
}

// ---------------------------------------------------------------- the sphere's reverse mode
// Reverse mode of sphere_update for a free node, as a change of the frame's output adjoint.
// Without the constraint, y = x + dt v and v' = v send (gy, gw) to gx = gy, gv = gw + dt gy.
// Inside the sphere, with u = y - c, r = |u|, n = u / r, s = v . n, k = max(s, 0) - (1 - fric) s,
// the step is y = c + R n, v' = (1 - fric) v + k n, whose chain rule gives
//   g_s = (gw . n)([s > 0] - (1 - fric)),  g_n = R gy + k gw + g_s v,  g_u = (I - n n^T) g_n / r,
//   gx = g_u,  gv = (1 - fric) gw + g_s n + dt g_u.
// Replacing (gy, gw) by (g_u, (1 - fric) gw + g_s n) makes the constraint-free reverse pass give
// exactly these. The inside test repeats the forward's FP32 arithmetic, so both take the same
// branch. v is the velocity before the constraint; g holds (gy, gw) and is updated in place.
__device__ __forceinline__ void sphere_adjoint(const float* __restrict__ sph, float dt, float x0, float x1, float x2,
                                               float v0, float v1, float v2, float g[6]) {
  const float R = sph[3];
  if (!(R > 0.f)) return;
  const float d0 = __builtin_fmaf(dt, v0, x0) - sph[0], d1 = __builtin_fmaf(dt, v1, x1) - sph[1],
              d2 = __builtin_fmaf(dt, v2, x2) - sph[2];
  const float r2 = __builtin_fmaf(d2, d2, __builtin_fmaf(d1, d1, d0 * d0));
  if (!(r2 < R * R)) return;
  float n0 = 0.f, n1 = 0.f, n2 = 1.f, ir = 0.f;  // at r = 0 the normal is constant: g_u = 0
  if (r2 > 0.f) {
    ir = 1.f / __builtin_sqrtf(r2);
    n0 = d0 * ir;
    n1 = d1 * ir;
    n2 = d2 * ir;
  }
  const float vn = __builtin_fmaf(v2, n2, __builtin_fmaf(v1, n1, v0 * n0));
  const float kf = 1.f - sph[4];
  const float k = (vn > 0.f ? vn : 0.f) - kf * vn;
  const float gs = (g[3] * n0 + g[4] * n1 + g[5] * n2) * ((vn > 0.f ? 1.f : 0.f) - kf);
  const float gn0 = R * g[0] + k * g[3] + gs * v0, gn1 = R * g[1] + k * g[4] + gs * v1,
              gn2 = R * g[2] + k * g[5] + gs * v2;
  const float ngn = n0 * gn0 + n1 * gn1 + n2 * gn2;
  g[0] = (gn0 - ngn * n0) * ir;
  g[1] = (gn1 - ngn * n1) * ir;
  g[2] = (gn2 - ngn * n2) * ir;
  g[3] = kf * g[3] + gs * n0;
  g[4] = kf * g[4] + gs * n1;
  g[5] = kf * g[5] + gs * n2;
}

// One thread per node over the 256-node chunks: rewrites the frame's output adjoint so that the
// constraint-free reverse pass that follows goes through each instance's sphere (sphere_adjoint).
// vfree holds the frame computed without spheres: its velocity rows are the velocities before the
// constraint.
__global__ __launch_bounds__(256) void sphere_adjoint_kernel(
    const InstDev* __restrict__ inst, const int32_t* __restrict__ prefix, const int32_t* __restrict__ chunk_inst,
    int64_t N, const uint8_t* __restrict__ pin, const float* __restrict__ sc, const float* __restrict__ vfree,
    const float* __restrict__ gn, const float* __restrict__ sphere, float dt, float* __restrict__ gt) {
  const int t = blockIdx.x;
  const int b = chunk_inst[t];
  const InstDev I = inst[b];
  const int local = (t - prefix[b]) * kChunk + (int)threadIdx.x;
  if (local >= I.H * I.W) return;
  const int64_t p = I.off + local;
  float g[6];
#pragma unroll
  for (int c = 0; c < 6; ++c) g[c] = gn[c * N + p];
  if (pin[p] == 0)
    sphere_adjoint(sphere + (int64_t)b * kSphereStride, dt, sc[p], sc[N + p], sc[2 * N + p], vfree[3 * N + p],
                   vfree[4 * N + p], vfree[5 * N + p], g);
#pragma unroll
  for (int c = 0; c < 6; ++c) gt[c * N + p] = g[c];
}

__global__ __launch_bounds__(256) void zero_floats_kernel(float* __restrict__ p, int64_t n) {
  const int64_t i = (int64_t)blockIdx.x * 256 + threadIdx.x;
  if (i < n) p[i] = 0.f;
}

int sphere_adjoint_launch(const pecnn_plan* plan, float dt, const float* sc, const float* vfree, const float* gn,
                          float* gt, hipStream_t st) {
  hipLaunchKernelGGL(sphere_adjoint_kernel, dim3(plan->n_tiles[kCfgChunk]), dim3(256), 0, st, plan->d_inst,
                     plan->d_prefix[kCfgChunk], plan->d_chunk_inst, plan->total, plan->pin, sc, vfree, gn,
                     plan->d_sphere, dt, gt);
  PECNN_LAUNCH_CHECK("sphere_adjoint_kernel");
  return PECNN_OK;
}

int zero_floats_launch(float* p, int64_t n, hipStream_t st) {
  hipLaunchKernelGGL(zero_floats_kernel, dim3((unsigned)((n + 255) / 256)), dim3(256), 0, st, p, n);
  PECNN_LAUNCH_CHECK("zero_floats_kernel");
  return PECNN_OK;
}

size_t bwd_tile_ws_bytes(const pecnn_plan*, int ch);
int bwd_tile_grid(const pecnn_plan*);
int bwd_tile_launch(const pecnn_plan*, const pecnn_model*, const float*, const float*, const float*, float*, float*,
                    hipStream_t);

size_t backward_ws_bytes(const pecnn_plan* plan, int ch) { return bwd_tile_ws_bytes(plan, ch); }

int backward_launch(const pecnn_plan* plan, const pecnn_model* m, const float* sp, const float* sc,
                    const float* gn, float* gc, float* gp, float* gth, void* ws, hipStream_t st) {
  float* tab = (float*)ws;
  const size_t tab_bytes = (size_t)bt_floats(plan->total) * sizeof(float);
  float* partial = (float*)((char*)ws + ((tab_bytes + 255) / 256) * 256);
  const int nt = plan->n_tiles[kCfgChunk];
  const int32_t* pre = plan->d_prefix[kCfgChunk];
  const int P = (int)theta_count(m->ch);
  int rc = bwd_tile_launch(plan, m, sp, sc, gn, tab, partial, st);
  if (rc) return rc;
  const int nrows = bwd_tile_grid(plan), nw = wgrad_final_blocks(P);
  if (gc || gp) {
    hipLaunchKernelGGL(bwd_gather_final_kernel, dim3(nw + nt), dim3(256), 0, st, nw, partial, nrows, P, gth, plan->d_inst,
                       pre, plan->d_chunk_inst, plan->pin, sc, gn, plan->total, m->dt, tab, gc, gp);
    PECNN_LAUNCH_CHECK("bwd_gather_final_kernel");
  } else {
    hipLaunchKernelGGL(wgrad_final_kernel, dim3(nw), dim3(256), 0, st, partial, nrows, P, gth);
    PECNN_LAUNCH_CHECK("wgrad_final_kernel");
  }
  return PECNN_OK;
}

}  // namespace pecnn
