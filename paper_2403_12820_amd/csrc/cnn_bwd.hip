// Reverse mode of the CNN frame (section 3.2.1: the parameters w, b are optimised by gradient
// backpropagation through eqs. 5-7). FP32 throughout. Three kernels, all deterministic:
//
//  1. bwd_node:   one thread per node. Recomputes the cell from (S^{k-1}, S^k), pulls the
//                 adjoint of eq. (5) back through the heads, the ISRU branches and the two
//                 Ch x Ch maps, and writes per-node factors to the workspace: the adjoints of the
//                 im2col entries (for the input gradients) and the vectors whose outer products
//                 over nodes give the parameter gradients.
//  2. bwd_gather: one thread per node: the adjoint of the clamped im2col, written as a gather
//                 over the (neighbour, tap) pairs that read this node, plus the direct terms of
//                 eq. (5). Accumulates into g_cur and g_prev.
//  3. bwd_wgrad:  per chunk of 256 nodes, the parameter-gradient partial sums (outer products
//                 staged through LDS), then a fixed-order sum over chunks into g_theta.
#include "common.hpp"

namespace pecnn {

struct BwdLayout {
  // feature rows of the per-node factor table, each a plane of N floats
  int uk, ud, gus, gud, phi, nn, dd, ga, gb, gphi, gxi, gdv, rows;
};
__host__ __device__ inline BwdLayout bwd_layout(int ch) {
  BwdLayout L;
  L.uk = 0;
  L.ud = 54;
  L.gus = 108;
  L.gud = 162;
  L.phi = 216;
  L.nn = L.phi + ch;
  L.dd = L.nn + ch;
  L.ga = L.dd + ch;
  L.gb = L.ga + ch;
  L.gphi = L.gb + ch;
  L.gxi = L.gphi + ch;
  L.gdv = L.gxi + ch;
  L.rows = L.gdv + 3;
  return L;
}

__host__ __device__ inline int64_t theta_count(int ch) { return (int64_t)ch * 54 + 2 * ch * ch + 9 * ch + 3; }

__device__ __forceinline__ int clampi(int v, int lo, int hi) { return v < lo ? lo : (v > hi ? hi : v); }

// Node kernels walk the batch in chunks of kChunk nodes (tile prefix of the chunk config).
__device__ __forceinline__ bool chunk_node(const InstDev* inst, const int32_t* prefix, int n_inst, int t,
                                           int& b, int64_t& local) {
  b = find_instance(prefix, n_inst, t);
  local = (int64_t)(t - prefix[b]) * kChunk + threadIdx.x;
  const int64_t n = (int64_t)inst[b].H * inst[b].W;
  return local < n;
}

template <int CH>
__global__ __launch_bounds__(256) void bwd_node_kernel(
    const InstDev* __restrict__ inst, const int32_t* __restrict__ prefix, int n_inst,
    const uint8_t* __restrict__ pin, const float* __restrict__ s_prev, const float* __restrict__ s_cur,
    const float* __restrict__ g_next, int64_t N, const float* __restrict__ theta, float dt, float alpha,
    float* __restrict__ fac) {
  constexpr int P = CH * 54 + 2 * CH * CH + 9 * CH + 3;
  constexpr int oA = CH * 54, oB = oA + CH * CH, oWL = oB + CH * CH, oWN = oWL + 3 * CH, oWD = oWN + 3 * CH;
  constexpr int SW = 2 * CH + 1;  // per-thread scratch row (odd stride: no bank conflicts)
  __shared__ float th[P];
  __shared__ float scr[256 * SW];
  for (int e = threadIdx.x; e < P; e += 256) th[e] = theta[e];
  __syncthreads();

  int b;
  int64_t local;
  if (!chunk_node(inst, prefix, n_inst, blockIdx.x, b, local)) return;
  const InstDev I = inst[b];
  const int i = (int)(local / I.W), j = (int)(local % I.W);
  const int64_t p = I.off + local;
  const BwdLayout L = bwd_layout(CH);
  float* __restrict__ F = fac + p;  // feature row r lives at F[r * N]
  float* __restrict__ my = scr + threadIdx.x * SW;

  // forward recompute: phi = K U(S^k), xi = K U(S^k - S^{k-1}); im2col entries go to the table
  float phi[CH], xi[CH];
#pragma unroll
  for (int c = 0; c < CH; ++c) { phi[c] = 0.f; xi[c] = 0.f; }
#pragma unroll 1
  for (int c = 0; c < 6; ++c) {
    float ck = 0.f, cd = 0.f;
    if (c < 3) {
      ck = s_cur[c * N + p];
      cd = ck - s_prev[c * N + p];
    }
#pragma unroll 1
    for (int o = 0; o < 9; ++o) {
      const int qi = clampi(i + o / 3 - 1, 0, I.H - 1), qj = clampi(j + o % 3 - 1, 0, I.W - 1);
      const int64_t q = c * N + I.off + (int64_t)qi * I.W + qj;
      const float uk = s_cur[q] - ck;
      const float ud = (s_cur[q] - s_prev[q]) - cd;
      const int t = c * 9 + o;
      F[(L.uk + t) * N] = uk;
      F[(L.ud + t) * N] = ud;
#pragma unroll
      for (int r = 0; r < CH; ++r) {
        phi[r] = __builtin_fmaf(th[r * 54 + t], uk, phi[r]);
        xi[r] = __builtin_fmaf(th[r * 54 + t], ud, xi[r]);
      }
    }
  }
  // the two Ch x Ch maps of the nonlinear branch
#pragma unroll
  for (int c = 0; c < CH; ++c) my[c] = phi[c];
  float a[CH], bb[CH];
#pragma unroll
  for (int r = 0; r < CH; ++r) { a[r] = 0.f; bb[r] = 0.f; }
#pragma unroll 1
  for (int c = 0; c < CH; ++c) {
    const float pc = my[c];
#pragma unroll
    for (int r = 0; r < CH; ++r) {
      a[r] = __builtin_fmaf(th[oA + r * CH + c], pc, a[r]);
      bb[r] = __builtin_fmaf(th[oB + r * CH + c], pc, bb[r]);
    }
  }
  // adjoint of eq. (5)
  float gdv[3];
  const bool pinned = pin[p] != 0;
#pragma unroll
  for (int k = 0; k < 3; ++k) {
    const float gvt = g_next[(3 + k) * N + p] + dt * g_next[k * N + p];
    gdv[k] = pinned ? 0.f : gvt;
    F[(L.gdv + k) * N] = gdv[k];
  }
  // heads and ISRU branches; afterwards phi holds the head/derivative part of dLoss/dphi,
  // xi holds dLoss/dxi, and my[] holds the adjoints of (A phi) and (B phi)
#pragma unroll
  for (int c = 0; c < CH; ++c) {
    const float r1 = __builtin_amdgcn_rsqf(1.f + alpha * phi[c] * phi[c]);
    const float gs = phi[c] * r1, dgs = r1 * r1 * r1;
    const float z = a[c] * bb[c];
    const float r2 = __builtin_amdgcn_rsqf(1.f + alpha * z * z);
    const float nn = z * r2, dnn = r2 * r2 * r2;
    const float dd = xi[c] * gs;
    const float gphi_h = th[oWL + c] * gdv[0] + th[oWL + CH + c] * gdv[1] + th[oWL + 2 * CH + c] * gdv[2];
    const float gnn = th[oWN + c] * gdv[0] + th[oWN + CH + c] * gdv[1] + th[oWN + 2 * CH + c] * gdv[2];
    const float gdd = th[oWD + c] * gdv[0] + th[oWD + CH + c] * gdv[1] + th[oWD + 2 * CH + c] * gdv[2];
    const float gz = gnn * dnn;
    const float ga = gz * bb[c], gb = gz * a[c];
    F[(L.phi + c) * N] = phi[c];
    F[(L.nn + c) * N] = nn;
    F[(L.dd + c) * N] = dd;
    F[(L.ga + c) * N] = ga;
    F[(L.gb + c) * N] = gb;
    my[c] = ga;
    my[CH + c] = gb;
    phi[c] = gphi_h + gdd * xi[c] * dgs;
    xi[c] = gdd * gs;
    F[(L.gxi + c) * N] = xi[c];
  }
#pragma unroll 1
  for (int r = 0; r < CH; ++r) {
    const float gar = my[r], gbr = my[CH + r];
#pragma unroll
    for (int c = 0; c < CH; ++c) phi[c] = __builtin_fmaf(th[oB + r * CH + c], gbr, __builtin_fmaf(th[oA + r * CH + c], gar, phi[c]));
  }
#pragma unroll
  for (int c = 0; c < CH; ++c) F[(L.gphi + c) * N] = phi[c];
  // adjoint of the im2col entries
#pragma unroll 1
  for (int t = 0; t < 54; ++t) {
    float gk = 0.f, gd = 0.f;
#pragma unroll
    for (int c = 0; c < CH; ++c) {
      gk = __builtin_fmaf(th[c * 54 + t], phi[c], gk);
      gd = __builtin_fmaf(th[c * 54 + t], xi[c], gd);
    }
    F[(L.gus + t) * N] = gk + gd;
    F[(L.gud + t) * N] = gd;
  }
}

// For node q: g_cur/g_prev += direct terms of eq. (5) + adjoint of the clamped, centre-differenced
// im2col: a tap (c, o) of node p read S_c(clamp(p + o)) (and, for positions, -S_c(p)).
__global__ __launch_bounds__(256) void bwd_gather_kernel(
    const InstDev* __restrict__ inst, const int32_t* __restrict__ prefix, int n_inst,
    const uint8_t* __restrict__ pin, const float* __restrict__ g_next, int64_t N, float dt, int ch,
    const float* __restrict__ fac, float* __restrict__ g_cur, float* __restrict__ g_prev) {
  int b;
  int64_t local;
  if (!chunk_node(inst, prefix, n_inst, blockIdx.x, b, local)) return;
  const InstDev I = inst[b];
  const int qi = (int)(local / I.W), qj = (int)(local % I.W);
  const int64_t q = I.off + local;
  const BwdLayout L = bwd_layout(ch);
  const float* __restrict__ gus = fac + (int64_t)L.gus * N;
  const float* __restrict__ gud = fac + (int64_t)L.gud * N;
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
            accC[c] += gus[(int64_t)(c * 9 + o) * N + pp];
            accP[c] -= gud[(int64_t)(c * 9 + o) * N + pp];
          }
        }
      }
    }
  // centre term of the position taps of q itself
#pragma unroll
  for (int c = 0; c < 3; ++c)
#pragma unroll
    for (int o = 0; o < 9; ++o) {
      accC[c] -= gus[(int64_t)(c * 9 + o) * N + q];
      accP[c] += gud[(int64_t)(c * 9 + o) * N + q];
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

// Parameter gradient partials of one chunk: parameter e of the flat theta layout is a sum over
// nodes of a product of two factor rows (conv taps have two such products).
template <int CH>
__device__ __forceinline__ void param_rows(int e, int& x1, int& y1, int& x2, int& y2) {
  const BwdLayout L = bwd_layout(CH);
  constexpr int oA = CH * 54, oB = oA + CH * CH, oWL = oB + CH * CH, oWN = oWL + 3 * CH, oWD = oWN + 3 * CH,
                obL = oWD + 3 * CH;
  x2 = y2 = -1;
  if (e < oA) {  // K[c][t] : gphi_c * uk_t + gxi_c * ud_t
    const int c = e / 54, t = e % 54;
    x1 = L.gphi + c; y1 = L.uk + t; x2 = L.gxi + c; y2 = L.ud + t;
  } else if (e < oB) {  // A[r][c] : ga_r * phi_c
    const int r = (e - oA) / CH, c = (e - oA) % CH;
    x1 = L.ga + r; y1 = L.phi + c;
  } else if (e < oWL) {
    const int r = (e - oB) / CH, c = (e - oB) % CH;
    x1 = L.gb + r; y1 = L.phi + c;
  } else if (e < oWN) {
    const int r = (e - oWL) / CH, c = (e - oWL) % CH;
    x1 = L.gdv + r; y1 = L.phi + c;
  } else if (e < oWD) {
    const int r = (e - oWN) / CH, c = (e - oWN) % CH;
    x1 = L.gdv + r; y1 = L.nn + c;
  } else if (e < obL) {
    const int r = (e - oWD) / CH, c = (e - oWD) % CH;
    x1 = L.gdv + r; y1 = L.dd + c;
  } else {
    x1 = L.gdv + (e - obL); y1 = -1;  // bias: plain sum
  }
}

template <int CH>
__global__ __launch_bounds__(256) void bwd_wgrad_kernel(
    const InstDev* __restrict__ inst, const int32_t* __restrict__ prefix, int n_inst, int64_t N,
    const float* __restrict__ fac, float* __restrict__ partial) {
  constexpr int P = CH * 54 + 2 * CH * CH + 9 * CH + 3;
  constexpr int PPT = (P + 255) / 256;  // parameters per thread
  constexpr int SUB = 16;               // nodes staged per LDS round
  const BwdLayout L = bwd_layout(CH);
  const int R = L.rows;
  extern __shared__ float lds[];  // [R][SUB]

  const int t = blockIdx.x;
  const int b = find_instance(prefix, n_inst, t);
  const InstDev I = inst[b];
  const int64_t n_inst_nodes = (int64_t)I.H * I.W;
  const int64_t first = (int64_t)(t - prefix[b]) * kChunk;
  const int nloc = (int)min((int64_t)kChunk, n_inst_nodes - first);
  const int64_t base = I.off + first;

  int x1[PPT], y1[PPT], x2[PPT], y2[PPT];
  float acc[PPT];
#pragma unroll
  for (int k = 0; k < PPT; ++k) {
    const int e = threadIdx.x + 256 * k;
    acc[k] = 0.f;
    if (e < P) param_rows<CH>(e, x1[k], y1[k], x2[k], y2[k]);
    else { x1[k] = -2; y1[k] = x2[k] = y2[k] = -1; }
  }
  for (int s0 = 0; s0 < nloc; s0 += SUB) {
    const int ns = min(SUB, nloc - s0);
    for (int e = threadIdx.x; e < R * SUB; e += 256) {
      const int r = e / SUB, n = e % SUB;
      lds[e] = n < ns ? fac[(int64_t)r * N + base + s0 + n] : 0.f;
    }
    __syncthreads();
#pragma unroll
    for (int k = 0; k < PPT; ++k) {
      if (x1[k] < -1) continue;
      float s = acc[k];
      if (y1[k] < 0) {
        for (int n = 0; n < SUB; ++n) s += lds[x1[k] * SUB + n];
      } else if (x2[k] < 0) {
        for (int n = 0; n < SUB; ++n) s = __builtin_fmaf(lds[x1[k] * SUB + n], lds[y1[k] * SUB + n], s);
      } else {
        for (int n = 0; n < SUB; ++n)
          s = __builtin_fmaf(lds[x2[k] * SUB + n], lds[y2[k] * SUB + n], __builtin_fmaf(lds[x1[k] * SUB + n], lds[y1[k] * SUB + n], s));
      }
      acc[k] = s;
    }
    __syncthreads();
  }
#pragma unroll
  for (int k = 0; k < PPT; ++k) {
    const int e = threadIdx.x + 256 * k;
    if (e < P) partial[(int64_t)t * P + e] = acc[k];
  }
}

// g_theta[e] += sum over chunks in index order.
__global__ void wgrad_final_kernel(const float* __restrict__ partial, int n_chunks, int P, float* __restrict__ g_theta) {
  const int e = blockIdx.x * blockDim.x + threadIdx.x;
  if (e >= P) return;
  double s = 0.0;
  for (int c = 0; c < n_chunks; ++c) s += (double)partial[(int64_t)c * P + e];
  g_theta[e] += (float)s;
}

size_t backward_ws_bytes(const pecnn_plan* plan, int ch) {
  const BwdLayout L = bwd_layout(ch);
  const size_t fac = (size_t)L.rows * (size_t)plan->total * sizeof(float);
  const size_t part = (size_t)plan->n_tiles[kCfgChunk] * (size_t)theta_count(ch) * sizeof(float);
  return fac + 256 + part;
}

int backward_launch(const pecnn_plan* plan, const pecnn_model* m, const float* sp, const float* sc,
                    const float* gn, float* gc, float* gp, float* gth, void* ws, hipStream_t st) {
  const BwdLayout L = bwd_layout(m->ch);
  float* fac = (float*)ws;
  const size_t fac_bytes = (size_t)L.rows * (size_t)plan->total * sizeof(float);
  float* partial = (float*)((char*)ws + ((fac_bytes + 255) / 256) * 256);
  const int nt = plan->n_tiles[kCfgChunk];
  const int32_t* pre = plan->d_prefix[kCfgChunk];
  const int P = (int)theta_count(m->ch);
  if (m->ch == 16) {
    hipLaunchKernelGGL(bwd_node_kernel<16>, dim3(nt), dim3(256), 0, st, plan->d_inst, pre, plan->n, plan->pin, sp, sc,
                       gn, plan->total, m->theta, m->dt, m->isru_alpha, fac);
  } else {
    hipLaunchKernelGGL(bwd_node_kernel<32>, dim3(nt), dim3(256), 0, st, plan->d_inst, pre, plan->n, plan->pin, sp, sc,
                       gn, plan->total, m->theta, m->dt, m->isru_alpha, fac);
  }
  PECNN_LAUNCH_CHECK("bwd_node_kernel");
  if (gc || gp) {
    hipLaunchKernelGGL(bwd_gather_kernel, dim3(nt), dim3(256), 0, st, plan->d_inst, pre, plan->n, plan->pin, gn,
                       plan->total, m->dt, m->ch, fac, gc, gp);
    PECNN_LAUNCH_CHECK("bwd_gather_kernel");
  }
  const size_t lds = (size_t)L.rows * 16 * sizeof(float);
  if (m->ch == 16)
    hipLaunchKernelGGL(bwd_wgrad_kernel<16>, dim3(nt), dim3(256), lds, st, plan->d_inst, pre, plan->n, plan->total,
                       fac, partial);
  else
    hipLaunchKernelGGL(bwd_wgrad_kernel<32>, dim3(nt), dim3(256), lds, st, plan->d_inst, pre, plan->n, plan->total,
                       fac, partial);
  PECNN_LAUNCH_CHECK("bwd_wgrad_kernel");
  hipLaunchKernelGGL(wgrad_final_kernel, dim3((P + 255) / 256), dim3(256), 0, st, partial, nt, P, gth);
  PECNN_LAUNCH_CHECK("wgrad_final_kernel");
  return PECNN_OK;
}

}  // namespace pecnn
