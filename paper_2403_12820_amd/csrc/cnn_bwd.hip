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
//  3. bwd_wgrad:  per range of nodes, the parameter-gradient partial sums: products of factor
//                 rows summed over nodes, on MFMA from LDS-staged node blocks; then a fixed-order
//                 sum over the ranges into g_theta.
#include "common.hpp"

namespace pecnn {

struct BwdLayout {
  // feature rows of the per-node factor table, each a plane of N floats
  int uk, ud, gus, gud, phi, nn, dd, ga, gb, gphi, gxi, gdv, rows;
};
__host__ __device__ constexpr BwdLayout bwd_layout(int ch) {
  BwdLayout L{};
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

// The per-node factor table is node-blocked: 32 consecutive nodes form a block of rows x 32
// floats, row-major, so a block is one contiguous run (the weight-gradient sums stream it) and a
// row of a block is one 128-byte line (node kernels write it coalesced). Node count padded to 32.
__host__ __device__ inline int64_t fac_node(int64_t q, int rows) { return (q >> 5) * (int64_t)rows * 32 + (q & 31); }
__host__ __device__ inline int64_t fac_floats(int64_t n, int rows) { return (n + 31) / 32 * 32 * (int64_t)rows; }

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

// theta in LDS for the node kernel: the conv block transposed to KT[t][c] (channel fastest), so
// that the per-tap loops read four channels per 16-byte LDS access; the other blocks as in theta.
template <int CH>
struct NodeTheta {
  static constexpr int KT = 0, A = 54 * CH, B = A + CH * CH, WL = B + CH * CH, WN = WL + 3 * CH, WD = WN + 3 * CH,
                       P = WD + 3 * CH + 3;
};

template <int CH>
__global__ __launch_bounds__(256) void bwd_node_kernel(
    const InstDev* __restrict__ inst, const int32_t* __restrict__ prefix, const int32_t* __restrict__ chunk_inst,
    const uint8_t* __restrict__ pin, const float* __restrict__ s_prev, const float* __restrict__ s_cur,
    const float* __restrict__ g_next, int64_t N, const float* __restrict__ theta, float dt, float alpha,
    float* __restrict__ fac) {
  using T = NodeTheta<CH>;
  __shared__ __align__(16) float th[T::P];
  for (int e = threadIdx.x; e < 54 * CH; e += 256) {
    const int t = e / CH, c = e - (e / CH) * CH;
    th[e] = theta[c * 54 + t];
  }
  for (int e = 54 * CH + threadIdx.x; e < T::P; e += 256) th[e] = theta[e];
  __syncthreads();

  int b;
  int local;
  if (!chunk_node(inst, prefix, chunk_inst, blockIdx.x, b, local)) return;
  const InstDev I = inst[b];
  const int i = local / I.W, j = local - (local / I.W) * I.W;
  const int64_t p = I.off + local;
  const BwdLayout L = bwd_layout(CH);
  float* __restrict__ F = fac + fac_node(p, L.rows);  // feature row r of node p lives at F[r * 32]
  auto th4 = [&](int e) { return *reinterpret_cast<const float4*>(&th[e]); };

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
      F[(L.uk + t) * 32] = uk;
      F[(L.ud + t) * 32] = ud;
#pragma unroll
      for (int r = 0; r < CH; r += 4) {
        const float4 w = th4(T::KT + t * CH + r);
        phi[r] = __builtin_fmaf(w.x, uk, phi[r]);
        phi[r + 1] = __builtin_fmaf(w.y, uk, phi[r + 1]);
        phi[r + 2] = __builtin_fmaf(w.z, uk, phi[r + 2]);
        phi[r + 3] = __builtin_fmaf(w.w, uk, phi[r + 3]);
        xi[r] = __builtin_fmaf(w.x, ud, xi[r]);
        xi[r + 1] = __builtin_fmaf(w.y, ud, xi[r + 1]);
        xi[r + 2] = __builtin_fmaf(w.z, ud, xi[r + 2]);
        xi[r + 3] = __builtin_fmaf(w.w, ud, xi[r + 3]);
      }
    }
  }
  // the two Ch x Ch maps of the nonlinear branch: a = A phi, bb = B phi (rows read along c)
  float a[CH], bb[CH];
#pragma unroll
  for (int r = 0; r < CH; ++r) {
    float sa = 0.f, sb = 0.f;
#pragma unroll
    for (int c = 0; c < CH; c += 4) {
      const float4 wa = th4(T::A + r * CH + c), wb = th4(T::B + r * CH + c);
      sa = __builtin_fmaf(wa.x, phi[c], sa);
      sa = __builtin_fmaf(wa.y, phi[c + 1], sa);
      sa = __builtin_fmaf(wa.z, phi[c + 2], sa);
      sa = __builtin_fmaf(wa.w, phi[c + 3], sa);
      sb = __builtin_fmaf(wb.x, phi[c], sb);
      sb = __builtin_fmaf(wb.y, phi[c + 1], sb);
      sb = __builtin_fmaf(wb.z, phi[c + 2], sb);
      sb = __builtin_fmaf(wb.w, phi[c + 3], sb);
    }
    a[r] = sa;
    bb[r] = sb;
  }
  // compiler fence: the weight reads below are issued again rather than kept live from above
  asm volatile("" ::: "memory");
  // adjoint of eq. (5)
  float gdv[3];
  const bool pinned = pin[p] != 0;
#pragma unroll
  for (int k = 0; k < 3; ++k) {
    const float gvt = g_next[(3 + k) * N + p] + dt * g_next[k * N + p];
    gdv[k] = pinned ? 0.f : gvt;
    F[(L.gdv + k) * 32] = gdv[k];
  }
  // heads and ISRU branches; afterwards phi holds the head/derivative part of dLoss/dphi, xi holds
  // dLoss/dxi, and a, bb hold the adjoints of (A phi) and (B phi)
#pragma unroll
  for (int c = 0; c < CH; ++c) {
    const float r1 = __builtin_amdgcn_rsqf(1.f + alpha * phi[c] * phi[c]);
    const float gs = phi[c] * r1, dgs = r1 * r1 * r1;
    const float z = a[c] * bb[c];
    const float r2 = __builtin_amdgcn_rsqf(1.f + alpha * z * z);
    const float nn = z * r2, dnn = r2 * r2 * r2;
    const float dd = xi[c] * gs;
    const float gphi_h = th[T::WL + c] * gdv[0] + th[T::WL + CH + c] * gdv[1] + th[T::WL + 2 * CH + c] * gdv[2];
    const float gnn = th[T::WN + c] * gdv[0] + th[T::WN + CH + c] * gdv[1] + th[T::WN + 2 * CH + c] * gdv[2];
    const float gdd = th[T::WD + c] * gdv[0] + th[T::WD + CH + c] * gdv[1] + th[T::WD + 2 * CH + c] * gdv[2];
    const float gz = gnn * dnn;
    const float ga = gz * bb[c], gb = gz * a[c];
    F[(L.phi + c) * 32] = phi[c];
    F[(L.nn + c) * 32] = nn;
    F[(L.dd + c) * 32] = dd;
    F[(L.ga + c) * 32] = ga;
    F[(L.gb + c) * 32] = gb;
    a[c] = ga;
    bb[c] = gb;
    phi[c] = gphi_h + gdd * xi[c] * dgs;
    xi[c] = gdd * gs;
    F[(L.gxi + c) * 32] = xi[c];
  }
  asm volatile("" ::: "memory");
  // dLoss/dphi += A^T ga + B^T gb (rows of A and B read along c)
#pragma unroll
  for (int r = 0; r < CH; ++r) {
    const float gar = a[r], gbr = bb[r];
#pragma unroll
    for (int c = 0; c < CH; c += 4) {
      const float4 wa = th4(T::A + r * CH + c), wb = th4(T::B + r * CH + c);
      phi[c] = __builtin_fmaf(wb.x, gbr, __builtin_fmaf(wa.x, gar, phi[c]));
      phi[c + 1] = __builtin_fmaf(wb.y, gbr, __builtin_fmaf(wa.y, gar, phi[c + 1]));
      phi[c + 2] = __builtin_fmaf(wb.z, gbr, __builtin_fmaf(wa.z, gar, phi[c + 2]));
      phi[c + 3] = __builtin_fmaf(wb.w, gbr, __builtin_fmaf(wa.w, gar, phi[c + 3]));
    }
  }
#pragma unroll
  for (int c = 0; c < CH; ++c) F[(L.gphi + c) * 32] = phi[c];
  // adjoint of the im2col entries
#pragma unroll 1
  for (int t = 0; t < 54; ++t) {
    float gk = 0.f, gd = 0.f;
#pragma unroll
    for (int c = 0; c < CH; c += 4) {
      const float4 w = th4(T::KT + t * CH + c);
      gk = __builtin_fmaf(w.x, phi[c], gk);
      gk = __builtin_fmaf(w.y, phi[c + 1], gk);
      gk = __builtin_fmaf(w.z, phi[c + 2], gk);
      gk = __builtin_fmaf(w.w, phi[c + 3], gk);
      gd = __builtin_fmaf(w.x, xi[c], gd);
      gd = __builtin_fmaf(w.y, xi[c + 1], gd);
      gd = __builtin_fmaf(w.z, xi[c + 2], gd);
      gd = __builtin_fmaf(w.w, xi[c + 3], gd);
    }
    F[(L.gus + t) * 32] = gk + gd;
    F[(L.gud + t) * 32] = gd;
  }
}

// For node q: g_cur/g_prev += direct terms of eq. (5) + adjoint of the clamped, centre-differenced
// im2col: a tap (c, o) of node p read S_c(clamp(p + o)) (and, for positions, -S_c(p)); plus, with a
// pressure, the adjoint of the eq. (3) term of q and of its four neighbours, which read x_q.
__global__ __launch_bounds__(256) void bwd_gather_kernel(
    const InstDev* __restrict__ inst, const int32_t* __restrict__ prefix, const int32_t* __restrict__ chunk_inst,
    const uint8_t* __restrict__ pin, const float* __restrict__ s_cur, const float* __restrict__ g_next, int64_t N,
    float dt, int ch, const float* __restrict__ fac, float* __restrict__ g_cur, float* __restrict__ g_prev) {
  int b;
  int local;
  if (!chunk_node(inst, prefix, chunk_inst, blockIdx.x, b, local)) return;
  const InstDev I = inst[b];
  const int qi = local / I.W, qj = local - (local / I.W) * I.W;
  const int64_t q = I.off + local;
  const BwdLayout L = bwd_layout(ch);
  const float* __restrict__ gus = fac + L.gus * 32;
  const float* __restrict__ gud = fac + L.gud * 32;
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
            accC[c] += gus[fac_node(pp, L.rows) + (c * 9 + o) * 32];
            accP[c] -= gud[fac_node(pp, L.rows) + (c * 9 + o) * 32];
          }
        }
      }
    }
  // centre term of the position taps of q itself
#pragma unroll
  for (int c = 0; c < 3; ++c)
#pragma unroll
    for (int o = 0; o < 9; ++o) {
      accC[c] -= gus[fac_node(q, L.rows) + (c * 9 + o) * 32];
      accP[c] += gud[fac_node(q, L.rows) + (c * 9 + o) * 32];
    }
  if (I.pres != 0.f) {  // eq. (3): the pressure terms that read x_q (dLoss/dv' of P from the table)
    float acc[3] = {0.f, 0.f, 0.f};
    auto gdv = [&](int64_t P, float (&l)[3]) {
      for (int k = 0; k < 3; ++k) l[k] = fac[fac_node(P, L.rows) + (L.gdv + k) * 32];
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

// Parameter gradients as GEMMs with the node axis as the contraction: for the conv,
// dK = [gphi | gxi] [uk | ud]^T, and dA = ga phi^T, dB = gb phi^T, dW_{L,N,D} = gdv [phi|n|d]^T,
// db_L = gdv 1. Instances are packed end to end in the factor table, so the sums run over the
// flat node range: block k takes nodes [k*NB, (k+1)*NB). Every round stages SUB nodes of all
// factor rows in LDS (the next round's loads are in flight in registers meanwhile) and the four
// waves run v_mfma_f32_16x16x4_f32 on 16 x 16 output tiles (4 nodes per instruction),
// accumulating over the block's nodes in registers. Deterministic: fixed order throughout.
constexpr int kWgSub = 32;          // nodes per LDS round
constexpr int kWgMaxBlocks = 1024;  // partial rows, bounded so the final sum stays small

// nodes per block: a multiple of kWgSub, at most kWgMaxBlocks blocks
inline int64_t wgrad_nodes_per_block(int64_t N) {
  int64_t nb = (N + kWgMaxBlocks - 1) / kWgMaxBlocks;
  nb = (nb + kWgSub - 1) / kWgSub * kWgSub;
  return nb < 256 ? 256 : nb;
}
inline int64_t wgrad_blocks(int64_t N) {
  const int64_t nb = wgrad_nodes_per_block(N);
  return N > 0 ? (N + nb - 1) / nb : 0;
}

struct WgTile {
  int x0, y0;    // first factor row of the X and Y blocks
  int x1, y1;    // second product (conv taps only), or -1
  int kind;      // 0 conv, 1 A, 2 B, 3 W_L, 4 W_N, 5 W_D, 6 b_L
  int xb, yb;    // block indices inside the parameter
};

// The weight sums never read the adjoints of the im2col entries (rows gus and gud, for the input
// gradients): the kernel stages the other rows only, and table row r >= L.phi sits at LDS row
// r - kWgSkip. wg_tile gives rows in that LDS numbering.
constexpr int kWgSkip = 108;  // rows gus and gud
template <int CH>
__host__ __device__ constexpr int wg_rows() { return bwd_layout(CH).rows - kWgSkip; }

template <int CH>
__device__ __forceinline__ WgTile wg_tile(int t) {
  constexpr BwdLayout L0 = bwd_layout(CH);
  static_assert(L0.gus == L0.ud + 54 && L0.phi == L0.gus + kWgSkip, "gus and gud lie between ud and phi");
  // the layout with the skipped rows taken out
  constexpr BwdLayout L = {L0.uk, L0.ud, -1, -1, L0.phi - kWgSkip, L0.nn - kWgSkip, L0.dd - kWgSkip,
                           L0.ga - kWgSkip, L0.gb - kWgSkip, L0.gphi - kWgSkip, L0.gxi - kWgSkip,
                           L0.gdv - kWgSkip, L0.rows - kWgSkip};
  constexpr int MB = CH / 16;
  WgTile T;
  T.x1 = T.y1 = -1;
  if (t < MB * 4) {  // conv: MB row blocks of channels x 4 blocks of taps (54 padded to 64)
    T.kind = 0; T.xb = t / 4; T.yb = t % 4;
    T.x0 = L.gphi + 16 * T.xb; T.y0 = L.uk + 16 * T.yb;
    T.x1 = L.gxi + 16 * T.xb; T.y1 = L.ud + 16 * T.yb;
    return T;
  }
  t -= MB * 4;
  if (t < 2 * MB * MB) {  // A then B: MB x MB blocks each
    const int which = t / (MB * MB), u = t % (MB * MB);
    T.kind = 1 + which; T.xb = u / MB; T.yb = u % MB;
    T.x0 = (which == 0 ? L.ga : L.gb) + 16 * T.xb; T.y0 = L.phi + 16 * T.yb;
    return T;
  }
  t -= 2 * MB * MB;
  T.xb = 0;
  T.x0 = L.gdv;  // three gdv rows; the rows after them are the pad block and are discarded
  if (t < 3 * MB) {  // heads: gdv x MB blocks of phi, n, d
    const int br = t / MB;
    T.kind = 3 + br; T.yb = t % MB;
    T.y0 = (br == 0 ? L.phi : br == 1 ? L.nn : L.dd) + 16 * T.yb;
    return T;
  }
  T.kind = 6; T.yb = 0; T.y0 = L.rows;  // bias: the first pad row holds ones
  return T;
}

template <int CH>
__global__ __launch_bounds__(256) void bwd_wgrad_kernel(const float* __restrict__ fac, int64_t N, int64_t NB,
                                                        float* __restrict__ partial) {
  constexpr int P = CH * 54 + 2 * CH * CH + 9 * CH + 3;
  constexpr int MB = CH / 16;
  constexpr int NT = MB * 4 + 2 * MB * MB + 3 * MB + 1;  // output tiles
  constexpr int TPW = (NT + 3) / 4;                      // tiles per wave
  constexpr BwdLayout L = bwd_layout(CH);
  constexpr int ROWS = L.rows;        // rows of a table block
  constexpr int WROWS = wg_rows<CH>(); // rows staged: all but gus and gud
  constexpr int LS = kWgSub + 4;      // LDS row stride (bank spread)
  extern __shared__ float lds[];      // [WROWS + 16][LS]: the rows, then a pad block (a ones row, then zeros)

  const int lane = threadIdx.x & 63;
  const int wave = __builtin_amdgcn_readfirstlane(threadIdx.x >> 6);
  const int li = lane & 15, g = lane >> 4;
  const int64_t n0 = (int64_t)blockIdx.x * NB;
  const int64_t n1 = min(N, n0 + NB);

  for (int e = threadIdx.x; e < 16 * LS; e += 256) lds[WROWS * LS + e] = (e < kWgSub) ? 1.f : 0.f;

  // a round is one node block of the table: ROWS x 32 contiguous floats; this thread stages the
  // float4 number tid + 256 i of its staged rows (LDS row e4 / 8, nodes 4 (e4 % 8) .. +3), which
  // is float4 e4 of the block before row gus and e4 + 8 kWgSkip after it
  typedef float f32x4 __attribute__((ext_vector_type(4)));
  constexpr int Q = WROWS * (kWgSub / 4);  // float4s per round
  constexpr int PF = (Q + 255) / 256;
  f32x4 pf[PF];
  const int c4 = (threadIdx.x & 7) * 4;
  auto fetch = [&](int64_t s) {
    const f32x4* src = reinterpret_cast<const f32x4*>(fac + (s >> 5) * (int64_t)(ROWS * 32));
    const int64_t left = n1 - s - c4;  // valid nodes from this thread's first column
#pragma unroll
    for (int i = 0; i < PF; ++i) {
      f32x4 v = f32x4{0.f, 0.f, 0.f, 0.f};
      const int e4 = (int)threadIdx.x + 256 * i;
      if (e4 < Q && left > 0) {
        v = src[e4 < L.gus * 8 ? e4 : e4 + 8 * kWgSkip];
        if (left < 4) {  // block tail: table padding beyond the last node is not initialised
          v[3] = 0.f;
          if (left < 3) v[2] = 0.f;
          if (left < 2) v[1] = 0.f;
        }
      }
      pf[i] = v;
    }
  };

  f32x4 acc[TPW];
  WgTile tl[TPW];
#pragma unroll
  for (int k = 0; k < TPW; ++k) {
    acc[k] = f32x4{0.f, 0.f, 0.f, 0.f};
    const int t = wave + 4 * k;
    tl[k] = wg_tile<CH>(t < NT ? t : 0);
  }

  if (n0 < n1) fetch(n0);
  for (int64_t s = n0; s < n1; s += kWgSub) {
#pragma unroll
    for (int i = 0; i < PF; ++i) {
      const int e4 = threadIdx.x + 256 * i;
      if (e4 < Q) *reinterpret_cast<f32x4*>(&lds[(e4 >> 3) * LS + c4]) = pf[i];
    }
    __syncthreads();
    if (s + kWgSub < n1) fetch(s + kWgSub);
#pragma unroll
    for (int k = 0; k < TPW; ++k) {
      if (wave + 4 * k >= NT) continue;  // uniform over the wave
#pragma unroll
      for (int q = 0; q < kWgSub / 4; ++q) {
        const int n = 4 * q + g;
        const float xa = lds[(tl[k].x0 + li) * LS + n], yb = lds[(tl[k].y0 + li) * LS + n];
        acc[k] = __builtin_amdgcn_mfma_f32_16x16x4f32(xa, yb, acc[k], 0, 0, 0);
        if (tl[k].x1 >= 0) {
          const float xc = lds[(tl[k].x1 + li) * LS + n], yd = lds[(tl[k].y1 + li) * LS + n];
          acc[k] = __builtin_amdgcn_mfma_f32_16x16x4f32(xc, yd, acc[k], 0, 0, 0);
        }
      }
    }
    __syncthreads();
  }
  // scatter the tiles to the flat parameter layout: lane holds rows 4g..4g+3, column li
  constexpr int oA = CH * 54, oB = oA + CH * CH, oWL = oB + CH * CH, oWN = oWL + 3 * CH, oWD = oWN + 3 * CH,
                obL = oWD + 3 * CH;
  float* out = partial + (int64_t)blockIdx.x * P;
#pragma unroll
  for (int k = 0; k < TPW; ++k) {
    if (wave + 4 * k >= NT) continue;
    const WgTile T = tl[k];
#pragma unroll
    for (int v = 0; v < 4; ++v) {
      const int i = 16 * T.xb + 4 * g + v, j = 16 * T.yb + li;
      int e = -1;
      if (T.kind == 0) e = j < 54 ? i * 54 + j : -1;
      else if (T.kind == 1) e = oA + i * CH + j;
      else if (T.kind == 2) e = oB + i * CH + j;
      else if (T.kind == 6) e = (i < 3 && j == 0) ? obL + i : -1;
      else if (i < 3) e = (T.kind == 3 ? oWL : T.kind == 4 ? oWN : oWD) + i * CH + j;
      if (e >= 0) out[e] = acc[k][v];
    }
  }
}

// g_theta[e] += sum over the partial rows: 32 threads per parameter each sum a fixed stride of
// rows, then a fixed-order combine in LDS (deterministic). 32 parameters per workgroup, so that a
// batch of 4,067 parameters spreads over 128 workgroups.
constexpr int kWfParams = 32, kWfGroups = 32;
__global__ __launch_bounds__(kWfParams * kWfGroups) void wgrad_final_kernel(const float* __restrict__ partial,
                                                                            int n_rows, int P,
                                                                            float* __restrict__ g_theta) {
  __shared__ double sh[kWfGroups][kWfParams + 1];
  const int pl = threadIdx.x % kWfParams, r0 = threadIdx.x / kWfParams;
  const int e = blockIdx.x * kWfParams + pl;
  double s = 0.0;
  if (e < P)
    for (int r = r0; r < n_rows; r += kWfGroups) s += (double)partial[(int64_t)r * P + e];
  sh[r0][pl] = s;
  __syncthreads();
  if (r0 == 0 && e < P) {
    double t = 0.0;
    for (int k = 0; k < kWfGroups; ++k) t += sh[k][pl];
    g_theta[e] += (float)t;
  }
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
  hipLaunchKernelGGL(wgrad_final_kernel, dim3((kPairP + kWfParams - 1) / kWfParams), dim3(kWfParams * kWfGroups), 0,
                     st, partial, nt, kPairP, gth);
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

size_t backward_ws_bytes(const pecnn_plan* plan, int ch) {
  const BwdLayout L = bwd_layout(ch);
  const size_t fac = (size_t)fac_floats(plan->total, L.rows) * sizeof(float);
  const size_t rows = (size_t)wgrad_blocks(plan->total);
  const size_t part = rows * (size_t)theta_count(ch) * sizeof(float);
  return fac + 256 + part;
}

int backward_launch(const pecnn_plan* plan, const pecnn_model* m, const float* sp, const float* sc,
                    const float* gn, float* gc, float* gp, float* gth, void* ws, hipStream_t st) {
  const BwdLayout L = bwd_layout(m->ch);
  float* fac = (float*)ws;
  const size_t fac_bytes = (size_t)fac_floats(plan->total, L.rows) * sizeof(float);
  float* partial = (float*)((char*)ws + ((fac_bytes + 255) / 256) * 256);
  const int nt = plan->n_tiles[kCfgChunk];
  const int32_t* pre = plan->d_prefix[kCfgChunk];
  const int P = (int)theta_count(m->ch);
  if (m->ch == 16) {
    hipLaunchKernelGGL(bwd_node_kernel<16>, dim3(nt), dim3(256), 0, st, plan->d_inst, pre, plan->d_chunk_inst, plan->pin, sp, sc,
                       gn, plan->total, m->theta, m->dt, m->isru_alpha, fac);
  } else {
    hipLaunchKernelGGL(bwd_node_kernel<32>, dim3(nt), dim3(256), 0, st, plan->d_inst, pre, plan->d_chunk_inst, plan->pin, sp, sc,
                       gn, plan->total, m->theta, m->dt, m->isru_alpha, fac);
  }
  PECNN_LAUNCH_CHECK("bwd_node_kernel");
  if (gc || gp) {
    hipLaunchKernelGGL(bwd_gather_kernel, dim3(nt), dim3(256), 0, st, plan->d_inst, pre, plan->d_chunk_inst, plan->pin, sc,
                       gn, plan->total, m->dt, m->ch, fac, gc, gp);
    PECNN_LAUNCH_CHECK("bwd_gather_kernel");
  }
  const size_t lds = (size_t)(L.rows - kWgSkip + 16) * (kWgSub + 4) * sizeof(float);
  const int64_t nb = wgrad_nodes_per_block(plan->total);
  const int nrows = (int)wgrad_blocks(plan->total);
  if (m->ch == 16)
    hipLaunchKernelGGL(bwd_wgrad_kernel<16>, dim3(nrows), dim3(256), lds, st, fac, plan->total, nb, partial);
  else
    hipLaunchKernelGGL(bwd_wgrad_kernel<32>, dim3(nrows), dim3(256), lds, st, fac, plan->total, nb, partial);
  PECNN_LAUNCH_CHECK("bwd_wgrad_kernel");
  hipLaunchKernelGGL(wgrad_final_kernel, dim3((P + kWfParams - 1) / kWfParams), dim3(kWfParams * kWfGroups), 0, st,
                     partial, nrows, P, gth);
  PECNN_LAUNCH_CHECK("wgrad_final_kernel");
  return PECNN_OK;
}

}  // namespace pecnn
