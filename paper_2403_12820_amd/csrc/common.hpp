// Shared device/host definitions of the pecnn HIP library (gfx950 only).
#pragma once
#include <hip/hip_runtime.h>
#include <stdint.h>
#include <stddef.h>

#include "../../include/pecnn.h"

namespace pecnn {

// ----------------------------------------------------------------- per-instance record
// One record per cloth instance, kept in the plan's device memory.
struct InstDev {
  int32_t H, W;    // rows, columns
  int64_t off;     // first node of the instance in the batch planes
  float h, mass;   // rest spacing, node mass
  float ax, ay, az;  // constant external (wind) acceleration
  float pres;        // uniform pressure of eq. (3), N/m^2 (0: none)
};
static_assert(sizeof(InstDev) == 40, "InstDev layout");

// Tile shapes. Each config has its own per-instance tile prefix in the plan.
// Mass-spring step: TX x TY nodes per workgroup, each thread RY nodes along y.
struct MsCfg { int tx, ty, ry; };
constexpr int kNumMsCfg = 5;
constexpr MsCfg kMsCfg[kNumMsCfg] = {{32, 8, 1}, {64, 4, 1}, {16, 16, 1}, {32, 16, 2}, {64, 8, 2}};
// CNN cell: TX x TY nodes per workgroup of 4 waves; TX is a multiple of 16 (one MFMA column block).
struct CnnCfg { int tx, ty; };
constexpr int kNumCnnCfg = 4;
constexpr CnnCfg kCnnCfg[kNumCnnCfg] = {{64, 4}, {32, 8}, {16, 16}, {64, 8}};
// Node-parallel kernels (reductions, backward): flat chunks of kChunk nodes per instance.
constexpr int kChunk = 256;
constexpr int kNumCfg = kNumMsCfg + kNumCnnCfg + 1;
constexpr int kCfgChunk = kNumMsCfg + kNumCnnCfg;
inline int ms_cfg_slot(int c) { return c; }
inline int cnn_cfg_slot(int c) { return kNumMsCfg + c; }

inline __host__ __device__ int tiles_of(int H, int W, int tx, int ty) {
  return ((H + ty - 1) / ty) * ((W + tx - 1) / tx);
}

// ----------------------------------------------------------------- tile scheduling
// Find the instance owning global tile t: largest b with prefix[b] <= t (prefix[0] = 0).
__device__ __forceinline__ int find_instance(const int32_t* __restrict__ prefix, int n, int t) {
  int lo = 0, hi = n;  // invariant: prefix[lo] <= t < prefix[hi]
  while (hi - lo > 1) {
    int mid = (lo + hi) >> 1;
    if (prefix[mid] <= t) lo = mid; else hi = mid;
  }
  return lo;
}

// A persistent workgroup visits its tiles in increasing order, so the owning instance only moves
// forward: the cursor keeps the current instance's record and tile range, and searches (from
// the next instance on) only when a tile leaves that range. Most tiles then cost no load at all
// instead of a chain of dependent loads down a binary search.
struct TileCursor {
  int b;          // current instance, -1 before the first tile
  int start, end; // its tiles: [start, end)
  int flag;       // flags[b] when a per-instance flag array is given, else 0
  InstDev I;
};
__device__ __forceinline__ void cursor_init(TileCursor& c) { c.b = -1; c.start = c.end = 0; }
template <typename F>
__device__ __forceinline__ void cursor_seek(TileCursor& c, const InstDev* __restrict__ inst,
                                            const int32_t* __restrict__ prefix, int n, int t,
                                            const F* __restrict__ flags) {
  if (c.b >= 0 && t < c.end) return;
  int lo = c.b + 1, hi = n;  // t >= prefix[lo] holds: t >= end = prefix[b + 1] (or lo = 0)
  while (hi - lo > 1) {
    const int mid = (lo + hi) >> 1;
    if (prefix[mid] <= t) lo = mid; else hi = mid;
  }
  c.b = lo;
  c.start = prefix[lo];
  c.end = prefix[lo + 1];
  c.I = inst[lo];
  c.flag = flags ? (int)flags[lo] : 0;
}

// Workgroups are dispatched round-robin over the 8 XCDs (each with its own L2). Give each XCD a
// contiguous range of tiles so that neighbouring tiles, which share halo rows, hit the same L2.
// Returns the first tile of this workgroup and the stride between its tiles.
__device__ __forceinline__ void xcd_tile_range(int n_tiles, int& first, int& stride, int& count) {
  const int G = gridDim.x;
  const int w = blockIdx.x;
  const int xcd = w & 7;
  const int groups = (G + 7) >> 3;          // workgroups per XCD (upper bound)
  const int slot = w >> 3;                  // index of this workgroup within its XCD
  const int per_xcd = (n_tiles + 7) >> 3;   // tiles per XCD
  const int base = xcd * per_xcd;
  const int end = min(n_tiles, base + per_xcd);
  // workgroups on this XCD: those w with w % 8 == xcd, w < G
  const int wg_here = (G - xcd + 7) >> 3;
  (void)groups;
  first = base + slot;
  stride = wg_here;
  count = (first < end) ? (end - first + stride - 1) / stride : 0;
}

// Global accesses through a 32-bit byte offset from a base pointer, which lets the compiler use the
// scalar-base + vector-offset addressing mode (batches are validated to stay below 4 GiB per
// state: 24 N_total < 2^32).
template <typename T>
__device__ __forceinline__ T gld(const T* __restrict__ base, unsigned idx) {
  return *reinterpret_cast<const T*>(reinterpret_cast<const char*>(base) + idx * (unsigned)sizeof(float));
}
template <typename T>
__device__ __forceinline__ void gst(T* __restrict__ base, unsigned idx, T v) {
  *reinterpret_cast<T*>(reinterpret_cast<char*>(base) + idx * (unsigned)sizeof(float)) = v;
}

// Eq. (3) at one node: the four nearest neighbours taken round the node in the order right,
// down, left, up; each consecutive pair (j1, j2) whose two nodes are on the grid adds
// (x_j1 - x) x (x_j2 - x). On the flat rest grid (x along columns, y along rows) every pair
// gives +h^2 along z. d[k] = x_k - x for k = right, down, left, up; has[k] says whether the
// neighbour is on the grid (a missing neighbour's d may hold anything finite).
__device__ __forceinline__ void pressure_pairs(const float (&d)[4][3], const bool (&has)[4], float& s0, float& s1,
                                               float& s2) {
  s0 = s1 = s2 = 0.f;
#pragma unroll
  for (int k = 0; k < 4; ++k) {
    const float* a = d[k];
    const float* b = d[(k + 1) & 3];
    const float c0 = __builtin_fmaf(a[1], b[2], -(a[2] * b[1]));
    const float c1 = __builtin_fmaf(a[2], b[0], -(a[0] * b[2]));
    const float c2 = __builtin_fmaf(a[0], b[1], -(a[1] * b[0]));
    const bool on = has[k] && has[(k + 1) & 3];
    s0 += on ? c0 : 0.f;
    s1 += on ? c1 : 0.f;
    s2 += on ? c2 : 0.f;
  }
}

// Adjoint of the eq. (3) term c (x_j1 - x_P) x (x_j2 - x_P) of every node P that reads the position
// of node q = (qi, qj): q itself and its four nearest neighbours. For the adjoint l = dLoss/dv'
// of P's velocity, d/dx_j1 = c (x_j2 - x_P) x l, d/dx_j2 = c l x (x_j1 - x_P), d/dx_P = minus both;
// node q adds the parts where it is P, j1 or j2 into acc. gdv(P, l) gives P's adjoint (zero when P
// is pinned); s_cur holds the positions (planes 0..2 of N floats); off is the instance's first node.
template <typename Gdv>
__device__ __forceinline__ void pressure_adjoint_gather(int H, int W, int64_t off, int qi, int qj, float c,
                                                        const float* __restrict__ s_cur, int64_t N, Gdv gdv,
                                                        float (&acc)[3]) {
  const int R[4][2] = {{0, 1}, {1, 0}, {0, -1}, {-1, 0}};  // right, down, left, up
  for (int o = 0; o < 5; ++o) {
    const int pi = qi + (o == 0 ? 0 : R[o - 1][0]), pj = qj + (o == 0 ? 0 : R[o - 1][1]);
    if (pi < 0 || pi >= H || pj < 0 || pj >= W) continue;
    const int64_t P = off + (int64_t)pi * W + pj;
    float l[3];
    gdv(P, l);
    const float xp0 = s_cur[P], xp1 = s_cur[N + P], xp2 = s_cur[2 * N + P];
    for (int k = 0; k < 4; ++k) {
      const int i1 = pi + R[k][0], j1 = pj + R[k][1];
      const int i2 = pi + R[(k + 1) & 3][0], j2 = pj + R[(k + 1) & 3][1];
      if (i1 < 0 || i1 >= H || j1 < 0 || j1 >= W || i2 < 0 || i2 >= H || j2 < 0 || j2 >= W) continue;
      const bool is1 = i1 == qi && j1 == qj, is2 = i2 == qi && j2 == qj;
      if (o != 0 && !is1 && !is2) continue;
      const int64_t q1 = off + (int64_t)i1 * W + j1, q2 = off + (int64_t)i2 * W + j2;
      const float A0 = s_cur[q1] - xp0, A1 = s_cur[N + q1] - xp1, A2 = s_cur[2 * N + q1] - xp2;
      const float B0 = s_cur[q2] - xp0, B1 = s_cur[N + q2] - xp1, B2 = s_cur[2 * N + q2] - xp2;
      const float g10 = c * (B1 * l[2] - B2 * l[1]), g11 = c * (B2 * l[0] - B0 * l[2]), g12 = c * (B0 * l[1] - B1 * l[0]);
      const float g20 = c * (l[1] * A2 - l[2] * A1), g21 = c * (l[2] * A0 - l[0] * A2), g22 = c * (l[0] * A1 - l[1] * A0);
      if (is1) { acc[0] += g10; acc[1] += g11; acc[2] += g12; }
      if (is2) { acc[0] += g20; acc[1] += g21; acc[2] += g22; }
      if (o == 0) { acc[0] -= g10 + g20; acc[1] -= g11 + g21; acc[2] -= g12 + g22; }
    }
  }
}

// Per-instance sphere record in the plan: centre x, y, z, radius (0: none), friction, padding.
constexpr int kSphereStride = 8;

// Position update of eq. (5) for a free node, x' = x + dt v', with the constraint operator
// extended by a sphere (cloth-object collision by intersection elimination, section 3.1): when
// x + dt v lies inside the sphere (|y - c| < R) the node moves to the nearest surface point
// c + R n, n = (y - c)/|y - c|, its inward normal velocity is removed and its tangential velocity
// is scaled by 1 - friction. sph: the instance's record; v is in/out.
__device__ __forceinline__ void sphere_update(const float* __restrict__ sph, float dt, float x0, float x1, float x2,
                                              float& v0, float& v1, float& v2, float& y0, float& y1, float& y2) {
  y0 = __builtin_fmaf(dt, v0, x0);
  y1 = __builtin_fmaf(dt, v1, x1);
  y2 = __builtin_fmaf(dt, v2, x2);
  const float R = sph[3];
  if (R > 0.f) {
    const float d0 = y0 - sph[0], d1 = y1 - sph[1], d2 = y2 - sph[2];
    const float r2 = __builtin_fmaf(d2, d2, __builtin_fmaf(d1, d1, d0 * d0));
    if (r2 < R * R) {
      float n0 = 0.f, n1 = 0.f, n2 = 1.f;
      if (r2 > 0.f) {
        const float ir = 1.f / __builtin_sqrtf(r2);
        n0 = d0 * ir;
        n1 = d1 * ir;
        n2 = d2 * ir;
      }
      const float vn = __builtin_fmaf(v2, n2, __builtin_fmaf(v1, n1, v0 * n0));
      const float k = 1.f - sph[4], vp = vn > 0.f ? vn : 0.f;
      v0 = __builtin_fmaf(k, v0 - vn * n0, vp * n0);
      v1 = __builtin_fmaf(k, v1 - vn * n1, vp * n1);
      v2 = __builtin_fmaf(k, v2 - vn * n2, vp * n2);
      y0 = __builtin_fmaf(R, n0, sph[0]);
      y1 = __builtin_fmaf(R, n1, sph[1]);
      y2 = __builtin_fmaf(R, n2, sph[2]);
    }
  }
}

struct MsParamsDev {
  float k[3];     // spring constants per family
  float mu, drag;
  float g[3];
  float dt;
};

// ----------------------------------------------------------------- plan
}  // namespace pecnn

struct pecnn_plan {
  int32_t n;
  int64_t total;
  int32_t* H;        // host copies
  int32_t* W;
  int64_t* off;
  float* h;
  float* mass;
  float* a_ext;
  const uint8_t* pin;                   // device, caller-owned
  pecnn::InstDev* d_inst;               // device, inside the caller's plan memory
  int32_t* d_prefix[pecnn::kNumCfg];    // device prefix of tiles per instance, per config
  int32_t* d_chunk_inst;                // device: instance of every node chunk (kChunk nodes)
  int32_t n_tiles[pecnn::kNumCfg];
  int32_t ms_cfg;                       // chosen configs (autotuner or defaults)
  int32_t cnn_cfg;
  int32_t max_hw;                       // largest H*W of an instance
  int32_t vec4;                         // every row of every plane starts 16-byte aligned
  float* pres;                          // host copy of the per-instance pressure (eq. 3)
  int32_t has_pressure;                 // some instance has a non-zero pressure
  float* d_sphere;                      // device: per-instance sphere records (kSphereStride floats)
  int32_t has_sphere;                   // some instance has a sphere
  void* graph_cache;                    // rollout graph cache (host object)
};

namespace pecnn {
void set_error(const char* fmt, ...);
int hip_fail(hipError_t e, const char* what);
int num_cus();
}  // namespace pecnn

#define PECNN_HIP(call)                                  \
  do {                                                   \
    hipError_t e_ = (call);                              \
    if (e_ != hipSuccess) return pecnn::hip_fail(e_, #call); \
  } while (0)

#define PECNN_LAUNCH_CHECK(what)                          \
  do {                                                    \
    hipError_t e_ = hipGetLastError();                    \
    if (e_ != hipSuccess) return pecnn::hip_fail(e_, what); \
  } while (0)
