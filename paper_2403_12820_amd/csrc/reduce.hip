// FP64 diagnostics (position error, energy, stretch ratio), the data term of the loss (eq. 8),
// Adam (Table 1) and the training-window gather. Reductions are two-stage with a fixed order
// (per-chunk sums across lanes and waves, then per-instance or global sums in index order):
// bitwise reproducible run to run.
#include <mutex>

#include "common.hpp"

namespace pecnn {

// forward half of the 12 springs, so that each spring is counted once
struct HalfSpring { int dy, dx, fam; };
__device__ constexpr HalfSpring kHalf[6] = {{0, 1, 0}, {1, 0, 0}, {1, 1, 1}, {1, -1, 1}, {0, 2, 2}, {2, 0, 2}};

// Block reductions of 256 threads in a fixed order: an xor tree inside each 64-lane wave
// (cross-lane moves, no barrier), then the four wave results in wave order through LDS.
constexpr int kWaves = 256 / 64;

template <typename T>
__device__ __forceinline__ T block_sum(T v, T* sh) {
  for (int o = 32; o > 0; o >>= 1) v += __shfl_xor(v, o, 64);
  if ((threadIdx.x & 63) == 0) sh[threadIdx.x >> 6] = v;
  __syncthreads();
  T r = sh[0];
  for (int k = 1; k < kWaves; ++k) r += sh[k];
  __syncthreads();  // sh is reused by the next reduction
  return r;
}
__device__ __forceinline__ double block_max(double v, double* sh) {
  for (int o = 32; o > 0; o >>= 1) v = fmax(v, __shfl_xor(v, o, 64));
  if ((threadIdx.x & 63) == 0) sh[threadIdx.x >> 6] = v;
  __syncthreads();
  double r = sh[0];
  for (int k = 1; k < kWaves; ++k) r = fmax(r, sh[k]);
  __syncthreads();
  return r;
}

// Wave-level reductions in a fixed order (an xor tree over the 64 lanes, no barrier).
__device__ __forceinline__ double wave_sum(double v) {
  for (int o = 32; o > 0; o >>= 1) v += __shfl_xor(v, o, 64);
  return v;
}
__device__ __forceinline__ double wave_max(double v) {
  for (int o = 32; o > 0; o >>= 1) v = fmax(v, __shfl_xor(v, o, 64));
  return v;
}

// Square root of d2 = |x_i - x_j|^2 for FP32 positions widened to FP64: d2 is 0 or at least
// 2^-298 (the square of the smallest FP32 step), so no rescaling of tiny arguments is needed.
// v_rsq_f64 gives the seed y ~ d2^-1/2; one coupled Newton step refines g ~ sqrt(d2) and
// h ~ 1/(2 sqrt(d2)) together, and two Newton corrections g += (d2 - g^2) h finish g (Markstein's
// iteration for the square root). d2 = 0 gives 0; a NaN stays NaN.
__device__ __forceinline__ double spring_length(double d2) {
  const double y = __builtin_amdgcn_rsq(d2);
  double g = d2 * y, h = 0.5 * y;
  const double r = __builtin_fma(-h, g, 0.5);
  g = __builtin_fma(g, r, g);
  h = __builtin_fma(h, r, h);
  double e = __builtin_fma(-g, g, d2);
  g = __builtin_fma(e, h, g);
  e = __builtin_fma(-g, g, d2);
  g = __builtin_fma(e, h, g);
  return d2 == 0.0 ? 0.0 : g;
}

// One wave per chunk of kChunk nodes: lane k takes nodes k, k + 64, k + 128, k + 192 of the
// chunk in that order (every load stays coalesced), then the wave sums its lanes. The stretch
// ratios keep the longest spring of each family and scale it once at the end: a product with a
// positive constant is monotone in its other factor, so max(r) / L = max(r / L) exactly.
constexpr int kLaneNodes = kChunk / 64;
static_assert(kChunk % 64 == 0, "a chunk is whole waves of nodes");

__global__ __launch_bounds__(64) void reduce_chunk_kernel(
    const InstDev* __restrict__ inst, const int32_t* __restrict__ prefix, const int32_t* __restrict__ chunk_inst,
    int64_t N, const float* __restrict__ s, const float* __restrict__ s_ref, MsParamsDev P,
    double* __restrict__ partial) {
  const int t = blockIdx.x;
  const int b = chunk_inst[t];
  const InstDev I = inst[b];
  const int N32 = (int)N;  // validated: 24 N < 2^32, so every element index below fits 31 bits
  const int n_nodes = I.H * I.W;
  const int first = (t - prefix[b]) * kChunk + (int)threadIdx.x;
  // row and column of the lane's first node; each further node is 64 along the row-major order
  int i = first / I.W, j = first - (first / I.W) * I.W;
  const int di = 64 / I.W, dj = 64 - (64 / I.W) * I.W;
  const double hm = 0.5 * (double)I.mass;
  const double mg[3] = {(double)I.mass * ((double)P.g[0] + I.ax), (double)I.mass * ((double)P.g[1] + I.ay),
                        (double)I.mass * ((double)P.g[2] + I.az)};
  const double h = I.h;
  const double L[3] = {h, 1.4142135623730951 * h, 2.0 * h};
  const double hk[3] = {0.5 * (double)P.k[0], 0.5 * (double)P.k[1], 0.5 * (double)P.k[2]};
  double e2 = 0.0, en = 0.0, rmax[3] = {0.0, 0.0, 0.0};
  for (int q = 0; q < kLaneNodes; ++q) {
    const int local = first + 64 * q;
    if (local >= n_nodes) break;
    const int p = (int)I.off + local;
    double x[3], v[3];
#pragma unroll
    for (int a = 0; a < 3; ++a) {
      x[a] = gld(s, (unsigned)(a * N32 + p));
      v[a] = gld(s, (unsigned)((3 + a) * N32 + p));
    }
    // kinetic energy minus the work of gravity and the external field
    const double vv = __builtin_fma(v[2], v[2], __builtin_fma(v[1], v[1], v[0] * v[0]));
    const double gx = __builtin_fma(mg[2], x[2], __builtin_fma(mg[1], x[1], mg[0] * x[0]));
    en += __builtin_fma(hm, vv, -gx);
    if (s_ref) {
#pragma unroll
      for (int a = 0; a < 3; ++a) {
        const double d = x[a] - (double)gld(s_ref, (unsigned)(a * N32 + p));
        e2 = __builtin_fma(d, d, e2);
      }
    }
    // the forward half of the 12 springs, so that each is counted once; which of them exist
    // follows from five comparisons of the node's row and column with the grid's edges
    const bool r1 = i + 1 < I.H, r2 = i + 2 < I.H, c1 = j + 1 < I.W, c2 = j + 2 < I.W, cm = j >= 1;
    const bool ok[6] = {c1, r1, r1 && c1, r1 && cm, c2, r2};
#pragma unroll
    for (int k = 0; k < 6; ++k) {
      if (!ok[k]) continue;
      const int pj = p + kHalf[k].dy * I.W + kHalf[k].dx;
      double d2 = 0.0;
#pragma unroll
      for (int a = 0; a < 3; ++a) {
        const double d = x[a] - (double)gld(s, (unsigned)(a * N32 + pj));
        d2 = __builtin_fma(d, d, d2);
      }
      const double r = spring_length(d2);
      const int f = kHalf[k].fam;
      const double dr = r - L[f];
      en = __builtin_fma(hk[f] * dr, dr, en);
      rmax[f] = fmax(rmax[f], r);
    }
    i += di;
    j += dj;
    if (j >= I.W) {
      j -= I.W;
      ++i;
    }
  }
  // stretch ratios r / L with 1 / L = 1 / h, 1 / (sqrt 2 h), 1 / (2 h)
  const double ih = 1.0 / h;
  const double rs = rmax[0] * ih;
  const double ra = fmax(rs, fmax(rmax[1] * (0.70710678118654752 * ih), rmax[2] * (0.5 * ih)));
  e2 = wave_sum(e2);
  en = wave_sum(en);
  const double st_s = wave_max(rs);
  const double st_a = wave_max(ra);
  if (threadIdx.x == 0) {
    partial[4 * t + 0] = e2;
    partial[4 * t + 1] = en;
    partial[4 * t + 2] = st_s;
    partial[4 * t + 3] = st_a;
  }
}

// One block per instance: thread k takes chunks k, k + 256, ... of the instance in order, then
// a fixed-order block reduction.
__global__ __launch_bounds__(256) void reduce_final_kernel(const int32_t* __restrict__ prefix, int n_inst,
                                                           const double* __restrict__ partial, double* __restrict__ out) {
  __shared__ double sh[kWaves];
  const int b = blockIdx.x;
  double e2 = 0.0, en = 0.0, s1 = 0.0, s2 = 0.0;
  for (int t = prefix[b] + (int)threadIdx.x; t < prefix[b + 1]; t += 256) {
    e2 += partial[4 * t + 0];
    en += partial[4 * t + 1];
    s1 = fmax(s1, partial[4 * t + 2]);
    s2 = fmax(s2, partial[4 * t + 3]);
  }
  e2 = block_sum(e2, sh);
  en = block_sum(en, sh);
  s1 = block_max(s1, sh);
  s2 = block_max(s2, sh);
  if (threadIdx.x == 0) {
    out[4 * b + 0] = e2;
    out[4 * b + 1] = en;
    out[4 * b + 2] = s1;
    out[4 * b + 3] = s2;
  }
}

size_t reduce_ws_bytes(const pecnn_plan* plan) {
  return (size_t)plan->n_tiles[kCfgChunk] * 4 * sizeof(double) + 256;
}

int reduce_launch(const pecnn_plan* plan, const MsParamsDev& P, const float* s, const float* s_ref, double* out,
                  void* ws, hipStream_t st) {
  const int nt = plan->n_tiles[kCfgChunk];
  double* partial = (double*)ws;
  hipLaunchKernelGGL(reduce_chunk_kernel, dim3(nt), dim3(64), 0, st, plan->d_inst, plan->d_prefix[kCfgChunk],
                     plan->d_chunk_inst, plan->total, s, s_ref, P, partial);
  PECNN_LAUNCH_CHECK("reduce_chunk_kernel");
  hipLaunchKernelGGL(reduce_final_kernel, dim3(plan->n), dim3(256), 0, st, plan->d_prefix[kCfgChunk],
                     plan->n, partial, out);
  PECNN_LAUNCH_CHECK("reduce_final_kernel");
  return PECNN_OK;
}

// ---------------------------------------------------------------- allocation-free diagnostics
// The per-chunk partials of cloth_reduce_fp64_noalloc live in this file-scope array: each device
// holds its own copy, at its own address, until the process ends. In host code the array's name
// is only a stand-in, so kernels get the address looked up below (once per device, with that
// device current), never the name.
static_assert(PECNN_NOALLOC_REDUCE_MAX_CHUNKS % 64 == 0, "partials array size");
static __device__ __align__(256) double scratch[4 * PECNN_NOALLOC_REDUCE_MAX_CHUNKS];

namespace {
constexpr int kMaxDevices = 64;
std::mutex g_scratch_mu;
double* g_scratch[kMaxDevices];
}  // namespace

int reduce_scratch(double** out) {
  int dev = -1;
  hipError_t e = hipGetDevice(&dev);
  if (e != hipSuccess) return hip_fail(e, "hipGetDevice");
  if (dev < 0 || dev >= kMaxDevices) {
    set_error("device %d is beyond the %d devices the library tracks", dev, kMaxDevices);
    return PECNN_E_UNSUPPORTED;
  }
  std::lock_guard<std::mutex> lock(g_scratch_mu);
  if (!g_scratch[dev]) {
    void* ptr = nullptr;
    e = hipGetSymbolAddress(&ptr, HIP_SYMBOL(scratch));
    if (e != hipSuccess) return hip_fail(e, "hipGetSymbolAddress(scratch)");
    if (!ptr) { set_error("hipGetSymbolAddress(scratch) gave a null address"); return PECNN_E_HIP; }
    g_scratch[dev] = (double*)ptr;
  }
  if (out) *out = g_scratch[dev];
  return PECNN_OK;
}

// ---------------------------------------------------------------- loss (eq. 8, data term)
__global__ __launch_bounds__(256) void loss_chunk_kernel(
    const InstDev* __restrict__ inst, const int32_t* __restrict__ prefix, const int32_t* __restrict__ chunk_inst,
    int64_t N, const uint8_t* __restrict__ pin, const float* __restrict__ sh_, const float* __restrict__ st_, float isx2,
    float isv2, float gscale, double* __restrict__ partial, float* __restrict__ g) {
  __shared__ double sh[256];
  const int t = blockIdx.x;
  const int b = chunk_inst[t];
  const InstDev I = inst[b];
  const int local = (t - prefix[b]) * kChunk + (int)threadIdx.x;
  double acc = 0.0;
  if (local < I.H * I.W) {
    const int64_t p = I.off + local;
    if (!pin[p]) {
      for (int c = 0; c < 6; ++c) {
        const float d = sh_[c * N + p] - st_[c * N + p];
        const float is2 = c < 3 ? isx2 : isv2;
        acc += (double)d * (double)d * (double)is2;
        if (g) g[c * N + p] += gscale * d * is2;
      }
    }
  }
  acc = block_sum(acc, sh);
  if (threadIdx.x == 0) partial[t] = acc;
}

__global__ __launch_bounds__(256) void loss_final_kernel(const double* __restrict__ partial, int n, double scale,
                                                          double* __restrict__ loss) {
  __shared__ double sh[256];
  double s = 0.0;
  for (int t = threadIdx.x; t < n; t += 256) s += partial[t];
  s = block_sum(s, sh);
  if (threadIdx.x == 0) *loss += scale * s;
}

// The gradient alone (no value asked for): the same per-element expression as loss_chunk_kernel,
// so g is the same to the bit, without the sums.
__global__ __launch_bounds__(256) void loss_grad_kernel(
    const InstDev* __restrict__ inst, const int32_t* __restrict__ prefix, const int32_t* __restrict__ chunk_inst,
    int64_t N, const uint8_t* __restrict__ pin, const float* __restrict__ sh_, const float* __restrict__ st_, float isx2,
    float isv2, float gscale, float* __restrict__ g) {
  const int t = blockIdx.x;
  const int b = chunk_inst[t];
  const InstDev I = inst[b];
  const int local = (t - prefix[b]) * kChunk + (int)threadIdx.x;
  if (local >= I.H * I.W) return;
  const int64_t p = I.off + local;
  if (pin[p]) return;
#pragma unroll
  for (int c = 0; c < 6; ++c) {
    const float d = sh_[c * N + p] - st_[c * N + p];
    const float is2 = c < 3 ? isx2 : isv2;
    g[c * N + p] += gscale * d * is2;
  }
}

int loss_launch(const pecnn_plan* plan, const float* s_hat, const float* s_true, float sx, float sv, float w,
                int64_t n_free, double* loss, float* g, void* ws, hipStream_t st) {
  const int nt = plan->n_tiles[kCfgChunk];
  double* partial = (double*)ws;
  const float isx2 = 1.f / (sx * sx), isv2 = 1.f / (sv * sv);
  const float gscale = (float)(2.0 * (double)w / (double)n_free);
  if (!loss) {
    hipLaunchKernelGGL(loss_grad_kernel, dim3(nt), dim3(256), 0, st, plan->d_inst, plan->d_prefix[kCfgChunk],
                       plan->d_chunk_inst, plan->total, plan->pin, s_hat, s_true, isx2, isv2, gscale, g);
    PECNN_LAUNCH_CHECK("loss_grad_kernel");
    return PECNN_OK;
  }
  hipLaunchKernelGGL(loss_chunk_kernel, dim3(nt), dim3(256), 0, st, plan->d_inst, plan->d_prefix[kCfgChunk],
                     plan->d_chunk_inst, plan->total, plan->pin, s_hat, s_true, isx2, isv2, gscale, partial, g);
  PECNN_LAUNCH_CHECK("loss_chunk_kernel");
  hipLaunchKernelGGL(loss_final_kernel, dim3(1), dim3(256), 0, st, partial, nt, (double)w / (double)n_free, loss);
  PECNN_LAUNCH_CHECK("loss_final_kernel");
  return PECNN_OK;
}

// ---------------------------------------------------------------- Adam
__global__ void adam_kernel(int64_t n, float lr, float b1, float b2, float eps, float ibc1, float ibc2,
                            float* __restrict__ th, float* __restrict__ m, float* __restrict__ v,
                            const float* __restrict__ g) {
  const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= n) return;
  const float gi = g[i];
  const float mi = b1 * m[i] + (1.f - b1) * gi;
  const float vi = b2 * v[i] + (1.f - b2) * gi * gi;
  m[i] = mi;
  v[i] = vi;
  th[i] -= lr * (mi * ibc1) / (sqrtf(vi * ibc2) + eps);
}

int adam_launch(int64_t n, float lr, float b1, float b2, float eps, int t, float* th, float* m, float* v,
                const float* g, hipStream_t st) {
  const double bc1 = 1.0 - pow((double)b1, t), bc2 = 1.0 - pow((double)b2, t);
  hipLaunchKernelGGL(adam_kernel, dim3((unsigned)((n + 255) / 256)), dim3(256), 0, st, n, lr, b1, b2, eps,
                     (float)(1.0 / bc1), (float)(1.0 / bc2), th, m, v, g);
  PECNN_LAUNCH_CHECK("adam_kernel");
  return PECNN_OK;
}

// ---------------------------------------------------------------- training windows
__global__ void gather_kernel(const float* __restrict__ traj, int64_t traj_nodes, int n_saved,
                              const int64_t* __restrict__ traj_off, int n_traj, const int32_t* __restrict__ traj_inst,
                              const int32_t* __restrict__ frame_idx, int n_win, int npw, int n_frames,
                              float* __restrict__ out) {
  const int w = blockIdx.y;
  const int tc = blockIdx.z;  // frame * 6 + channel
  const int t = tc / 6, c = tc % 6;
  const int64_t node = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (node >= npw) return;
  int f = frame_idx[w] + t;
  f = f < 0 ? 0 : (f >= n_saved ? n_saved - 1 : f);
  int b = traj_inst[w];
  b = b < 0 ? 0 : (b >= n_traj ? n_traj - 1 : b);
  const int64_t lo = traj_off[b], hi = traj_off[b + 1];
  const int64_t tot = (int64_t)n_win * npw;
  float v = 0.f;
  if (lo + node < hi && hi <= traj_nodes) v = traj[((int64_t)f * 6 + c) * traj_nodes + lo + node];
  out[((int64_t)t * 6 + c) * tot + (int64_t)w * npw + node] = v;
}

int gather_launch(const float* traj, int64_t traj_nodes, int n_saved, const int64_t* traj_off, int n_traj,
                  const int32_t* traj_inst, const int32_t* frame_idx, int n_win, int npw, int n_frames,
                  float* out, hipStream_t st) {
  dim3 grid((npw + 255) / 256, n_win, n_frames * 6);
  hipLaunchKernelGGL(gather_kernel, grid, dim3(256), 0, st, traj, traj_nodes, n_saved, traj_off, n_traj, traj_inst,
                     frame_idx, n_win, npw, n_frames, out);
  PECNN_LAUNCH_CHECK("gather_kernel");
  return PECNN_OK;
}

}  // namespace pecnn
