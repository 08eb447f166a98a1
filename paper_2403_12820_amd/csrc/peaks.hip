// Peaks of the device, measured with short synthetic kernels, so that the rooflines can be quoted
// against the chip at hand as well as against the datasheet: a streaming copy (HBM), chains of
// FP32 and FP64 fused multiply-adds and of v_rsq_f32 (vector ALU), and chains of the two MFMA
// forms the frame and the training kernels use. Every loop has a fixed trip count and every
// result is stored, so nothing is optimised away and every launch ends.
#include "cnn_common.hpp"

namespace pecnn {

constexpr int kPeakChains = 16;  // independent dependency chains per lane
constexpr int kPeakBlocksPerCu = 4;

// Each thread keeps four 16-byte loads in flight (one per quarter of a block-sized stride) before
// it stores them; the tail of the buffer goes one piece at a time.
constexpr int kCopyUnroll = 4;
__global__ __launch_bounds__(256) void copy_peak_kernel(const float4* __restrict__ src, float4* __restrict__ dst,
                                                        int64_t n4) {
  const int64_t step = (int64_t)gridDim.x * 256 * kCopyUnroll;
  const int64_t full = n4 / step * step;
  int64_t i = (int64_t)blockIdx.x * 256 * kCopyUnroll + threadIdx.x;
  const f32x4* __restrict__ s4 = reinterpret_cast<const f32x4*>(src);
  f32x4* __restrict__ d4 = reinterpret_cast<f32x4*>(dst);
  for (; i < full; i += step) {
    f32x4 v[kCopyUnroll];
#pragma unroll
    for (int k = 0; k < kCopyUnroll; ++k) v[k] = __builtin_nontemporal_load(&s4[i + 256 * k]);
#pragma unroll
    for (int k = 0; k < kCopyUnroll; ++k) __builtin_nontemporal_store(v[k], &d4[i + 256 * k]);
  }
  for (int64_t j = full + (int64_t)blockIdx.x * 256 + threadIdx.x; j < n4; j += (int64_t)gridDim.x * 256)
    dst[j] = src[j];
}

__global__ __launch_bounds__(256) void fma32_peak_kernel(float* __restrict__ out, int iters, float b, float c) {
  float a[kPeakChains];
#pragma unroll
  for (int k = 0; k < kPeakChains; ++k) a[k] = 1e-3f * (float)(threadIdx.x & 63) + (float)k;
  for (int it = 0; it < iters; ++it)
#pragma unroll
    for (int k = 0; k < kPeakChains; ++k) a[k] = __builtin_fmaf(a[k], b, c);
  float s = 0.f;
#pragma unroll
  for (int k = 0; k < kPeakChains; ++k) s += a[k];
  out[(int64_t)blockIdx.x * 256 + threadIdx.x] = s;
}

__global__ __launch_bounds__(256) void rsq_peak_kernel(float* __restrict__ out, int iters, float c) {
  float a[kPeakChains];
#pragma unroll
  for (int k = 0; k < kPeakChains; ++k) a[k] = 1.f + 1e-3f * (float)k;
  for (int it = 0; it < iters; ++it)
#pragma unroll
    for (int k = 0; k < kPeakChains; ++k) a[k] = __builtin_amdgcn_rsqf(a[k] + c);  // stays near 0.8
  float s = 0.f;
#pragma unroll
  for (int k = 0; k < kPeakChains; ++k) s += a[k];
  out[(int64_t)blockIdx.x * 256 + threadIdx.x] = s;
}

__global__ __launch_bounds__(256) void fma64_peak_kernel(double* __restrict__ out, int iters, double b, double c) {
  double a[kPeakChains];
#pragma unroll
  for (int k = 0; k < kPeakChains; ++k) a[k] = 1e-3 * (double)(threadIdx.x & 63) + (double)k;
  for (int it = 0; it < iters; ++it)
#pragma unroll
    for (int k = 0; k < kPeakChains; ++k) a[k] = __builtin_fma(a[k], b, c);
  double s = 0.0;
#pragma unroll
  for (int k = 0; k < kPeakChains; ++k) s += a[k];
  out[(int64_t)blockIdx.x * 256 + threadIdx.x] = s;
}

// Four independent accumulators per wave; operands from the lane id (small values, no overflow).
__global__ __launch_bounds__(256) void mfma_bf16_peak_kernel(float* __restrict__ out, int iters) {
  const int lane = threadIdx.x & 63;
  bf16x8 a, b;
#pragma unroll
  for (int e = 0; e < 8; ++e) {
    a[e] = (__bf16)(1e-3f * (float)((lane + e) & 15));
    b[e] = (__bf16)(1e-3f * (float)((lane * 3 + e) & 15));
  }
  f32x4 acc[4];
#pragma unroll
  for (int k = 0; k < 4; ++k) acc[k] = f32x4{0.f, 0.f, 0.f, 0.f};
  for (int it = 0; it < iters; ++it)
#pragma unroll
    for (int k = 0; k < 4; ++k) acc[k] = __builtin_amdgcn_mfma_f32_16x16x32_bf16(a, b, acc[k], 0, 0, 0);
  float s = 0.f;
#pragma unroll
  for (int k = 0; k < 4; ++k) s += acc[k][0] + acc[k][1] + acc[k][2] + acc[k][3];
  out[(int64_t)blockIdx.x * 256 + threadIdx.x] = s;
}

__global__ __launch_bounds__(256) void mfma_f32_peak_kernel(float* __restrict__ out, int iters) {
  const int lane = threadIdx.x & 63;
  const float a = 1e-3f * (float)(lane & 15), b = 1e-3f * (float)((lane * 3) & 15);
  f32x4 acc[4];
#pragma unroll
  for (int k = 0; k < 4; ++k) acc[k] = f32x4{0.f, 0.f, 0.f, 0.f};
  for (int it = 0; it < iters; ++it)
#pragma unroll
    for (int k = 0; k < 4; ++k) acc[k] = __builtin_amdgcn_mfma_f32_16x16x4f32(a, b, acc[k], 0, 0, 0);
  float s = 0.f;
#pragma unroll
  for (int k = 0; k < 4; ++k) s += acc[k][0] + acc[k][1] + acc[k][2] + acc[k][3];
  out[(int64_t)blockIdx.x * 256 + threadIdx.x] = s;
}

// Time one launch (after an untimed one) and return work / second.
template <typename F>
static int timed_rate(hipStream_t st, hipEvent_t e0, hipEvent_t e1, double work, const F& launch, double* rate) {
  launch();
  PECNN_LAUNCH_CHECK("peak kernel");
  PECNN_HIP(hipEventRecord(e0, st));
  launch();
  PECNN_LAUNCH_CHECK("peak kernel");
  PECNN_HIP(hipEventRecord(e1, st));
  PECNN_HIP(hipEventSynchronize(e1));
  float ms = 0.f;
  PECNN_HIP(hipEventElapsedTime(&ms, e0, e1));
  *rate = ms > 0.f ? work / (1e-3 * (double)ms) : 0.0;
  return PECNN_OK;
}

static int measure(double* out, char* scratch, size_t bytes, hipStream_t st, hipEvent_t e0, hipEvent_t e1) {
  const int grid = num_cus() * kPeakBlocksPerCu;
  const size_t res_bytes = ((size_t)grid * 256 * sizeof(double) + 255) / 256 * 256;
  float* r32 = (float*)scratch;
  double* r64 = (double*)scratch;
  const double lanes = (double)grid * 256.0, waves = (double)grid * 4.0;
  // HBM: the two halves of the rest of the buffer
  const int64_t n4 = (int64_t)((bytes - res_bytes) / 2 / sizeof(float4));
  const float4* src = (const float4*)(scratch + res_bytes);
  float4* dst = (float4*)(scratch + res_bytes) + n4;
  int rc = timed_rate(st, e0, e1, 2.0 * (double)n4 * sizeof(float4), [&] {
    hipLaunchKernelGGL(copy_peak_kernel, dim3(grid * 2), dim3(256), 0, st, src, dst, n4);
  }, &out[0]);
  if (rc) return rc;
  // about 2 ms per kernel at the datasheet rates
  const int it_valu = 20000, it_rsq = 5000, it_mfma = 20000, it_mfma32 = 10000;
  if ((rc = timed_rate(st, e0, e1, lanes * it_valu * kPeakChains, [&] {
         hipLaunchKernelGGL(fma32_peak_kernel, dim3(grid), dim3(256), 0, st, r32, it_valu, 0.999f, 1e-3f);
       }, &out[1])))
    return rc;
  if ((rc = timed_rate(st, e0, e1, lanes * it_rsq * kPeakChains, [&] {
         hipLaunchKernelGGL(rsq_peak_kernel, dim3(grid), dim3(256), 0, st, r32, it_rsq, 0.5f);
       }, &out[2])))
    return rc;
  if ((rc = timed_rate(st, e0, e1, lanes * it_valu * kPeakChains, [&] {
         hipLaunchKernelGGL(fma64_peak_kernel, dim3(grid), dim3(256), 0, st, r64, it_valu, 0.999, 1e-3);
       }, &out[3])))
    return rc;
  if ((rc = timed_rate(st, e0, e1, waves * it_mfma * 4 * 16.0 * 16.0 * 32.0 * 2.0, [&] {
         hipLaunchKernelGGL(mfma_bf16_peak_kernel, dim3(grid), dim3(256), 0, st, r32, it_mfma);
       }, &out[4])))
    return rc;
  return timed_rate(st, e0, e1, waves * it_mfma32 * 4 * 16.0 * 16.0 * 4.0 * 2.0, [&] {
    hipLaunchKernelGGL(mfma_f32_peak_kernel, dim3(grid), dim3(256), 0, st, r32, it_mfma32);
  }, &out[5]);
}

}  // namespace pecnn

using namespace pecnn;

extern "C" int pecnn_measure_peaks(double* out, void* scratch, size_t scratch_bytes, void* stream) {
  if (!out || !scratch) {
    set_error("null output or scratch");
    return PECNN_E_INVALID;
  }
  if (scratch_bytes < ((size_t)64 << 20) || ((uintptr_t)scratch & 255) != 0) {
    set_error("scratch of at least 64 MiB, 256-byte aligned, needed (%zu bytes given)", scratch_bytes);
    return PECNN_E_WORKSPACE;
  }
  hipEvent_t e0 = nullptr, e1 = nullptr;
  PECNN_HIP(hipEventCreate(&e0));
  hipError_t e = hipEventCreate(&e1);
  if (e != hipSuccess) {
    (void)hipEventDestroy(e0);
    return hip_fail(e, "hipEventCreate");
  }
  const int rc = measure(out, (char*)scratch, scratch_bytes, (hipStream_t)stream, e0, e1);
  (void)hipEventDestroy(e0);
  (void)hipEventDestroy(e1);
  return rc;
}
