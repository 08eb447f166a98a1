// C ABI of the pecnn library: argument validation, plans, workspace queries, the rollout
// orchestration (hipGraph-captured chunks with a per-instance guard and fall-back to the
// mass-spring step) and the tile autotuner.
#include <math.h>
#include <stdarg.h>
#include <stdio.h>
#include <stdlib.h>
#include <string.h>

#include <functional>
#include <vector>

#include <rocprofiler-sdk-roctx/roctx.h>

#include "common.hpp"

namespace pecnn {
// kernels in the other translation units
MsParamsDev ms_params_dev(const cloth_ms_params* p);
int ms_step_once(const pecnn_plan*, int cfg, const MsParamsDev&, const float*, float*, const uint8_t*, hipStream_t);
int ms_step_run(const pecnn_plan*, int cfg, const MsParamsDev&, const float*, float*, float*, int,
                const uint8_t*, hipStream_t);
int cnn_forward_launch(const pecnn_plan*, int cfg, const pecnn_model*, const float*, const float*, float*,
                       const int32_t*, hipStream_t);
size_t backward_ws_bytes(const pecnn_plan*, int ch);
size_t pair_backward_ws_bytes(const pecnn_plan*);
int pair_backward_launch(const pecnn_plan*, const pecnn_model*, const float*, const float*, float*, float*, void*,
                         hipStream_t);
int backward_launch(const pecnn_plan*, const pecnn_model*, const float*, const float*, const float*, float*,
                    float*, float*, void*, hipStream_t);
int sphere_adjoint_launch(const pecnn_plan*, float, const float*, const float*, const float*, float*, hipStream_t);
int zero_floats_launch(float*, int64_t, hipStream_t);
size_t reduce_ws_bytes(const pecnn_plan*);
int reduce_launch(const pecnn_plan*, const MsParamsDev&, const float*, const float*, double*, void*, hipStream_t);
int reduce_scratch(double**);
int loss_launch(const pecnn_plan*, const float*, const float*, float, float, float, int64_t, double*, float*, void*,
                hipStream_t);
int adam_launch(int64_t, float, float, float, float, int, float*, float*, float*, const float*, hipStream_t);
int gather_launch(const float*, int64_t, int, const int64_t*, int, const int32_t*, const int32_t*, int, int, int,
                  float*, hipStream_t);

static thread_local char g_err[512] = "";

void set_error(const char* fmt, ...) {
  va_list ap;
  va_start(ap, fmt);
  vsnprintf(g_err, sizeof(g_err), fmt, ap);
  va_end(ap);
}

int hip_fail(hipError_t e, const char* what) {
  set_error("%s: %s", what, hipGetErrorString(e));
  return PECNN_E_HIP;
}

int num_cus() {
  static int cached = 0;
  if (cached == 0) {
    int dev = 0, n = 0;
    if (hipGetDevice(&dev) == hipSuccess && hipDeviceGetAttribute(&n, hipDeviceAttributeMultiprocessorCount, dev) == hipSuccess && n > 0)
      cached = n;
    else
      cached = 256;
  }
  return cached;
}

static bool finite_pos(float x) { return isfinite(x) && x > 0.f; }
static bool finite_nonneg(float x) { return isfinite(x) && x >= 0.f; }

static size_t align256(size_t x) { return (x + 255) & ~(size_t)255; }

// A roctx range over a host-side scope (a no-op unless a tracer such as rocprofv3
// --marker-trace is attached): the entry points that queue many kernels mark their phases.
struct TraceRange {
  explicit TraceRange(const char* what) { roctxRangePushA(what); }
  ~TraceRange() { roctxRangePop(); }
  TraceRange(const TraceRange&) = delete;
  TraceRange& operator=(const TraceRange&) = delete;
};

static int check_ms_params(const cloth_ms_params* p) {
  if (!p) { set_error("null cloth_ms_params"); return PECNN_E_INVALID; }
  if (!finite_nonneg(p->k_struct) || !finite_nonneg(p->k_shear) || !finite_nonneg(p->k_bend) ||
      !finite_nonneg(p->mu) || !finite_nonneg(p->drag) || !finite_pos(p->dt) || !isfinite(p->g[0]) ||
      !isfinite(p->g[1]) || !isfinite(p->g[2])) {
    set_error("cloth_ms_params: spring constants, damping and drag must be finite and >= 0, dt finite and > 0");
    return PECNN_E_INVALID;
  }
  return PECNN_OK;
}

static int check_model(const pecnn_model* m) {
  if (!m || !m->theta) { set_error("null model or theta"); return PECNN_E_INVALID; }
  if (m->cell == PECNN_CELL_PAIR) {
    if (m->ch != 12 || m->precision != PECNN_FP32) {
      set_error("the pair cell has 12 channels and FP32 operands");
      return PECNN_E_UNSUPPORTED;
    }
  } else if (m->cell != PECNN_CELL_CONV) {
    set_error("cell %d unsupported", m->cell);
    return PECNN_E_UNSUPPORTED;
  } else if (m->ch != 16 && m->ch != 32) { set_error("channel count %d unsupported (16 or 32)", m->ch); return PECNN_E_UNSUPPORTED; }
  if (m->precision != PECNN_FP32 && m->precision != PECNN_BF16) { set_error("precision %d unsupported", m->precision); return PECNN_E_UNSUPPORTED; }
  if (!finite_pos(m->dt) || !finite_pos(m->isru_alpha)) { set_error("model dt and isru_alpha must be finite and > 0"); return PECNN_E_INVALID; }
  return PECNN_OK;
}

static int check_plan(const pecnn_plan* plan) {
  if (!plan || !plan->d_inst) { set_error("null plan"); return PECNN_E_INVALID; }
  return PECNN_OK;
}

// ---------------------------------------------------------------- rollout graph cache
struct GraphKey {
  const void* buf[2];       // the caller's s_prev, s_cur (the other states live in ws)
  int pi, ci;               // states S^{k-1}, S^k of the chunk's first frame (indices, see rollout)
  int pre_len, pre_code;    // leading frames of the chunk that follow the prefix schedule
  int len, with_ms, guard, ms_cfg, cnn_cfg, ch, prec, cell, substeps;
  float dt, alpha;
  const float* theta;
  cloth_ms_params sim;
  pecnn_guard gd;
  const int32_t* fallback;
  const void* ws;
  const double* stats;
  bool operator==(const GraphKey& o) const { return memcmp(this, &o, sizeof(GraphKey)) == 0; }
};
struct GraphEntry {
  GraphKey key;
  hipGraphExec_t exec;
};
struct GraphCache {
  std::vector<GraphEntry> entries;
  hipStream_t capture = nullptr;
  int* host_count = nullptr;           // [2] pinned: fallen instances after a check, two in flight
  hipEvent_t count_ready[2] = {nullptr, nullptr};
};

static void graph_cache_free(pecnn_plan* plan) {
  GraphCache* gc = (GraphCache*)plan->graph_cache;
  if (!gc) return;
  for (auto& e : gc->entries) (void)hipGraphExecDestroy(e.exec);
  if (gc->capture) (void)hipStreamDestroy(gc->capture);
  if (gc->host_count) (void)hipHostFree(gc->host_count);
  for (hipEvent_t e : gc->count_ready)
    if (e) (void)hipEventDestroy(e);
  delete gc;
  plan->graph_cache = nullptr;
}

// ---------------------------------------------------------------- guard kernels
// Every check: per instance, compare the largest structural stretch ratio and the energy gain
// with the guard's bounds (no energy check where the energy scale is infinite: instances with a
// pressure) and, when the frame-error test is on, the squared position difference from the
// simulator's frame times escale = 1 / (nodes width^2) with the squared bound; a tripped
// instance falls back for good. Also counts fallen instances.
// count[0] receives the number of fallen instances, count[1] keeps the index of the check.
// mode 0: a check; 1: the prologue (starting energy and stretch, no test); 2: the diagnostics of
// the last check taken again from a repaired state (no test, same check index). len: frames of
// the chunk the check ends (all chunks but a call's last have check_every).
__global__ __launch_bounds__(256) void guard_kernel(int n, const double* __restrict__ now, double* __restrict__ e0,
                                                    const double* __restrict__ eref,
                                                    const double* __restrict__ escale, pecnn_guard G, int mode,
                                                    int len,
                                                    int32_t* __restrict__ fallback, uint8_t* __restrict__ active_ms,
                                                    uint8_t* __restrict__ tripped, double* __restrict__ stats,
                                                    int* __restrict__ count) {
  __shared__ int sh[256];
  const int chk = mode == 1 ? 0 : (mode == 2 ? count[1] : count[1] + 1);
  const int step = (chk - 1) * G.check_every + len;  // frames since the call began
  const bool ferr = G.frame_err_max > 0.f;
  const double ferr2 = (double)G.frame_err_max * (double)G.frame_err_max;
  int cnt = 0;
  for (int b = threadIdx.x; b < n; b += 256) {
    const double e = now[4 * b + 1], st = now[4 * b + 2];
    if (mode != 2) tripped[b] = 0;
    if (mode == 1) {
      e0[b] = e;
      stats[4 * b + 0] = e;
      stats[4 * b + 2] = st;
      stats[4 * b + 3] = fallback[b] ? 0.0 : -1.0;
    } else if (mode == 0 && fallback[b] == 0 &&
               (!(st <= (double)G.stretch_max) ||
                (isfinite(eref[b]) && !((e - e0[b]) / eref[b] <= (double)G.energy_gain_max)) ||
                (ferr && !(now[4 * b] * escale[b] <= ferr2)))) {
      fallback[b] = 1;
      tripped[b] = 1;
      stats[4 * b + 3] = step;
    }
    stats[4 * b + 1] = e;
    stats[4 * b + 2] = fmax(stats[4 * b + 2], st);
    active_ms[b] = fallback[b] != 0;
    cnt += fallback[b] != 0;
  }
  sh[threadIdx.x] = cnt;
  __syncthreads();
  for (int s = 128; s > 0; s >>= 1) {
    if (threadIdx.x < s) sh[threadIdx.x] += sh[threadIdx.x + s];
    __syncthreads();
  }
  if (threadIdx.x == 0) {
    count[0] = sh[0];
    count[1] = chk;
  }
}

// active[b] = instance b fell back before the last check (fallen, but not at that check).
__global__ __launch_bounds__(256) void late_mask_kernel(int n, const int32_t* __restrict__ fallback,
                                                        const uint8_t* __restrict__ tripped,
                                                        uint8_t* __restrict__ active) {
  for (int b = threadIdx.x; b < n; b += 256) active[b] = fallback[b] != 0 && tripped[b] == 0;
}

// Copies the six state planes of every instance flagged in 'tripped' from src to dst (one
// thread per node over the 256-node chunks).
__global__ __launch_bounds__(256) void take_tripped_kernel(const InstDev* __restrict__ inst,
                                                           const int32_t* __restrict__ prefix,
                                                           const int32_t* __restrict__ chunk_inst, int64_t N,
                                                           const uint8_t* __restrict__ tripped,
                                                           const float* __restrict__ src, float* __restrict__ dst) {
  const int t = blockIdx.x;
  const int b = chunk_inst[t];
  if (!tripped[b]) return;
  const InstDev I = inst[b];
  const int local = (t - prefix[b]) * kChunk + (int)threadIdx.x;
  if (local >= I.H * I.W) return;
  const int64_t p = I.off + local;
#pragma unroll
  for (int c = 0; c < 6; ++c) dst[c * N + p] = src[c * N + p];
}

struct RolloutWs {
  float* X;        // third rotating state
  float* Y;        // fourth rotating state (the prefix schedule)
  float* T;        // mass-spring substep temporary
  double* part;    // reduction partials
  double* now;     // [4n] diagnostics of the current check
  double* e0;      // [n] energy at the start
  double* eref;    // [n] energy scale
  double* escale;  // [n] 1 / (nodes width^2) for the frame-error test
  double* stats;   // [4n] used when the caller passes NULL
  uint8_t* active; // [n]
  uint8_t* tripped; // [n] fell back at the current check
  int* count;      // [1]
  size_t bytes;
};

static RolloutWs rollout_layout(const pecnn_plan* plan, void* base) {
  RolloutWs w;
  char* p = (char*)base;
  size_t o = 0;
  const size_t st = align256(6 * (size_t)plan->total * sizeof(float));
  w.X = (float*)(p + o); o += st;
  w.Y = (float*)(p + o); o += st;
  w.T = (float*)(p + o); o += st;
  w.part = (double*)(p + o); o += align256(reduce_ws_bytes(plan));
  w.now = (double*)(p + o); o += align256(4 * (size_t)plan->n * sizeof(double));
  w.e0 = (double*)(p + o); o += align256((size_t)plan->n * sizeof(double));
  w.eref = (double*)(p + o); o += align256((size_t)plan->n * sizeof(double));
  w.escale = (double*)(p + o); o += align256((size_t)plan->n * sizeof(double));
  w.stats = (double*)(p + o); o += align256(4 * (size_t)plan->n * sizeof(double));
  w.active = (uint8_t*)(p + o); o += align256((size_t)plan->n);
  w.tripped = (uint8_t*)(p + o); o += align256((size_t)plan->n);
  w.count = (int*)(p + o); o += 256;
  w.bytes = o;
  return w;
}

}  // namespace pecnn

using namespace pecnn;

extern "C" {

int32_t pecnn_version(void) { return 1; }

const char* pecnn_status_string(int s) {
  switch (s) {
    case PECNN_OK: return "ok";
    case PECNN_E_INVALID: return "invalid argument";
    case PECNN_E_SHAPE: return "inconsistent shape";
    case PECNN_E_UNSUPPORTED: return "unsupported configuration";
    case PECNN_E_WORKSPACE: return "workspace missing or too small";
    case PECNN_E_HIP: return "HIP runtime error";
    default: return "unknown status";
  }
}

const char* pecnn_last_error(void) { return g_err; }

int64_t pecnn_theta_size(int32_t ch) {
  if (ch <= 0 || ch > 64) return -1;
  return (int64_t)ch * 54 + 2 * (int64_t)ch * ch + 9 * (int64_t)ch + 3;
}

int64_t pecnn_cell_theta_size(int32_t cell, int32_t ch) {
  if (cell == PECNN_CELL_PAIR) return ch == 12 ? 51 : -1;
  return cell == PECNN_CELL_CONV ? pecnn_theta_size(ch) : -1;
}

static int check_desc(const pecnn_batch_desc* d) {
  if (!d || !d->H || !d->W || !d->h || !d->mass || !d->a_ext) { set_error("null batch description"); return PECNN_E_INVALID; }
  if (d->n < 1 || d->n > 65536) { set_error("instance count %d out of range", d->n); return PECNN_E_SHAPE; }
  int64_t tot = 0;
  for (int b = 0; b < d->n; ++b) {
    const int64_t hw = (int64_t)d->H[b] * d->W[b];
    if (d->H[b] < 1 || d->W[b] < 1 || hw < 2 || hw >= (1 << 24)) {
      set_error("instance %d: grid %d x %d out of range", b, d->H[b], d->W[b]);
      return PECNN_E_SHAPE;
    }
    if (!finite_pos(d->h[b]) || !finite_pos(d->mass[b]) || !isfinite(d->a_ext[3 * b]) ||
        !isfinite(d->a_ext[3 * b + 1]) || !isfinite(d->a_ext[3 * b + 2])) {
      set_error("instance %d: spacing and mass must be finite and > 0, a_ext finite", b);
      return PECNN_E_INVALID;
    }
    tot += hw;
  }
  if (tot >= ((int64_t)1 << 32) / 24) { set_error("batch too large (%lld nodes)", (long long)tot); return PECNN_E_SHAPE; }
  return PECNN_OK;
}

static void tile_counts(const pecnn_batch_desc* d, std::vector<int64_t>& ntile) {
  ntile.assign(kNumCfg, 0);
  for (int b = 0; b < d->n; ++b) {
    for (int c = 0; c < kNumMsCfg; ++c) ntile[ms_cfg_slot(c)] += tiles_of(d->H[b], d->W[b], kMsCfg[c].tx, kMsCfg[c].ty);
    for (int c = 0; c < kNumCnnCfg; ++c) ntile[cnn_cfg_slot(c)] += tiles_of(d->H[b], d->W[b], kCnnCfg[c].tx, kCnnCfg[c].ty);
    ntile[kCfgChunk] += ((int64_t)d->H[b] * d->W[b] + kChunk - 1) / kChunk;
  }
}

int pecnn_plan_device_bytes(const pecnn_batch_desc* d, size_t* bytes) {
  int rc = check_desc(d);
  if (rc) return rc;
  if (!bytes) { set_error("null bytes"); return PECNN_E_INVALID; }
  std::vector<int64_t> nt;
  tile_counts(d, nt);
  *bytes = align256((size_t)d->n * sizeof(InstDev)) + kNumCfg * align256((size_t)(d->n + 1) * sizeof(int32_t)) +
           align256((size_t)nt[kCfgChunk] * sizeof(int32_t)) + align256((size_t)d->n * kSphereStride * sizeof(float));
  return PECNN_OK;
}

int pecnn_plan_create(const pecnn_batch_desc* d, const uint8_t* pin, void* dev_mem, size_t dev_bytes, void* stream,
                      pecnn_plan** out) {
  int rc = check_desc(d);
  if (rc) return rc;
  if (!pin || !dev_mem || !out) { set_error("null pin, plan memory or output handle"); return PECNN_E_INVALID; }
  size_t need = 0;
  pecnn_plan_device_bytes(d, &need);
  if (dev_bytes < need) { set_error("plan memory %zu < %zu bytes", dev_bytes, need); return PECNN_E_WORKSPACE; }
  std::vector<int64_t> nt;
  tile_counts(d, nt);
  for (int c = 0; c < kNumCfg; ++c)
    if (nt[c] >= ((int64_t)1 << 31)) { set_error("too many tiles"); return PECNN_E_SHAPE; }

  const int n = d->n;
  std::vector<char> host(need, 0);
  InstDev* hi = (InstDev*)host.data();
  int64_t off = 0;
  int max_hw = 0;
  for (int b = 0; b < n; ++b) {
    hi[b].H = d->H[b];
    hi[b].W = d->W[b];
    hi[b].off = off;
    hi[b].h = d->h[b];
    hi[b].mass = d->mass[b];
    hi[b].ax = d->a_ext[3 * b];
    hi[b].ay = d->a_ext[3 * b + 1];
    hi[b].az = d->a_ext[3 * b + 2];
    hi[b].pres = 0.f;
    off += (int64_t)d->H[b] * d->W[b];
    if (d->H[b] * d->W[b] > max_hw) max_hw = d->H[b] * d->W[b];
  }
  size_t o = align256((size_t)n * sizeof(InstDev));
  size_t pre_off[kNumCfg];
  for (int c = 0; c < kNumCfg; ++c) {
    pre_off[c] = o;
    int32_t* pre = (int32_t*)(host.data() + o);
    int32_t acc = 0;
    for (int b = 0; b < n; ++b) {
      pre[b] = acc;
      int tiles;
      if (c < kNumMsCfg) tiles = tiles_of(d->H[b], d->W[b], kMsCfg[c].tx, kMsCfg[c].ty);
      else if (c < kNumMsCfg + kNumCnnCfg) tiles = tiles_of(d->H[b], d->W[b], kCnnCfg[c - kNumMsCfg].tx, kCnnCfg[c - kNumMsCfg].ty);
      else tiles = (int)(((int64_t)d->H[b] * d->W[b] + kChunk - 1) / kChunk);
      acc += tiles;
    }
    pre[n] = acc;
    o += align256((size_t)(n + 1) * sizeof(int32_t));
  }
  // instance of every node chunk (the node-parallel kernels look it up instead of searching)
  const size_t chunk_off = o;
  {
    int32_t* ci = (int32_t*)(host.data() + o);
    int64_t t = 0;
    for (int b = 0; b < n; ++b) {
      const int64_t chunks = ((int64_t)d->H[b] * d->W[b] + kChunk - 1) / kChunk;
      for (int64_t k = 0; k < chunks; ++k) ci[t++] = b;
    }
    o += align256((size_t)nt[kCfgChunk] * sizeof(int32_t));
  }
  // per-instance sphere records (all zero: no sphere)
  const size_t sphere_off = o;
  hipStream_t st = (hipStream_t)stream;
  PECNN_HIP(hipMemcpyAsync(dev_mem, host.data(), need, hipMemcpyHostToDevice, st));
  PECNN_HIP(hipStreamSynchronize(st));

  pecnn_plan* p = (pecnn_plan*)calloc(1, sizeof(pecnn_plan));
  if (!p) { set_error("out of host memory"); return PECNN_E_INVALID; }
  p->n = n;
  p->total = off;
  p->H = (int32_t*)malloc(sizeof(int32_t) * n);
  p->W = (int32_t*)malloc(sizeof(int32_t) * n);
  p->off = (int64_t*)malloc(sizeof(int64_t) * (n + 1));
  p->h = (float*)malloc(sizeof(float) * n);
  p->mass = (float*)malloc(sizeof(float) * n);
  p->a_ext = (float*)malloc(sizeof(float) * 3 * n);
  p->pres = (float*)calloc(n, sizeof(float));
  if (!p->H || !p->W || !p->off || !p->h || !p->mass || !p->a_ext || !p->pres) {
    pecnn_plan_destroy(p);
    set_error("out of host memory");
    return PECNN_E_INVALID;
  }
  for (int b = 0; b < n; ++b) {
    p->H[b] = d->H[b];
    p->W[b] = d->W[b];
    p->off[b] = hi[b].off;
    p->h[b] = d->h[b];
    p->mass[b] = d->mass[b];
    for (int a = 0; a < 3; ++a) p->a_ext[3 * b + a] = d->a_ext[3 * b + a];
  }
  p->off[n] = off;
  p->pin = pin;
  p->d_inst = (InstDev*)dev_mem;
  for (int c = 0; c < kNumCfg; ++c) {
    p->d_prefix[c] = (int32_t*)((char*)dev_mem + pre_off[c]);
    p->n_tiles[c] = (int32_t)nt[c];
  }
  p->d_chunk_inst = (int32_t*)((char*)dev_mem + chunk_off);
  p->d_sphere = (float*)((char*)dev_mem + sphere_off);
  // defaults: wide rows for large instances, square tiles when most instances are small
  p->ms_cfg = max_hw >= 64 * 64 ? 3 : 2;
  p->cnn_cfg = max_hw >= 64 * 64 ? 0 : 2;
  p->max_hw = max_hw;
  p->vec4 = (off % 4) == 0;
  for (int b = 0; b < n; ++b)
    if (p->W[b] % 4 != 0 || p->off[b] % 4 != 0) p->vec4 = 0;
  p->graph_cache = nullptr;
  // set-up of the allocation-free diagnostics on this device; a failure here is reported by
  // cloth_reduce_fp64_noalloc, which looks the address up again
  if (reduce_scratch(nullptr) != PECNN_OK) set_error("");
  *out = p;
  return PECNN_OK;
}

int pecnn_plan_destroy(pecnn_plan* p) {
  if (!p) return PECNN_OK;
  graph_cache_free(p);
  free(p->H);
  free(p->W);
  free(p->off);
  free(p->h);
  free(p->mass);
  free(p->a_ext);
  free(p->pres);
  free(p);
  return PECNN_OK;
}

int pecnn_plan_set_spheres(pecnn_plan* p, const float* sphere, void* stream) {
  if (check_plan(p)) return PECNN_E_INVALID;
  if (!sphere) { set_error("null sphere records"); return PECNN_E_INVALID; }
  std::vector<float> rec((size_t)p->n * kSphereStride, 0.f);
  int any = 0;
  for (int b = 0; b < p->n; ++b) {
    const float* r = sphere + 5 * (size_t)b;
    if (!isfinite(r[0]) || !isfinite(r[1]) || !isfinite(r[2]) || !isfinite(r[3]) || r[3] < 0.f || !(r[4] >= 0.f && r[4] <= 1.f)) {
      set_error("instance %d: sphere centre finite, radius >= 0, friction in [0, 1]", b);
      return PECNN_E_INVALID;
    }
    for (int k = 0; k < 5; ++k) rec[(size_t)b * kSphereStride + k] = r[k];
    any |= r[3] > 0.f;
  }
  hipStream_t st = (hipStream_t)stream;
  PECNN_HIP(hipMemcpyAsync(p->d_sphere, rec.data(), rec.size() * sizeof(float), hipMemcpyHostToDevice, st));
  PECNN_HIP(hipStreamSynchronize(st));
  const int ext_before = p->has_pressure || p->has_sphere;
  p->has_sphere = any;
  if ((p->has_pressure || p->has_sphere) != ext_before) graph_cache_free(p);
  return PECNN_OK;
}

int pecnn_plan_set_pressure(pecnn_plan* p, const float* pressure, void* stream) {
  if (check_plan(p)) return PECNN_E_INVALID;
  if (!pressure) { set_error("null pressure"); return PECNN_E_INVALID; }
  for (int b = 0; b < p->n; ++b)
    if (!isfinite(pressure[b])) { set_error("instance %d: pressure must be finite", b); return PECNN_E_INVALID; }
  // rebuild the instance records from the host copies and replace them in the plan memory
  std::vector<InstDev> hi(p->n);
  int any = 0;
  for (int b = 0; b < p->n; ++b) {
    hi[b].H = p->H[b];
    hi[b].W = p->W[b];
    hi[b].off = p->off[b];
    hi[b].h = p->h[b];
    hi[b].mass = p->mass[b];
    hi[b].ax = p->a_ext[3 * b];
    hi[b].ay = p->a_ext[3 * b + 1];
    hi[b].az = p->a_ext[3 * b + 2];
    hi[b].pres = pressure[b];
    any |= pressure[b] != 0.f;
  }
  hipStream_t st = (hipStream_t)stream;
  PECNN_HIP(hipMemcpyAsync(p->d_inst, hi.data(), sizeof(InstDev) * p->n, hipMemcpyHostToDevice, st));
  PECNN_HIP(hipStreamSynchronize(st));
  for (int b = 0; b < p->n; ++b) p->pres[b] = pressure[b];
  // captured chunks hold the kernel variants of the old setting
  if ((any || p->has_sphere) != (p->has_pressure || p->has_sphere)) graph_cache_free(p);
  p->has_pressure = any;
  return PECNN_OK;
}

int64_t pecnn_plan_nodes(const pecnn_plan* p) { return p ? p->total : -1; }

int pecnn_plan_set_tiles(pecnn_plan* p, int32_t ms_cfg, int32_t cnn_cfg) {
  if (check_plan(p)) return PECNN_E_INVALID;
  if (ms_cfg < -1 || ms_cfg >= kNumMsCfg || cnn_cfg < -1 || cnn_cfg >= kNumCnnCfg) {
    set_error("tile configuration out of range");
    return PECNN_E_INVALID;
  }
  if (ms_cfg >= 0) p->ms_cfg = ms_cfg;
  if (cnn_cfg >= 0) p->cnn_cfg = cnn_cfg;
  return PECNN_OK;
}

int pecnn_plan_get_tiles(const pecnn_plan* p, int32_t* ms_cfg, int32_t* cnn_cfg) {
  if (check_plan(p) || !ms_cfg || !cnn_cfg) { set_error("null argument"); return PECNN_E_INVALID; }
  *ms_cfg = p->ms_cfg;
  *cnn_cfg = p->cnn_cfg;
  return PECNN_OK;
}

// Backward workspace: the reverse pass's own part, then, when some instance has a sphere, the
// frame without spheres, the rewritten output adjoint and zeroed sphere records.
static size_t backward_ws_base(const pecnn_plan* p, const pecnn_model* m) {
  return align256(m->cell == PECNN_CELL_PAIR ? pair_backward_ws_bytes(p) : backward_ws_bytes(p, m->ch));
}

static size_t backward_ws_total(const pecnn_plan* p, const pecnn_model* m) {
  size_t b = backward_ws_base(p, m);
  if (p->has_sphere)
    b += 2 * align256(6 * (size_t)p->total * sizeof(float)) + align256((size_t)p->n * kSphereStride * sizeof(float));
  return b;
}

int pecnn_workspace_bytes(const pecnn_plan* p, const pecnn_model* m, int32_t which, size_t* bytes) {
  if (check_plan(p) || !bytes) { set_error("null plan or bytes"); return PECNN_E_INVALID; }
  switch (which) {
    case PECNN_WS_MS_STEP: *bytes = align256(6 * (size_t)p->total * sizeof(float)); return PECNN_OK;
    case PECNN_WS_REDUCE: *bytes = align256(reduce_ws_bytes(p)); return PECNN_OK;
    case PECNN_WS_BACKWARD: {
      int rc = check_model(m);
      if (rc) return rc;
      *bytes = backward_ws_total(p, m);
      return PECNN_OK;
    }
    case PECNN_WS_ROLLOUT: *bytes = rollout_layout(p, nullptr).bytes; return PECNN_OK;
    default: set_error("unknown workspace kind %d", which); return PECNN_E_INVALID;
  }
}

int cloth_ms_step(const pecnn_plan* p, const cloth_ms_params* prm, const float* s_in, float* s_out, int32_t n_steps,
                  const uint8_t* active, void* ws, size_t ws_bytes, void* stream) {
  int rc = check_plan(p);
  if (rc) return rc;
  if ((rc = check_ms_params(prm))) return rc;
  if (!s_in || !s_out) { set_error("null state"); return PECNN_E_INVALID; }
  if (n_steps < 1) { set_error("n_steps must be >= 1"); return PECNN_E_INVALID; }
  const size_t sb = 6 * (size_t)p->total * sizeof(float);
  const char *a = (const char*)s_in, *b = (const char*)s_out;
  if (a < b + sb && b < a + sb) { set_error("s_in and s_out overlap"); return PECNN_E_INVALID; }
  if (n_steps > 1) {
    if (!ws || ws_bytes < sb) { set_error("workspace of %zu bytes needed for n_steps > 1", sb); return PECNN_E_WORKSPACE; }
    const char* w = (const char*)ws;
    if ((w < a + sb && a < w + sb) || (w < b + sb && b < w + sb)) { set_error("workspace overlaps a state"); return PECNN_E_INVALID; }
  }
  return ms_step_run(p, p->ms_cfg, ms_params_dev(prm), s_in, s_out, (float*)ws, n_steps, active, (hipStream_t)stream);
}

int pecnn_forward(const pecnn_plan* p, const pecnn_model* m, const float* s_prev, const float* s_cur, float* s_next,
                  void* stream) {
  int rc = check_plan(p);
  if (rc) return rc;
  if ((rc = check_model(m))) return rc;
  if (!s_prev || !s_cur || !s_next) { set_error("null state"); return PECNN_E_INVALID; }
  const size_t sb = 6 * (size_t)p->total * sizeof(float);
  const char *a = (const char*)s_prev, *c = (const char*)s_cur, *n = (const char*)s_next;
  if ((n < a + sb && a < n + sb) || (n < c + sb && c < n + sb)) { set_error("s_next overlaps an input"); return PECNN_E_INVALID; }
  return cnn_forward_launch(p, p->cnn_cfg, m, s_prev, s_cur, s_next, nullptr, (hipStream_t)stream);
}

int pecnn_backward(const pecnn_plan* p, const pecnn_model* m, const float* s_prev, const float* s_cur,
                   const float* g_next, float* g_cur, float* g_prev, float* g_theta, void* ws, size_t ws_bytes,
                   void* stream) {
  TraceRange tr("pecnn_backward");
  int rc = check_plan(p);
  if (rc) return rc;
  if ((rc = check_model(m))) return rc;
  if (m->precision != PECNN_FP32) { set_error("backward needs an FP32 model"); return PECNN_E_UNSUPPORTED; }
  if (!s_prev || !s_cur || !g_next || !g_theta) { set_error("null state, gradient or theta gradient"); return PECNN_E_INVALID; }
  if (g_cur && g_prev && g_cur == g_prev) { set_error("g_cur and g_prev must differ"); return PECNN_E_INVALID; }
  const size_t need = backward_ws_total(p, m);
  if (!ws || ws_bytes < need) { set_error("backward workspace of %zu bytes needed", need); return PECNN_E_WORKSPACE; }
  hipStream_t st = (hipStream_t)stream;
  if (p->has_sphere) {
    // The frame without spheres gives the velocities before the constraint; the sphere's
    // reverse mode then rewrites g_next for the constraint-free reverse pass below.
    const size_t sb = align256(6 * (size_t)p->total * sizeof(float));
    char* e = (char*)ws + backward_ws_base(p, m);
    float* vfree = (float*)e;
    float* g_sph = (float*)(e + sb);
    float* no_sphere = (float*)(e + 2 * sb);
    rc = zero_floats_launch(no_sphere, (int64_t)p->n * kSphereStride, st);
    if (rc) return rc;
    pecnn_plan q = *p;
    q.d_sphere = no_sphere;
    q.has_sphere = 0;
    rc = cnn_forward_launch(&q, q.cnn_cfg, m, s_prev, s_cur, vfree, nullptr, st);
    if (rc) return rc;
    rc = sphere_adjoint_launch(p, m->dt, s_cur, vfree, g_next, g_sph, st);
    if (rc) return rc;
    g_next = g_sph;
  }
  if (m->cell == PECNN_CELL_PAIR)  // the pair cell does not read S^{k-1}: g_prev gets nothing
    return pair_backward_launch(p, m, s_cur, g_next, g_cur, g_theta, ws, st);
  return backward_launch(p, m, s_prev, s_cur, g_next, g_cur, g_prev, g_theta, ws, st);
}

int cloth_reduce_fp64(const pecnn_plan* p, const cloth_ms_params* prm, const float* s, const float* s_ref, double* out,
                      void* ws, size_t ws_bytes, void* stream) {
  int rc = check_plan(p);
  if (rc) return rc;
  if ((rc = check_ms_params(prm))) return rc;
  if (!s || !out) { set_error("null state or output"); return PECNN_E_INVALID; }
  if (!ws || ws_bytes < reduce_ws_bytes(p)) { set_error("reduce workspace too small"); return PECNN_E_WORKSPACE; }
  return reduce_launch(p, ms_params_dev(prm), s, s_ref, out, ws, (hipStream_t)stream);
}

int cloth_reduce_fp64_noalloc(const pecnn_plan* p, const cloth_ms_params* prm, const float* s, const float* s_ref,
                              double* out, void* stream) {
  int rc = check_plan(p);
  if (rc) return rc;
  if ((rc = check_ms_params(prm))) return rc;
  if (!s || !out) { set_error("null state or output"); return PECNN_E_INVALID; }
  const int chunks = p->n_tiles[kCfgChunk];
  if (chunks > PECNN_NOALLOC_REDUCE_MAX_CHUNKS) {
    set_error("the plan has %d node chunks; the allocation-free reduction holds partials for at most %d", chunks,
              PECNN_NOALLOC_REDUCE_MAX_CHUNKS);
    return PECNN_E_WORKSPACE;
  }
  double* part = nullptr;
  if ((rc = reduce_scratch(&part))) return rc;
  return reduce_launch(p, ms_params_dev(prm), s, s_ref, out, part, (hipStream_t)stream);
}

int pecnn_loss_mse(const pecnn_plan* p, const float* s_hat, const float* s_true, float sx, float sv, float w,
                   int64_t n_free, double* loss, float* g_hat, void* ws, size_t ws_bytes, void* stream) {
  int rc = check_plan(p);
  if (rc) return rc;
  if (!s_hat || !s_true || (!loss && !g_hat)) {
    set_error("null state, or neither loss nor gradient");
    return PECNN_E_INVALID;
  }
  if (!finite_pos(sx) || !finite_pos(sv) || !isfinite(w) || n_free < 1) {
    set_error("scales must be finite and > 0, weight finite, n_free >= 1");
    return PECNN_E_INVALID;
  }
  if (!ws || ws_bytes < reduce_ws_bytes(p)) { set_error("loss workspace too small"); return PECNN_E_WORKSPACE; }
  return loss_launch(p, s_hat, s_true, sx, sv, w, n_free, loss, g_hat, ws, (hipStream_t)stream);
}

int pecnn_adam_step(int64_t n, float lr, float b1, float b2, float eps, int32_t t, float* th, float* m, float* v,
                    const float* g, void* stream) {
  if (!th || !m || !v || !g || n < 1) { set_error("null buffer or n < 1"); return PECNN_E_INVALID; }
  if (!finite_pos(lr) || !(b1 >= 0.f && b1 < 1.f) || !(b2 >= 0.f && b2 < 1.f) || !finite_pos(eps) || t < 1) {
    set_error("Adam: lr, eps > 0, betas in [0, 1), t >= 1");
    return PECNN_E_INVALID;
  }
  return adam_launch(n, lr, b1, b2, eps, t, th, m, v, g, (hipStream_t)stream);
}

int pecnn_gather_windows(const float* traj, int64_t traj_nodes, int32_t n_saved, const int64_t* traj_off,
                         int32_t n_traj, const int32_t* traj_inst, const int32_t* frame_idx, int32_t n_win,
                         int32_t npw, int32_t n_frames, float* out, void* stream) {
  if (!traj || !traj_off || !traj_inst || !frame_idx || !out) { set_error("null buffer"); return PECNN_E_INVALID; }
  if (traj_nodes < 1 || n_saved < 1 || n_traj < 1 || n_win < 1 || npw < 1 || n_frames < 1 || n_win > 65535 ||
      n_frames * 6 > 65535) {
    set_error("gather sizes out of range");
    return PECNN_E_SHAPE;
  }
  return gather_launch(traj, traj_nodes, n_saved, traj_off, n_traj, traj_inst, frame_idx, n_win, npw, n_frames, out,
                       (hipStream_t)stream);
}

// ---------------------------------------------------------------- rollout
// The rollout rotates four device states: the caller's s_prev and s_cur (indices 0 and 1) and
// X, Y in the workspace (2 and 3). Frame k reads S^{k-1}, S^k and writes S^{k+1} into a state
// holding neither. The three-state cycle (write the one of 0, 1, 2 not read) returns S^{n-1},
// S^n to indices 0, 1 every 3 frames, the four-state cycle 2, 3, 0, 1 every 4, so a call of
// n = 3i + 4j frames starts with j four-state cycles and needs no copy at the end (every n but
// 1, 2 and 5).
static int rollout_prefix(int n) {
  if (n % 3 == 1 && n >= 4) return 4;
  if (n % 3 == 2 && n >= 8) return 8;
  return 0;
}
static int rollout_dest(int k, int prefix, int pi, int ci) {
  static const int c4[4] = {2, 3, 0, 1};
  return k < prefix ? c4[k & 3] : 3 - pi - ci;
}

// Record the network steps of one chunk (frames k0 .. k0 + len - 1 of the call, starting from
// states pi, ci) and the guard check that ends it, on 'st'. With the frame-error test on, the
// simulator's answer for the chunk's last frame is written into the state the next frame would
// write, which holds nothing the rollout still needs.
static int record_chunk(pecnn_plan* p, const pecnn_model* m, const MsParamsDev& sim, const pecnn_guard* g,
                        float* const B[4], int pi, int ci, int k0, int prefix, float* T, int len, bool with_ms,
                        bool guard_on, int32_t* fallback, double* stats, const RolloutWs& w, hipStream_t st) {
  for (int k = k0; k < k0 + len; ++k) {
    const int di = rollout_dest(k, prefix, pi, ci);
    int rc = cnn_forward_launch(p, p->cnn_cfg, m, B[pi], B[ci], B[di], fallback, st);
    if (rc) return rc;
    if (with_ms) {
      rc = ms_step_run(p, p->ms_cfg, sim, B[ci], B[di], T, g->substeps, w.active, st);
      if (rc) return rc;
    }
    pi = ci;
    ci = di;
  }
  if (guard_on) {
    float* P = B[pi];
    float* C = B[ci];
    float* X = B[rollout_dest(k0 + len, prefix, pi, ci)];
    const bool ferr = g->frame_err_max > 0.f;
    if (ferr) {
      int rc = ms_step_run(p, p->ms_cfg, sim, P, X, T, g->substeps, nullptr, st);
      if (rc) return rc;
    }
    int rc = reduce_launch(p, sim, C, ferr ? X : nullptr, w.now, w.part, st);
    if (rc) return rc;
    hipLaunchKernelGGL(guard_kernel, dim3(1), dim3(256), 0, st, p->n, w.now, w.e0, w.eref, w.escale, *g, 0, len,
                       fallback, w.active, w.tripped, stats, w.count);
    PECNN_LAUNCH_CHECK("guard_kernel");
    if (ferr) {  // an instance that fell back here takes the simulator's frame instead of the network's
      hipLaunchKernelGGL(take_tripped_kernel, dim3(p->n_tiles[kCfgChunk]), dim3(256), 0, st, p->d_inst,
                         p->d_prefix[kCfgChunk], p->d_chunk_inst, p->total, w.tripped, X, C);
      PECNN_LAUNCH_CHECK("take_tripped_kernel");
    }
  }
  return PECNN_OK;
}

// Repair of a chunk that ran without the mass-spring steps although instances had fallen back at
// the check before it (see pecnn_rollout): the frame kernels skipped those instances, so their
// frames are computed here by the mass-spring steps alone, in the chunk's buffer order; then the
// diagnostics of the chunk's own check are taken again for every instance. The instances that
// tripped at that check itself ran the network through the chunk and are left alone.
static int repair_chunk(pecnn_plan* p, const MsParamsDev& sim, const pecnn_guard* g, float* const B[4], int pi,
                        int ci, int k0, int prefix, float* T, int len, bool guard_on, int32_t* fallback,
                        double* stats, const RolloutWs& w, hipStream_t st) {
  hipLaunchKernelGGL(late_mask_kernel, dim3(1), dim3(256), 0, st, p->n, fallback, w.tripped, w.active);
  PECNN_LAUNCH_CHECK("late_mask_kernel");
  for (int k = k0; k < k0 + len; ++k) {
    const int di = rollout_dest(k, prefix, pi, ci);
    int rc = ms_step_run(p, p->ms_cfg, sim, B[ci], B[di], T, g->substeps, w.active, st);
    if (rc) return rc;
    pi = ci;
    ci = di;
  }
  if (guard_on) {
    int rc = reduce_launch(p, sim, B[ci], nullptr, w.now, w.part, st);
    if (rc) return rc;
    hipLaunchKernelGGL(guard_kernel, dim3(1), dim3(256), 0, st, p->n, w.now, w.e0, w.eref, w.escale, *g, 2, len,
                       fallback, w.active, w.tripped, stats, w.count);
    PECNN_LAUNCH_CHECK("guard_kernel");
  }
  return PECNN_OK;
}

int pecnn_rollout(pecnn_plan* p, const pecnn_model* m, const cloth_ms_params* simp, const pecnn_guard* g,
                  float* s_prev, float* s_cur, int32_t n_steps, int32_t* fallback, double* stats, void* ws,
                  size_t ws_bytes, void* stream) {
  TraceRange tr("pecnn_rollout");
  int rc = check_plan(p);
  if (rc) return rc;
  if ((rc = check_model(m))) return rc;
  if ((rc = check_ms_params(simp))) return rc;
  if (!g || !s_prev || !s_cur || !fallback) { set_error("null guard, state or fallback flags"); return PECNN_E_INVALID; }
  if (n_steps < 0) { set_error("n_steps must be >= 0"); return PECNN_E_INVALID; }
  if (g->substeps < 1 || g->substeps > 1000) { set_error("guard substeps must be in [1, 1000]"); return PECNN_E_INVALID; }
  if (g->check_every > 0 && (!(g->stretch_max > 0.f) || isnan(g->energy_gain_max) || isnan(g->frame_err_max))) {
    set_error("guard bounds must be > 0 / not NaN");
    return PECNN_E_INVALID;
  }
  const size_t sb = 6 * (size_t)p->total * sizeof(float);
  if (s_prev == s_cur || ((const char*)s_prev < (const char*)s_cur + sb && (const char*)s_cur < (const char*)s_prev + sb)) {
    set_error("s_prev and s_cur overlap");
    return PECNN_E_INVALID;
  }
  const RolloutWs w = rollout_layout(p, ws);
  if (!ws || ws_bytes < w.bytes) { set_error("rollout workspace of %zu bytes needed", w.bytes); return PECNN_E_WORKSPACE; }
  hipStream_t st = (hipStream_t)stream;
  if (n_steps == 0) return PECNN_OK;
  const MsParamsDev sim = ms_params_dev(simp);
  double* stats_d = stats ? stats : w.stats;
  const bool guard_on = g->check_every > 0;

  GraphCache* gc = (GraphCache*)p->graph_cache;
  if (!gc) {
    gc = new GraphCache();
    p->graph_cache = gc;
    PECNN_HIP(hipStreamCreateWithFlags(&gc->capture, hipStreamNonBlocking));
    PECNN_HIP(hipHostMalloc((void**)&gc->host_count, 2 * sizeof(int), hipHostMallocDefault));
    for (hipEvent_t& e : gc->count_ready) PECNN_HIP(hipEventCreateWithFlags(&e, hipEventDisableTiming));
  }

  // prologue: energy scale, starting diagnostics, fall-back mask
  {
    TraceRange tp("pecnn_rollout prologue");
    std::vector<double> eref(p->n), escale(p->n);
    const double gn = sqrt((double)simp->g[0] * simp->g[0] + (double)simp->g[1] * simp->g[1] + (double)simp->g[2] * simp->g[2]);
    for (int b = 0; b < p->n; ++b) {
      double e = (double)p->H[b] * p->W[b] * p->mass[b] * (gn > 0 ? gn : 1.0) * (p->W[b] > 1 ? p->W[b] - 1 : 1) * p->h[b];
      eref[b] = e > 0 ? e : 1.0;
      // pressure does work on the cloth, so its energy may rise: the energy check is off there
      if (p->pres[b] != 0.f) eref[b] = INFINITY;
      const double width = (double)(p->W[b] > 1 ? p->W[b] - 1 : 1) * p->h[b];
      escale[b] = 1.0 / ((double)p->H[b] * p->W[b] * width * width);
    }
    PECNN_HIP(hipMemcpyAsync(w.eref, eref.data(), sizeof(double) * p->n, hipMemcpyHostToDevice, st));
    PECNN_HIP(hipMemcpyAsync(w.escale, escale.data(), sizeof(double) * p->n, hipMemcpyHostToDevice, st));
    rc = reduce_launch(p, sim, s_cur, nullptr, w.now, w.part, st);
    if (rc) return rc;
    hipLaunchKernelGGL(guard_kernel, dim3(1), dim3(256), 0, st, p->n, w.now, w.e0, w.eref, w.escale, *g, 1, 0,
                       fallback, w.active, w.tripped, stats_d, w.count);
    PECNN_LAUNCH_CHECK("guard_kernel");
    PECNN_HIP(hipMemcpyAsync(&gc->host_count[0], w.count, sizeof(int), hipMemcpyDeviceToHost, st));
    PECNN_HIP(hipEventRecord(gc->count_ready[0], st));
    PECNN_HIP(hipEventSynchronize(gc->count_ready[0]));
  }

  float* const B[4] = {s_prev, s_cur, w.X, w.Y};
  const int prefix = rollout_prefix(n_steps);
  int pi = 0, ci = 1;
  int k = 0;
  const int chunk = guard_on ? g->check_every : n_steps;
  // The host runs one chunk ahead of the fall-back count it has read: after the first chunk
  // (decided by the prologue's count), a chunk is launched with or without the mass-spring steps
  // of fallen instances according to the last count known on the host, and the count of the
  // check before it is read only after the launch, so the GPU does not wait for the host. If
  // that count shows the first instances fallen while the chunk was launched without the
  // mass-spring steps, the chunk skipped them (the frame kernels skip fallen instances), and
  // repair_chunk computes their frames.
  bool any_fallen = gc->host_count[0] > 0;  // last count read on the host was nonzero
  int pending = -1;                          // host slot of a count not yet read
  int nchunk = 0;
  while (k < n_steps) {
    const int len = chunk < n_steps - k ? chunk : n_steps - k;
    const bool with_ms = any_fallen;
    GraphKey key;
    memset(&key, 0, sizeof(key));
    key.buf[0] = s_prev; key.buf[1] = s_cur; key.pi = pi; key.ci = ci;
    for (int i = 0; i < len && k + i < prefix; ++i) {
      key.pre_len = i + 1;
      key.pre_code |= rollout_dest(k + i, prefix, 0, 0) << (2 * i);
    }
    key.len = len; key.with_ms = with_ms; key.guard = guard_on; key.ms_cfg = p->ms_cfg; key.cnn_cfg = p->cnn_cfg;
    key.ch = m->ch; key.prec = m->precision; key.cell = m->cell; key.substeps = g->substeps; key.dt = m->dt; key.alpha = m->isru_alpha;
    key.theta = m->theta; key.sim = *simp; key.gd = *g; key.fallback = fallback; key.ws = ws;
    key.stats = stats_d;
    hipGraphExec_t exec = nullptr;
    for (auto& e : gc->entries)
      if (e.key == key) { exec = e.exec; break; }
    if (!exec) {
      hipGraph_t graph;
      PECNN_HIP(hipStreamBeginCapture(gc->capture, hipStreamCaptureModeThreadLocal));
      rc = record_chunk(p, m, sim, g, B, pi, ci, k, prefix, w.T, len, with_ms, guard_on, fallback, stats_d, w,
                        gc->capture);
      hipError_t e2 = hipStreamEndCapture(gc->capture, &graph);
      if (rc) {
        if (e2 == hipSuccess) (void)hipGraphDestroy(graph);
        return rc;
      }
      if (e2 != hipSuccess) return hip_fail(e2, "hipStreamEndCapture");
      hipError_t e3 = hipGraphInstantiate(&exec, graph, nullptr, nullptr, 0);
      (void)hipGraphDestroy(graph);
      if (e3 != hipSuccess) return hip_fail(e3, "hipGraphInstantiate");
      if (gc->entries.size() >= 24) {
        (void)hipGraphExecDestroy(gc->entries.front().exec);
        gc->entries.erase(gc->entries.begin());
      }
      gc->entries.push_back(GraphEntry{key, exec});
    }
    {
      TraceRange tc(with_ms ? "pecnn_rollout chunk (with mass-spring steps)" : "pecnn_rollout chunk");
      PECNN_HIP(hipGraphLaunch(exec, st));
    }
    const int k0 = k, pi0 = pi, ci0 = ci;
    for (int i = 0; i < len; ++i) {
      const int di = rollout_dest(k + i, prefix, pi, ci);
      pi = ci;
      ci = di;
    }
    k += len;
    int next = -1;
    if (guard_on && k < n_steps) {  // this chunk's count, read after the next chunk's launch
      next = nchunk & 1;
      PECNN_HIP(hipMemcpyAsync(&gc->host_count[next], w.count, sizeof(int), hipMemcpyDeviceToHost, st));
      PECNN_HIP(hipEventRecord(gc->count_ready[next], st));
    }
    if (pending >= 0) {  // the previous chunk's count
      PECNN_HIP(hipEventSynchronize(gc->count_ready[pending]));
      const bool fallen = gc->host_count[pending] > 0;
      if (fallen && !with_ms) {
        TraceRange trp("pecnn_rollout repair");
        rc = repair_chunk(p, sim, g, B, pi0, ci0, k0, prefix, w.T, len, guard_on, fallback, stats_d, w, st);
        if (rc) return rc;
      }
      any_fallen = any_fallen || fallen;
    }
    pending = next;
    ++nchunk;
  }
  // hand the last two states back in the caller's buffers (only n = 1, 2, 5 end elsewhere; the
  // three-state cycle then leaves them at (1, 2) or (2, 0))
  if (pi != 0 || ci != 1) {
    if (pi == 1) {  // (s_cur, X)
      PECNN_HIP(hipMemcpyAsync(s_prev, s_cur, sb, hipMemcpyDeviceToDevice, st));
      PECNN_HIP(hipMemcpyAsync(s_cur, B[ci], sb, hipMemcpyDeviceToDevice, st));
    } else {  // (X, s_prev)
      PECNN_HIP(hipMemcpyAsync(s_cur, s_prev, sb, hipMemcpyDeviceToDevice, st));
      PECNN_HIP(hipMemcpyAsync(s_prev, B[pi], sb, hipMemcpyDeviceToDevice, st));
    }
  }
  return PECNN_OK;
}

// ---------------------------------------------------------------- autotuner
static int time_launches(hipStream_t st, hipEvent_t e0, hipEvent_t e1, int reps, float* out_ms,
                         const std::function<int(int)>& launch) {
  int rc = launch(0);  // warm-up
  if (rc) return rc;
  PECNN_HIP(hipEventRecord(e0, st));
  for (int r = 0; r < reps; ++r)
    if ((rc = launch(r))) return rc;
  PECNN_HIP(hipEventRecord(e1, st));
  PECNN_HIP(hipEventSynchronize(e1));
  float t = 0.f;
  PECNN_HIP(hipEventElapsedTime(&t, e0, e1));
  *out_ms = t / reps;
  return PECNN_OK;
}

// The configurations are timed in interleaved rounds (each round times every configuration
// once) and each keeps its best round: the chip's clock ramps for a few hundred milliseconds under
// a new load, and configurations timed one after another would favour the later ones.
constexpr int kTuneRounds = 3;

static int autotune_impl(pecnn_plan* p, const cloth_ms_params* prm, const pecnn_model* m, float* s_a, float* s_b,
                         float* s_c, int reps, float* ms_ms, float* cnn_ms, hipStream_t st, hipEvent_t e0,
                         hipEvent_t e1) {
  const MsParamsDev P = ms_params_dev(prm);
  float ms_t[kNumMsCfg], cnn_t[kNumCnnCfg];
  for (int c = 0; c < kNumMsCfg; ++c) ms_t[c] = 1e30f;
  for (int c = 0; c < kNumCnnCfg; ++c) cnn_t[c] = 1e30f;
  float* bs[3] = {s_a, s_b, s_c};
  for (int round = 0; round < kTuneRounds; ++round) {
    for (int c = 0; c < kNumMsCfg; ++c) {
      float t = 0.f;
      int rc = time_launches(st, e0, e1, reps, &t, [&](int r) {
        return ms_step_once(p, c, P, (r & 1) ? s_b : s_a, (r & 1) ? s_a : s_b, nullptr, st);
      });
      if (rc) return rc;
      ms_t[c] = std::min(ms_t[c], t);
    }
    if (!m) continue;
    for (int c = 0; c < kNumCnnCfg; ++c) {
      float t = 0.f;
      int rc = time_launches(st, e0, e1, reps, &t, [&](int r) {
        return cnn_forward_launch(p, c, m, bs[r % 3], bs[(r + 1) % 3], bs[(r + 2) % 3], nullptr, st);
      });
      if (rc) return rc;
      cnn_t[c] = std::min(cnn_t[c], t);
    }
  }
  int best = 0;
  for (int c = 0; c < kNumMsCfg; ++c) {
    if (ms_ms) ms_ms[c] = ms_t[c];
    if (ms_t[c] < ms_t[best]) best = c;
  }
  p->ms_cfg = best;
  if (!m) return PECNN_OK;
  best = 0;
  for (int c = 0; c < kNumCnnCfg; ++c) {
    if (cnn_ms) cnn_ms[c] = cnn_t[c];
    if (cnn_t[c] < cnn_t[best]) best = c;
  }
  p->cnn_cfg = best;
  return PECNN_OK;
}

int pecnn_autotune(pecnn_plan* p, const cloth_ms_params* prm, const pecnn_model* m, float* s_a, float* s_b,
                   float* s_c, int32_t reps, float* ms_ms, float* cnn_ms, void* stream) {
  TraceRange tr("pecnn_autotune");
  int rc = check_plan(p);
  if (rc) return rc;
  if ((rc = check_ms_params(prm))) return rc;
  if (m && (rc = check_model(m))) return rc;
  if (!s_a || !s_b || !s_c || reps < 1) { set_error("null scratch state or reps < 1"); return PECNN_E_INVALID; }
  hipEvent_t e0, e1;
  PECNN_HIP(hipEventCreate(&e0));
  hipError_t e = hipEventCreate(&e1);
  if (e != hipSuccess) {
    (void)hipEventDestroy(e0);
    return hip_fail(e, "hipEventCreate");
  }
  rc = autotune_impl(p, prm, m, s_a, s_b, s_c, reps, ms_ms, cnn_ms, (hipStream_t)stream, e0, e1);
  (void)hipEventDestroy(e0);
  (void)hipEventDestroy(e1);
  return rc;
}

}  // extern "C"
