/*
 * pecnn — MI355X (gfx950) library for the physics-embedded CNN cloth method of
 * Zhao, "A Physics-embedded Deep Learning Framework for Cloth Simulation" (arXiv 2403.12820).
 *
 * C ABI. Plain pointers and sizes only. "device" means HIP device memory of the current
 * device, "host" means ordinary CPU memory. All calls are asynchronous on the given HIP
 * stream (passed as void*, a hipStream_t; NULL = the default stream) unless stated.
 *
 * State layout (all entry points): a batch of cloth instances, each a regular grid of
 * H x W mass points (node p = i*W + j, row i = 0 is the "top" edge), concatenated along
 * the node axis (instance b owns nodes [off_b, off_b + H_b*W_b)). A state is six FP32
 * planes of N_total floats each: x0 x1 x2 (position, m) v0 v1 v2 (velocity, m/s);
 * plane c starts at c*N_total.
 *
 * Ownership: the caller allocates and frees every buffer (state, gradients, parameters,
 * workspaces, plan memory). The library never allocates device memory at run time; its one
 * fixed device array (4 MiB per device, for cloth_reduce_fp64_noalloc) is part of the loaded
 * code object. Host memory is
 * allocated only for plan handles (pecnn_plan_create / pecnn_plan_destroy) and the
 * rollout's graph cache inside a plan (its graphs, a capture stream and one pinned int).
 *
 * Threads: entry points that take a const plan may run concurrently from several host threads
 * (with distinct outputs and workspaces). pecnn_rollout, pecnn_autotune, pecnn_plan_set_* and
 * pecnn_plan_destroy change the plan (its tile choice, records or graph cache): the caller
 * serialises them against every other call on the same plan.
 *
 * Errors: every entry point validates its arguments before any launch and returns a
 * negative pecnn_status with no side effect on invalid input. A failed HIP call returns
 * PECNN_E_HIP; pecnn_last_error() gives a message (thread-local). Kernel faults surface at
 * the caller's next synchronisation. No C++ exception crosses this boundary.
 */
#ifndef PECNN_H
#define PECNN_H

#include <stddef.h>
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

typedef enum {
  PECNN_OK = 0,
  PECNN_E_INVALID = -1,     /* null pointer, non-finite or out-of-range scalar */
  PECNN_E_SHAPE = -2,       /* grid sizes or buffer sizes inconsistent */
  PECNN_E_UNSUPPORTED = -3, /* channel count or precision not supported */
  PECNN_E_WORKSPACE = -4,   /* workspace missing or too small */
  PECNN_E_HIP = -5          /* a HIP runtime call failed */
} pecnn_status;

/* ------------------------------------------------------------------ batch and plan */

/* Host description of a batch of cloths. All arrays are host memory of length n (a_ext: 3n),
   read during pecnn_plan_create only. */
typedef struct {
  int32_t n;              /* number of instances, 1 .. 65536 */
  const int32_t* H;       /* rows per instance, >= 1 */
  const int32_t* W;       /* columns per instance, >= 1; H*W >= 2 and H*W < 2^24; total nodes
                             N_total < 2^32 / 24 (a state stays below 4 GiB) */
  const float* h;         /* rest spacing of the grid (m), > 0: rest lengths h, sqrt(2)h, 2h */
  const float* mass;      /* node mass (kg), > 0 (section 3.1: mass points) */
  const float* a_ext;     /* constant external acceleration per instance (wind), [n][3] */
} pecnn_batch_desc;

typedef struct pecnn_plan pecnn_plan; /* opaque host handle */

/* Device bytes needed by a plan for this batch (instance records, tile tables, node-chunk table). */
int pecnn_plan_device_bytes(const pecnn_batch_desc* desc, size_t* bytes);

/* Build a plan: validates the batch, writes its tables into dev_mem (device, caller-owned,
   >= pecnn_plan_device_bytes, must outlive the plan) with a synchronous upload on 'stream'.
   pin: device uint8 [N_total], 1 = node pinned (Dirichlet condition of eq. 5); caller-owned,
   must outlive the plan. On success *out receives a handle for pecnn_plan_destroy. */
int pecnn_plan_create(const pecnn_batch_desc* desc, const uint8_t* pin, void* dev_mem,
                      size_t dev_bytes, void* stream, pecnn_plan** out);
int pecnn_plan_destroy(pecnn_plan* plan);
int64_t pecnn_plan_nodes(const pecnn_plan* plan);   /* N_total, or -1 for a null plan */

/* Tile configurations chosen for the mass-spring step and the CNN cell (see pecnn_autotune).
   ms_cfg in [0, 5), cnn_cfg in [0, 4); -1 keeps the current choice. */
int pecnn_plan_set_tiles(pecnn_plan* plan, int32_t ms_cfg, int32_t cnn_cfg);
int pecnn_plan_get_tiles(const pecnn_plan* plan, int32_t* ms_cfg, int32_t* cnn_cfg);

/* Uniform pressure p_b of eq. (3) per instance, N/m^2 (host float [n], finite; 0 = none, the
   default of a new plan). On every node the four nearest neighbours are taken round it in the
   order right (0,+1), down (+1,0), left (0,-1), up (-1,0); each consecutive pair (j1, j2)
   whose two nodes lie on the grid adds p_b (x_j1 - x_i) x (x_j2 - x_i), so on the flat rest
   grid X = (j h, i h, 0) p_b > 0 pushes along +z. The mass-spring step adds it to the force;
   the CNN frames add it at the positions of S^k as a known external force,
   dt p_b / m sum_pairs (...), next to the wind (pecnn_forward, pecnn_backward, pecnn_rollout).
   The rollout guard's energy check is off for instances with p_b != 0 (pressure does work).
   Copies the values into the plan's device records (synchronous on `stream`); drops the
   rollout's cached graphs when the set of kernels changes. */
int pecnn_plan_set_pressure(pecnn_plan* plan, const float* pressure, void* stream);

/* A sphere per instance in the constraint operator C of eq. (5) (section 3.1: cloth-object
   collision handled by intersection elimination; the ball absorbs the bounce and its friction
   resists relative motion). sphere: host float [n][5] = centre x, y, z, radius R (>= 0; 0 = no
   sphere, the default of a new plan), friction f in [0, 1]. For a free node with velocity v'
   after the rest of eq. (5), y = x + dt v'; if |y - c| < R the node moves to c + R n,
   n = (y - c)/|y - c| (n = +z when y = c), the inward part of v'.n is removed and the
   tangential part of v' is scaled by 1 - f. Applies to the mass-spring step, to every frame
   (pecnn_forward, pecnn_rollout) and to the reverse pass (pecnn_backward; set the spheres before
   sizing its workspace, which grows by two states when a plan has one). Synchronous on `stream`;
   drops the rollout's cached graphs when the kernels change. */
int pecnn_plan_set_spheres(pecnn_plan* plan, const float* sphere, void* stream);

/* ------------------------------------------------------------------ mass-spring step */

/* Material and integration parameters of the mass-spring model (section 3.1). */
typedef struct {
  float k_struct, k_shear, k_bend; /* spring constants (E of eq. 1), N/m, >= 0 */
  float mu;                        /* spring damping coefficient of eq. (2), >= 0 */
  float drag;                      /* air drag d of eq. (4), >= 0 */
  float g[3];                      /* gravity acceleration of eq. (4) */
  float dt;                        /* time step of eq. (5), > 0 */
} cloth_ms_params;

/* n_steps >= 1 steps of the mass-spring cloth (section 3.1, eqs. 1, 2, 3, 4, 5):
     f_i = m (g + a_ext) - d v_i + sum_j [ -k_j (r - L_j) x_ij/r - mu ((v_ij . x_ij)/r^2) x_ij ]
           + the pressure force of eq. (3) (pecnn_plan_set_pressure)
   over the 12 springs of the 13-point stencil (8 nodes of the 3x3 block, 4 nodes two steps
   away in the cardinal directions; springs exist only inside the grid), x_ij = x_i - x_j,
   r = |x_ij|, then v' = C(v + dt f/m), x' = x + dt v' with C zeroing pinned velocities.
   s_in, s_out: device state [6][N_total]; must not overlap. active: device uint8 [n] or NULL;
   instances with active[b] == 0 are skipped and their part of s_out is not written.
   ws: device workspace of pecnn_workspace_bytes(plan, NULL, PECNN_WS_MS_STEP) bytes when
   n_steps > 1 (the intermediate state), may be NULL when n_steps == 1. */
int cloth_ms_step(const pecnn_plan* plan, const cloth_ms_params* p, const float* s_in, float* s_out,
                  int32_t n_steps, const uint8_t* active, void* ws, size_t ws_bytes, void* stream);

/* ------------------------------------------------------------------ physics-embedded CNN */

enum { PECNN_FP32 = 0, PECNN_BF16 = 1 };

/* The CNN cell (section 3.2, eqs. 6 and 7) with Ch channels, Ch in {16, 32}. theta: device FP32,
   row-major blocks K[Ch][6][3][3] | A[Ch][Ch] | B[Ch][Ch] | W_L[3][Ch] | W_N[3][Ch] | W_D[3][Ch] |
   b_L[3] (pecnn_theta_size(Ch) floats). precision PECNN_BF16 rounds the operands of the
   convolution, of A and B and of the three heads to bfloat16 (round to nearest even) with FP32
   accumulation; PECNN_FP32 keeps every operand in FP32. State and integration stay FP32. */
enum { PECNN_CELL_CONV = 0, PECNN_CELL_PAIR = 1 };

/* cell PECNN_CELL_CONV (default): the channel-mixing convolution cell described above.
   cell PECNN_CELL_PAIR: section 3.2's own cell read literally, Ch = 12 and FP32 only. Channel c
   belongs to neighbour j = i + o_c of the 13-point stencil (o_c in the spring order (0,1),
   (0,-1), (1,0), (-1,0), (1,1), (1,-1), (-1,1), (-1,-1), (0,2), (0,-2), (2,0), (-2,0)); its
   filter is predetermined (+s_c at j, -s_c at the centre, zero elsewhere) and acts alike on each
   axis (eq. 6):  phi_c = s_c (x_j - x_i),  xi_c = s_c (v_j - v_i)  (zero when j is off the grid).
   Eq. (7) axis by axis: dv = sum_c [wL_c phi_c + wN_c sigma(phi_c) + wD_c xi_c sigma(phi_c)] + b_L.
   theta: s[12] | wL[12] | wN[12] | wD[12] | b_L[3] (51 floats). It reads S^k only (S^{k-1} is
   ignored) and runs on the mass-spring step's tiles (configuration ms_cfg). */
typedef struct {
  int32_t ch;
  int32_t precision;
  float dt;          /* time step of one network step (eq. 5 inside the frame), > 0 */
  float isru_alpha;  /* ISRU sigma(z) = z / sqrt(1 + alpha z^2), alpha > 0 */
  const float* theta;
  int32_t cell;      /* PECNN_CELL_CONV or PECNN_CELL_PAIR */
} pecnn_model;

int64_t pecnn_theta_size(int32_t ch);                       /* the convolution cell */
int64_t pecnn_cell_theta_size(int32_t cell, int32_t ch);    /* either cell; -1 if unsupported */

/* One network frame (Fig. 2): per node p,
     U(S)[c][o] = S_c(clamp(p+o)) - [c < 3] S_c(p)    (o in {-1,0,1}^2, clamp-to-edge)
     phi = K U(S^k),  xi = K U(S^k - S^{k-1})                            (eq. 6)
     dv = W_L phi + b_L + W_N sigma((A phi) * (B phi)) + W_D (xi * sigma(phi))   (eq. 7)
     v^{k+1} = C(v^k + dv + dt a_ext + dt f_p(x^k) / m),  x^{k+1} = x^k + dt v^{k+1}   (eq. 5)
   with f_p the pressure force of eq. (3) (zero unless pecnn_plan_set_pressure set one).
   s_prev = S^{k-1}, s_cur = S^k, s_next = S^{k+1}: device [6][N_total]; s_next must not overlap
   the inputs. No workspace. */
int pecnn_forward(const pecnn_plan* plan, const pecnn_model* model, const float* s_prev,
                  const float* s_cur, float* s_next, void* stream);

/* Reverse mode of pecnn_forward (FP32 models only; section 3.2.1: parameters are optimised by
   gradient backpropagation). g_next = dLoss/dS^{k+1} (device [6][N_total]). Accumulates (+=)
   dLoss/dS^k into g_cur, dLoss/dS^{k-1} into g_prev (both device [6][N_total], may be NULL to
   skip) and dLoss/dtheta into g_theta (device [theta size]). Activations are recomputed from
   (s_prev, s_cur); no tape. Deterministic: fixed-order reductions. With spheres in the plan the
   frame is first recomputed without them (for the velocities before the constraint) and g_next
   is carried back through each sphere's projection and friction (the constraint is piecewise
   smooth: at its switching points, |y - c| = R and v.n = 0, the branch the forward took is
   differentiated). ws: pecnn_workspace_bytes(plan, model, PECNN_WS_BACKWARD) bytes, queried
   after the plan's spheres are set. */
int pecnn_backward(const pecnn_plan* plan, const pecnn_model* model, const float* s_prev,
                   const float* s_cur, const float* g_next, float* g_cur, float* g_prev,
                   float* g_theta, void* ws, size_t ws_bytes, void* stream);

/* ------------------------------------------------------------------ rollout */

/* Guard of the learned rollout. Every check_every network steps each active instance is
   checked: if its largest structural stretch ratio r/L exceeds stretch_max, or its energy
   gain (E_now - E_start)/E_ref exceeds energy_gain_max (E_ref = total mass |g| (W-1) h; no
   energy check for instances with a pressure, which does work on the cloth), the
   instance falls back for good to the mass-spring step with 'substeps' steps of sim->dt per
   network step (substeps * sim->dt should equal model->dt). check_every <= 0 disables it.
   frame_err_max > 0 adds a third test at every check, an online physics residual (eq. (8)
   measures the network against the equations in its physics term; here positions are
   compared): the last network step of the chunk is compared with 'substeps' mass-spring steps
   from the same input state, and an instance whose position RMS over its nodes, divided by its
   width (W-1) h, exceeds frame_err_max falls back. That costs
   'substeps' mass-spring steps of the whole batch per check. With the test on, an instance
   that falls back at a check (by any of the three tests) takes the simulator's answer for that
   frame in place of the network's; with it off, the frame that tripped is kept. The fall-back
   starts with the next frame. frame_err_max <= 0 disables the test; NaN is an error. */
typedef struct {
  float stretch_max;
  float energy_gain_max;
  int32_t check_every;
  int32_t substeps;
  float frame_err_max;
} pecnn_guard;

/* n_steps network frames of the whole batch. In/out: s_prev = S^{k-1}, s_cur = S^k; on return
   they hold S^{k+n-1}, S^{k+n}. fallback: device int32 [n], in/out; nonzero marks an instance
   that uses the mass-spring step (set by the guard; the caller may preset it). stats: device
   FP64 [n][4] or NULL: energy at the start, energy at the last check, largest structural
   stretch seen at checks, network step of the fall-back (-1 if none). At a check that trips an
   instance with the frame-error test on, the energy and stretch recorded are those of the
   network's frame that the check judged, before the simulator's frame replaces it.
   ws: pecnn_workspace_bytes(plan, model, PECNN_WS_ROLLOUT). The steps between checks run as
   one captured HIP graph (cached in the plan per buffer set). The host reads the fallback
   count at the start (waiting for the stream) and after every check but the last; it reads a
   check's count after launching the chunk that follows it, so it waits only for work queued
   before that chunk. A chunk launched before the first instances fell back is completed for
   them afterwards by the mass-spring steps alone. The call returns with the last chunk still
   queued. */
int pecnn_rollout(pecnn_plan* plan, const pecnn_model* model, const cloth_ms_params* sim,
                  const pecnn_guard* guard, float* s_prev, float* s_cur, int32_t n_steps,
                  int32_t* fallback, double* stats, void* ws, size_t ws_bytes, void* stream);

/* ------------------------------------------------------------------ diagnostics (FP64) */

/* Per instance b, in FP64 from the FP32 state (two-stage, fixed-order reduction):
     out[4b+0] = sum over nodes of |x - x_ref|^2 (0 when s_ref is NULL)
     out[4b+1] = energy: sum 1/2 m |v|^2 + sum over springs 1/2 k (r - L)^2 - sum m (g + a_ext).x
     out[4b+2] = largest r/L over structural springs
     out[4b+3] = largest r/L over all springs
   out: device double [4n]. ws: pecnn_workspace_bytes(plan, NULL, PECNN_WS_REDUCE). */
int cloth_reduce_fp64(const pecnn_plan* plan, const cloth_ms_params* p, const float* s,
                      const float* s_ref, double* out, void* ws, size_t ws_bytes, void* stream);

/* Allocation-free cloth_reduce_fp64, for callers that cannot allocate device memory or hand
   over a workspace (code under HIP graph capture, tight serving loops, harnesses that forbid
   hipMalloc). Same arguments without ws, the same kernels and the same results bit for bit: the
   per-chunk FP64 partials live in a fixed device array inside the library, 4 MiB per device,
   held until the process ends. Its device address is looked up once per device (by
   pecnn_plan_create, or else by the first call with that device current). A plan with more
   than PECNN_NOALLOC_REDUCE_MAX_CHUNKS node chunks (instance b has ceil(H_b W_b / 256) chunks;
   e.g. 512 cloths of 256 x 256 are 2^17 chunks) returns PECNN_E_WORKSPACE with no side effect.
   Every call on one device shares that array: calls that can overlap on one device (other
   streams, other host threads) race and must be serialised by the caller. Each call writes
   every partial it reads, so the array never needs clearing. Calls no allocating routine. */
#define PECNN_NOALLOC_REDUCE_MAX_CHUNKS 131072
int cloth_reduce_fp64_noalloc(const pecnn_plan* plan, const cloth_ms_params* p, const float* s,
                              const float* s_ref, double* out, void* stream);

/* ------------------------------------------------------------------ training helpers */

/* Data term of eq. (8) for one predicted state: w / n_free * sum over unpinned nodes of
   |x_hat - x|^2 / sx^2 + |v_hat - v|^2 / sv^2. Adds the value to *loss (device double, one
   value) and its gradient w.r.t. s_hat to g_hat (device [6][N_total], +=). Either may be NULL,
   not both: with loss NULL only the gradient is formed (the same bits, no sums; one launch
   instead of two). n_free = number of unpinned nodes over which the mean is taken (> 0).
   ws: pecnn_workspace_bytes(plan, NULL, PECNN_WS_REDUCE). */
int pecnn_loss_mse(const pecnn_plan* plan, const float* s_hat, const float* s_true, float sx,
                   float sv, float w, int64_t n_free, double* loss, float* g_hat, void* ws,
                   size_t ws_bytes, void* stream);

/* Adam (Table 1), step t >= 1 with bias correction, over n parameters (device FP32). */
int pecnn_adam_step(int64_t n, float lr, float beta1, float beta2, float eps, int32_t t,
                    float* theta, float* m, float* v, const float* g, void* stream);

/* Gather training windows: for window w = 0..n_win-1 and t = 0..n_frames-1 copy frame
   frame_idx[w] + t of trajectory instance traj_inst[w] into instance w of out[t].
   traj: device FP32 frames [n_saved][6][traj_nodes] of a trajectory batch whose instance
   offsets are traj_off (device int64 [n_traj + 1]); frame_idx, traj_inst: device int32 [n_win];
   out: device FP32 [n_frames][6][n_win * nodes_per_win]; every window instance has
   nodes_per_win nodes (same grid). Frames out of range are an error the caller must avoid:
   indices are clamped to the valid range. */
int pecnn_gather_windows(const float* traj, int64_t traj_nodes, int32_t n_saved,
                         const int64_t* traj_off, int32_t n_traj, const int32_t* traj_inst,
                         const int32_t* frame_idx, int32_t n_win, int32_t nodes_per_win,
                         int32_t n_frames, float* out, void* stream);

/* ------------------------------------------------------------------ workspace and tuning */

enum { PECNN_WS_MS_STEP = 0, PECNN_WS_BACKWARD = 1, PECNN_WS_ROLLOUT = 2, PECNN_WS_REDUCE = 3 };

/* Device workspace bytes for the given entry point (model may be NULL except for
   PECNN_WS_BACKWARD and PECNN_WS_ROLLOUT). */
int pecnn_workspace_bytes(const pecnn_plan* plan, const pecnn_model* model, int32_t which,
                          size_t* bytes);

/* Time every tile configuration of the mass-spring step and the CNN cell on this batch
   (synchronous: three interleaved rounds, each running 'reps' timed launches of every
   configuration on 'stream' using the given buffers, which are overwritten) and store the
   fastest in the plan; a configuration's time is its best round, so a clock still ramping under
   the new load favours none. s_a, s_b, s_c: device [6][N_total] scratch states (contents
   preserved are not guaranteed). ms_ms/cnn_ms (host, nullable, length 5 and 4) receive the
   best round's mean milliseconds per launch of each configuration. */
int pecnn_autotune(pecnn_plan* plan, const cloth_ms_params* p, const pecnn_model* model,
                   float* s_a, float* s_b, float* s_c, int32_t reps, float* ms_ms, float* cnn_ms,
                   void* stream);

/* ------------------------------------------------------------------ measured peaks */

/* Peaks of the current device measured with short synthetic kernels, for quoting the rooflines
   against the chip at hand as well as its datasheet (not a step of the method). out: host
   double [6]: [0] HBM copy bandwidth, bytes read plus written per second; [1] FP32 VALU FMA
   lane operations per second; [2] v_rsq_f32 lane operations per second; [3] FP64 VALU FMA lane
   operations per second; [4] bf16 MFMA (16x16x32) FLOP per second; [5] FP32 MFMA (16x16x4)
   FLOP per second. scratch: caller-owned device buffer, 256-byte aligned, of at least 64 MiB;
   the copy moves half of what is left after 2 MiB of kernel results into the other half, so a
   buffer of 2 GiB or more measures HBM rather than the 256 MB last-level cache. Its contents
   are overwritten. Synchronous on 'stream' (about 15 ms). */
int pecnn_measure_peaks(double* out, void* scratch, size_t scratch_bytes, void* stream);

const char* pecnn_status_string(int status);
const char* pecnn_last_error(void);
/* Library version, incremented when the ABI changes. */
int32_t pecnn_version(void);

#ifdef __cplusplus
}
#endif
#endif /* PECNN_H */
