"""ctypes binding of libpecnn.so (include/pecnn.h), with the same entry-point names.

Argument marshalling only: every step of the path runs in the HIP library. PyTorch
provides device memory (tensors) and the stream. There is no fallback: if the library
is not built, or a call fails, a PecnnError is raised.
"""
from __future__ import annotations

import ctypes as C
import os

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
# the in-tree build; PECNN_LIB names another build of the same sources (the sanitizer test's)
LIB_PATH = os.environ.get("PECNN_LIB") or os.path.join(_HERE, "lib", "libpecnn.so")

PECNN_FP32, PECNN_BF16 = 0, 1
CELL_CONV, CELL_PAIR = 0, 1
WS_MS_STEP, WS_BACKWARD, WS_ROLLOUT, WS_REDUCE = 0, 1, 2, 3
N_MS_CFG, N_CNN_CFG = 5, 4


class PecnnError(RuntimeError):
    pass


class BatchDesc(C.Structure):
    _fields_ = [("n", C.c_int32), ("H", C.c_void_p), ("W", C.c_void_p), ("h", C.c_void_p),
                ("mass", C.c_void_p), ("a_ext", C.c_void_p)]


class MsParams(C.Structure):
    _fields_ = [("k_struct", C.c_float), ("k_shear", C.c_float), ("k_bend", C.c_float), ("mu", C.c_float),
                ("drag", C.c_float), ("g", C.c_float * 3), ("dt", C.c_float)]


class Model(C.Structure):
    _fields_ = [("ch", C.c_int32), ("precision", C.c_int32), ("dt", C.c_float), ("isru_alpha", C.c_float),
                ("theta", C.c_void_p), ("cell", C.c_int32)]


class Guard(C.Structure):
    _fields_ = [("stretch_max", C.c_float), ("energy_gain_max", C.c_float), ("check_every", C.c_int32),
                ("substeps", C.c_int32), ("frame_err_max", C.c_float)]


_lib = None


def lib():
    """Load libpecnn.so (built in-tree by __graft_entry__.build())."""
    global _lib
    if _lib is not None:
        return _lib
    if not os.path.exists(LIB_PATH):
        raise PecnnError("libpecnn.so is not built (%s); run __graft_entry__.build()" % LIB_PATH)
    L = C.CDLL(LIB_PATH)
    i32, i64, f32, vp, sz = C.c_int32, C.c_int64, C.c_float, C.c_void_p, C.c_size_t
    P = C.POINTER
    sig = {
        "pecnn_plan_device_bytes": ([P(BatchDesc), P(sz)], i32),
        "pecnn_plan_create": ([P(BatchDesc), vp, vp, sz, vp, P(vp)], i32),
        "pecnn_plan_destroy": ([vp], i32),
        "pecnn_plan_nodes": ([vp], i64),
        "pecnn_plan_set_tiles": ([vp, i32, i32], i32),
        "pecnn_plan_get_tiles": ([vp, P(i32), P(i32)], i32),
        "pecnn_plan_set_pressure": ([vp, vp, vp], i32),
        "pecnn_plan_set_spheres": ([vp, vp, vp], i32),
        "cloth_ms_step": ([vp, P(MsParams), vp, vp, i32, vp, vp, sz, vp], i32),
        "pecnn_theta_size": ([i32], i64),
        "pecnn_cell_theta_size": ([i32, i32], i64),
        "pecnn_forward": ([vp, P(Model), vp, vp, vp, vp], i32),
        "pecnn_backward": ([vp, P(Model), vp, vp, vp, vp, vp, vp, vp, sz, vp], i32),
        "pecnn_rollout": ([vp, P(Model), P(MsParams), P(Guard), vp, vp, i32, vp, vp, vp, sz, vp], i32),
        "cloth_reduce_fp64": ([vp, P(MsParams), vp, vp, vp, vp, sz, vp], i32),
        "cloth_reduce_fp64_noalloc": ([vp, P(MsParams), vp, vp, vp, vp], i32),
        "pecnn_loss_mse": ([vp, vp, vp, f32, f32, f32, i64, vp, vp, vp, sz, vp], i32),
        "pecnn_adam_step": ([i64, f32, f32, f32, f32, i32, vp, vp, vp, vp, vp], i32),
        "pecnn_gather_windows": ([vp, i64, i32, vp, i32, vp, vp, i32, i32, i32, vp, vp], i32),
        "pecnn_workspace_bytes": ([vp, P(Model), i32, P(sz)], i32),
        "pecnn_autotune": ([vp, P(MsParams), P(Model), vp, vp, vp, i32, vp, vp, vp], i32),
        "pecnn_measure_peaks": ([vp, vp, sz, vp], i32),
        "pecnn_status_string": ([i32], C.c_char_p),
        "pecnn_last_error": ([], C.c_char_p),
        "pecnn_version": ([], i32),
    }
    for name, (args, res) in sig.items():
        fn = getattr(L, name)
        fn.argtypes = args
        fn.restype = res
    _lib = L
    return L


def exported_symbols():
    return ["pecnn_plan_device_bytes", "pecnn_plan_create", "pecnn_plan_destroy", "pecnn_plan_nodes",
            "pecnn_plan_set_tiles", "pecnn_plan_get_tiles", "pecnn_plan_set_pressure", "pecnn_plan_set_spheres",
            "cloth_ms_step",
            "pecnn_theta_size", "pecnn_cell_theta_size",
            "pecnn_forward", "pecnn_backward", "pecnn_rollout", "cloth_reduce_fp64", "cloth_reduce_fp64_noalloc",
            "pecnn_loss_mse",
            "pecnn_adam_step", "pecnn_gather_windows", "pecnn_workspace_bytes", "pecnn_autotune",
            "pecnn_measure_peaks",
            "pecnn_status_string", "pecnn_last_error", "pecnn_version"]


def check(rc: int, what: str = ""):
    if rc != 0:
        L = lib()
        msg = L.pecnn_last_error().decode()
        raise PecnnError("%s failed: %s (%s)" % (what, L.pecnn_status_string(rc).decode(), msg))


def _ptr(t):
    if t is None:
        return None
    return C.c_void_p(t.data_ptr())


def _stream(stream=None):
    import torch
    s = stream if stream is not None else torch.cuda.current_stream()
    return C.c_void_p(s.cuda_stream)


def ms_params(mat, dt=None) -> MsParams:
    p = MsParams()
    p.k_struct, p.k_shear, p.k_bend = mat.k_struct, mat.k_shear, mat.k_bend
    p.mu, p.drag = mat.mu, mat.drag
    p.g[0], p.g[1], p.g[2] = mat.g
    p.dt = mat.dt if dt is None else dt
    return p


class Plan:
    """A batch of cloth instances bound to device tables (pecnn_plan_create)."""

    def __init__(self, H, W, h, mass, a_ext, pin, device="cuda"):
        import torch
        self._H = np.ascontiguousarray(H, np.int32)
        self._W = np.ascontiguousarray(W, np.int32)
        self._h = np.ascontiguousarray(h, np.float32)
        self._m = np.ascontiguousarray(mass, np.float32)
        self._a = np.ascontiguousarray(np.asarray(a_ext, np.float32).reshape(-1))
        self.n = len(self._H)
        d = BatchDesc(self.n, self._H.ctypes.data, self._W.ctypes.data, self._h.ctypes.data,
                      self._m.ctypes.data, self._a.ctypes.data)
        self.desc = d
        L = lib()
        nb = C.c_size_t(0)
        check(L.pecnn_plan_device_bytes(C.byref(d), C.byref(nb)), "pecnn_plan_device_bytes")
        if isinstance(pin, torch.Tensor) and pin.is_cuda:
            # already on the device (the plan keeps the reference; nothing is copied)
            if pin.dtype != torch.uint8 or not pin.is_contiguous() or pin.numel() != int(np.sum(
                    self._H.astype(np.int64) * self._W)):
                raise ValueError("pin: a contiguous uint8 device tensor of one byte per node")
            self.pin = pin
        else:
            self.pin = torch.as_tensor(np.ascontiguousarray(pin, np.uint8), device=device)
        self.mem = torch.empty(nb.value, dtype=torch.uint8, device=device)
        h = C.c_void_p()
        check(L.pecnn_plan_create(C.byref(d), _ptr(self.pin), _ptr(self.mem), nb.value, _stream(), C.byref(h)),
              "pecnn_plan_create")
        self.handle = h
        self.total = int(L.pecnn_plan_nodes(h))
        self.H, self.W = self._H, self._W
        off = np.zeros(self.n + 1, np.int64)
        off[1:] = np.cumsum(self._H.astype(np.int64) * self._W)
        self.node_off = off

    @classmethod
    def from_batch(cls, batch, device="cuda"):
        plan = cls(batch.H, batch.W, batch.h, batch.mass, batch.a_ext, batch.pin, device)
        pres = getattr(batch, "pressure", None)
        if pres is not None and np.any(np.asarray(pres) != 0):
            plan.set_pressure(pres)
        sph = getattr(batch, "sphere", None)
        if sph is not None and np.any(np.asarray(sph)[:, 3] > 0):
            plan.set_spheres(sph)
        return plan

    def set_spheres(self, spheres):
        """Per-instance sphere (centre x, y, z, radius, friction) of the constraint in eq. (5)."""
        self._s = np.ascontiguousarray(spheres, np.float32).reshape(-1)
        if self._s.size != 5 * self.n:
            raise ValueError("need five values per instance")
        check(lib().pecnn_plan_set_spheres(self.handle, self._s.ctypes.data, _stream()), "pecnn_plan_set_spheres")

    def set_pressure(self, pressure):
        """Per-instance uniform pressure of eq. (3), N/m^2 (pecnn_plan_set_pressure)."""
        self._p = np.ascontiguousarray(pressure, np.float32).reshape(-1)
        if self._p.size != self.n:
            raise ValueError("need one pressure per instance")
        check(lib().pecnn_plan_set_pressure(self.handle, self._p.ctypes.data, _stream()), "pecnn_plan_set_pressure")

    def close(self):
        if getattr(self, "handle", None) is not None and _lib is not None:
            _lib.pecnn_plan_destroy(self.handle)
            self.handle = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass

    def set_tiles(self, ms_cfg=-1, cnn_cfg=-1):
        check(lib().pecnn_plan_set_tiles(self.handle, ms_cfg, cnn_cfg), "pecnn_plan_set_tiles")

    def get_tiles(self):
        a, b = C.c_int32(), C.c_int32()
        check(lib().pecnn_plan_get_tiles(self.handle, C.byref(a), C.byref(b)), "pecnn_plan_get_tiles")
        return a.value, b.value

    def workspace(self, which, model=None):
        import torch
        nb = C.c_size_t(0)
        check(lib().pecnn_workspace_bytes(self.handle, C.byref(model) if model is not None else None, which,
                                          C.byref(nb)), "pecnn_workspace_bytes")
        return torch.empty(max(nb.value, 1), dtype=torch.uint8, device=self.mem.device)


def make_model(theta, ch, precision=PECNN_FP32, dt=5e-3, alpha=1.0, cell=CELL_CONV) -> Model:
    m = Model()
    m.ch, m.precision, m.dt, m.isru_alpha, m.cell = ch, precision, dt, alpha, cell
    m.theta = theta.data_ptr()
    m._theta_ref = theta  # keep the tensor alive
    return m


def pecnn_theta_size(ch: int) -> int:
    return int(lib().pecnn_theta_size(ch))


def cloth_ms_step(plan: Plan, params: MsParams, s_in, s_out, n_steps=1, active=None, ws=None, stream=None):
    if n_steps > 1 and ws is None:
        ws = plan.workspace(WS_MS_STEP)
    check(lib().cloth_ms_step(plan.handle, C.byref(params), _ptr(s_in), _ptr(s_out), int(n_steps), _ptr(active),
                              _ptr(ws), ws.numel() if ws is not None else 0, _stream(stream)), "cloth_ms_step")


def pecnn_forward(plan: Plan, model: Model, s_prev, s_cur, s_next, stream=None):
    check(lib().pecnn_forward(plan.handle, C.byref(model), _ptr(s_prev), _ptr(s_cur), _ptr(s_next),
                              _stream(stream)), "pecnn_forward")


def pecnn_backward(plan: Plan, model: Model, s_prev, s_cur, g_next, g_cur, g_prev, g_theta, ws=None, stream=None):
    if ws is None:
        ws = plan.workspace(WS_BACKWARD, model)
    check(lib().pecnn_backward(plan.handle, C.byref(model), _ptr(s_prev), _ptr(s_cur), _ptr(g_next), _ptr(g_cur),
                               _ptr(g_prev), _ptr(g_theta), _ptr(ws), ws.numel(), _stream(stream)), "pecnn_backward")


def pecnn_rollout(plan: Plan, model: Model, sim: MsParams, guard: Guard, s_prev, s_cur, n_steps, fallback,
                  stats=None, ws=None, stream=None):
    if ws is None:
        ws = plan.workspace(WS_ROLLOUT)
    check(lib().pecnn_rollout(plan.handle, C.byref(model), C.byref(sim), C.byref(guard), _ptr(s_prev), _ptr(s_cur),
                              int(n_steps), _ptr(fallback), _ptr(stats), _ptr(ws), ws.numel(), _stream(stream)),
          "pecnn_rollout")


def cloth_reduce_fp64(plan: Plan, params: MsParams, s, s_ref, out, ws=None, stream=None):
    if ws is None:
        ws = plan.workspace(WS_REDUCE)
    check(lib().cloth_reduce_fp64(plan.handle, C.byref(params), _ptr(s), _ptr(s_ref), _ptr(out), _ptr(ws), ws.numel(),
                                  _stream(stream)), "cloth_reduce_fp64")


def cloth_reduce_fp64_noalloc(plan: Plan, params: MsParams, s, s_ref, out, stream=None):
    check(lib().cloth_reduce_fp64_noalloc(plan.handle, C.byref(params), _ptr(s), _ptr(s_ref), _ptr(out),
                                          _stream(stream)), "cloth_reduce_fp64_noalloc")


def pecnn_loss_mse(plan: Plan, s_hat, s_true, sx, sv, w, n_free, loss, g_hat, ws=None, stream=None):
    if ws is None:
        ws = plan.workspace(WS_REDUCE)
    check(lib().pecnn_loss_mse(plan.handle, _ptr(s_hat), _ptr(s_true), sx, sv, w, int(n_free), _ptr(loss),
                               _ptr(g_hat), _ptr(ws), ws.numel(), _stream(stream)), "pecnn_loss_mse")


def pecnn_adam_step(theta, m, v, g, t, lr=1e-3, beta1=0.9, beta2=0.999, eps=1e-8, stream=None):
    check(lib().pecnn_adam_step(theta.numel(), lr, beta1, beta2, eps, int(t), _ptr(theta), _ptr(m), _ptr(v), _ptr(g),
                                _stream(stream)), "pecnn_adam_step")


def pecnn_gather_windows(traj, traj_nodes, n_saved, traj_off, n_traj, traj_inst, frame_idx, n_win, npw, n_frames,
                         out, stream=None):
    check(lib().pecnn_gather_windows(_ptr(traj), int(traj_nodes), int(n_saved), _ptr(traj_off), int(n_traj),
                                     _ptr(traj_inst), _ptr(frame_idx), int(n_win), int(npw), int(n_frames), _ptr(out),
                                     _stream(stream)), "pecnn_gather_windows")


def pecnn_autotune(plan: Plan, params: MsParams, model, s_a, s_b, s_c, reps=10, stream=None):
    ms = (C.c_float * N_MS_CFG)()
    cn = (C.c_float * N_CNN_CFG)()
    check(lib().pecnn_autotune(plan.handle, C.byref(params), C.byref(model) if model is not None else None,
                               _ptr(s_a), _ptr(s_b), _ptr(s_c), int(reps), ms, cn, _stream(stream)), "pecnn_autotune")
    return list(ms), list(cn)


PEAK_KEYS = ("hbm_copy_bytes_per_s", "fp32_valu_fma_lane_ops_per_s", "rsq_f32_lane_ops_per_s",
             "fp64_valu_fma_lane_ops_per_s", "bf16_mfma_flop_per_s", "fp32_mfma_flop_per_s")


def pecnn_measure_peaks(scratch, stream=None):
    """The device's measured peaks (pecnn_measure_peaks) as a dict keyed by PEAK_KEYS."""
    out = (C.c_double * 6)()
    check(lib().pecnn_measure_peaks(out, _ptr(scratch), scratch.numel() * scratch.element_size(), _stream(stream)),
          "pecnn_measure_peaks")
    return dict(zip(PEAK_KEYS, list(out)))
