"""FP64 CPU oracle of the physics-embedded cloth method (arXiv 2403.12820).

TEST INFRASTRUCTURE ONLY: the tests, the smoke check and the CPU-baseline leg of
the benchmark use it; the product library never imports, links or runs it.

`oracle.c` holds the arithmetic (plain loops in double precision); this module
compiles it with gcc and marshals numpy arrays through ctypes. Every function
works on one cloth instance at a time; the batch helpers loop over instances.

Paper passages followed (section / equation):
  ms_force, ms_step, ms_run  - section 3.1, eqs. (1), (2), (3), (4), (5); the constraint of
                               eq. (5) also handles a sphere (intersection elimination, friction)
  cnn_forward                - section 3.2, eqs. (6), (7), then (5) (Fig. 2), with wind and the
                               pressure of eq. (3) as known external forces
  cnn_backward               - section 3.2.1, reverse mode of the above
  pair_forward, pair_backward - section 3.2 read literally: twelve frozen neighbour-difference
                               channels shared by the axes, eqs. (6), (7), then (5)
  loss_mse                   - eq. (8), data term
  adam                       - Table 1 (optimizer Adam)
  energy, max_stretch, rms   - diagnostics of the rollout (no paper formula)
  bf16_round                 - the operand rounding of the emulated-bf16 forward: float32,
                               then bfloat16 by round to nearest, ties to even (no paper
                               formula: the precision of the inference path is a design choice)
"""
from __future__ import annotations

import ctypes as C
import os
import subprocess

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
_SRC = os.path.join(_HERE, "oracle.c")
_LIB = os.path.join(_HERE, "lib", "liboracle.so")
_lib = None


def build(force: bool = True) -> str:
    """Compile oracle.c into oracle/lib/liboracle.so (plain -O2, no fast-math)."""
    os.makedirs(os.path.dirname(_LIB), exist_ok=True)
    if force or not os.path.exists(_LIB) or os.path.getmtime(_LIB) < os.path.getmtime(_SRC):
        tmp = _LIB + ".tmp%d" % os.getpid()
        subprocess.check_call(["gcc", "-O2", "-std=c99", "-fPIC", "-shared", "-fno-fast-math",
                               "-ffp-contract=off", "-o", tmp, _SRC, "-lm"])
        os.replace(tmp, _LIB)
    return _LIB


def _load():
    global _lib
    if _lib is None:
        alt = os.environ.get("PECNN_ORACLE_LIB")  # another build of oracle.c (the sanitizer test's)
        if alt:
            _lib = C.CDLL(alt)
        else:
            if not os.path.exists(_LIB) or os.path.getmtime(_LIB) < os.path.getmtime(_SRC):
                build(force=True)
            _lib = C.CDLL(_LIB)
        d, i, l, p = C.c_double, C.c_int, C.c_long, C.c_void_p
        _lib.or_ms_force.argtypes = [i, i, d, d, p, d, p, p, p, p]
        _lib.or_ms_step.argtypes = [i, i, d, d, p, d, p, p, p, p, p]
        _lib.or_ms_run.argtypes = [i, i, d, d, p, d, p, p, p, i, p]
        _lib.or_energy.argtypes = [i, i, d, d, p, p, p]
        _lib.or_energy.restype = d
        _lib.or_max_stretch.argtypes = [i, i, d, p, i]
        _lib.or_max_stretch.restype = d
        _lib.or_sq_pos_err.argtypes = [i, i, p, p]
        _lib.or_sq_pos_err.restype = d
        _lib.or_theta_size.argtypes = [i]
        _lib.or_theta_size.restype = l
        _lib.or_cnn_forward.argtypes = [i, i, i, d, d, p, d, p, p, p, p, p, i, p, p]
        _lib.or_cnn_backward.argtypes = [i, i, i, d, d, p, d, p, p, p, p, p, p, p, p, p]
        _lib.or_pair_theta_size.argtypes = []
        _lib.or_pair_theta_size.restype = l
        _lib.or_pair_forward.argtypes = [i, i, d, d, p, d, p, p, p, p, p, p]
        _lib.or_pair_backward.argtypes = [i, i, d, d, p, d, p, p, p, p, p, p, p]
        _lib.or_loss_mse.argtypes = [l, p, l, d, d, d, p, p, p]
        _lib.or_loss_mse.restype = d
        _lib.or_adam.argtypes = [l, d, d, d, d, i, p, p, p, p]
        _lib.or_bf16_array.argtypes = [l, p, p]
    return _lib


class _MsParams(C.Structure):
    _fields_ = [("k", C.c_double * 3), ("mu", C.c_double), ("drag", C.c_double),
                ("g", C.c_double * 3), ("dt", C.c_double)]


def _f64(a) -> np.ndarray:
    return np.ascontiguousarray(a, dtype=np.float64)


def _u8(a) -> np.ndarray:
    return np.ascontiguousarray(a, dtype=np.uint8)


def _ptr(a: np.ndarray):
    return a.ctypes.data_as(C.c_void_p)


def ms_params(mat, dt=None) -> _MsParams:
    p = _MsParams()
    p.k[0], p.k[1], p.k[2] = mat.k_struct, mat.k_shear, mat.k_bend
    p.mu, p.drag = mat.mu, mat.drag
    p.g[0], p.g[1], p.g[2] = mat.g
    p.dt = mat.dt if dt is None else dt
    return p


def ms_force(H, W, h, m, a_ext, pin, s, mat, pressure=0.0):
    s = _f64(s).reshape(6, H * W)
    f = np.zeros((3, H * W))
    a, pn, P = _f64(a_ext), _u8(pin), ms_params(mat)
    _load().or_ms_force(H, W, h, m, _ptr(a), float(pressure), C.byref(P), _ptr(pn), _ptr(s), _ptr(f))
    return f


def _sphere(sphere):
    """(cx, cy, cz, R, friction) as a float64 array, or None for no sphere."""
    return None if sphere is None else _f64(sphere).reshape(5)


def ms_step(H, W, h, m, a_ext, pin, s, mat, dt=None, pressure=0.0, sphere=None):
    s = _f64(s).reshape(6, H * W)
    out = np.empty_like(s)
    a, pn, P, sp = _f64(a_ext), _u8(pin), ms_params(mat, dt), _sphere(sphere)
    _load().or_ms_step(H, W, h, m, _ptr(a), float(pressure), C.byref(P), _ptr(pn), _ptr(s), _ptr(out),
                       _ptr(sp) if sp is not None else None)
    return out


def ms_run(H, W, h, m, a_ext, pin, s, mat, n_steps, dt=None, pressure=0.0, sphere=None):
    s = _f64(s).reshape(6, H * W).copy()
    a, pn, P, sp = _f64(a_ext), _u8(pin), ms_params(mat, dt), _sphere(sphere)
    _load().or_ms_run(H, W, h, m, _ptr(a), float(pressure), C.byref(P), _ptr(pn), _ptr(s), int(n_steps),
                      _ptr(sp) if sp is not None else None)
    return s


def energy(H, W, h, m, a_ext, s, mat) -> float:
    s = _f64(s).reshape(6, H * W)
    a, P = _f64(a_ext), ms_params(mat)
    return _load().or_energy(H, W, h, m, _ptr(a), C.byref(P), _ptr(s))


def max_stretch(H, W, h, s, fam_mask=1) -> float:
    s = _f64(s).reshape(6, H * W)
    return _load().or_max_stretch(H, W, h, _ptr(s), int(fam_mask))


def sq_pos_err(H, W, s, ref) -> float:
    s, ref = _f64(s).reshape(6, H * W), _f64(ref).reshape(6, H * W)
    return _load().or_sq_pos_err(H, W, _ptr(s), _ptr(ref))


def bf16_round(x) -> np.ndarray:
    """The operand rounding of the emulated-bf16 forward (emu flags of cnn_forward): each value
    taken to float32, then to bfloat16 with round to nearest, ties to even."""
    x = _f64(x)
    y = np.empty_like(x)
    _load().or_bf16_array(x.size, _ptr(x), _ptr(y))
    return y


def theta_size(ch) -> int:
    return int(_load().or_theta_size(ch))


def cnn_forward(H, W, ch, alpha, dt, a_ext, pin, theta, s_prev, s_cur, emu=0, pm=0.0, sphere=None):
    """Returns (s_next [6, n], dv [3, n]). emu: bf16 operand-rounding flags (0 = exact FP64);
    pm: pressure per unit node mass (eq. 3 force / m)."""
    sp, sc = _f64(s_prev).reshape(6, H * W), _f64(s_cur).reshape(6, H * W)
    th, a, pn = _f64(theta), _f64(a_ext), _u8(pin)
    assert th.size == theta_size(ch) and ch <= 64
    out = np.empty((6, H * W))
    dv = np.empty((3, H * W))
    sph = _sphere(sphere)
    _load().or_cnn_forward(H, W, ch, alpha, dt, _ptr(a), float(pm), _ptr(pn), _ptr(th), _ptr(sp), _ptr(sc),
                           _ptr(out), int(emu), _ptr(dv), _ptr(sph) if sph is not None else None)
    return out, dv


def cnn_backward(H, W, ch, alpha, dt, pin, theta, s_prev, s_cur, g_next, pm=0.0, a_ext=(0.0, 0.0, 0.0),
                 sphere=None):
    """Returns (g_cur, g_prev, g_theta) for g_next = dLoss/dS^{k+1}. a_ext matters only with a
    sphere (the constraint's adjoint needs the velocity before it)."""
    sp, sc, gn = (_f64(x).reshape(6, H * W) for x in (s_prev, s_cur, g_next))
    th, pn, a = _f64(theta), _u8(pin), _f64(a_ext)
    gc, gp, gt = np.zeros((6, H * W)), np.zeros((6, H * W)), np.zeros(th.size)
    sph = _sphere(sphere)
    _load().or_cnn_backward(H, W, ch, alpha, dt, _ptr(a), float(pm), _ptr(pn), _ptr(th), _ptr(sp), _ptr(sc),
                            _ptr(gn), _ptr(gc), _ptr(gp), _ptr(gt), _ptr(sph) if sph is not None else None)
    return gc, gp, gt


def pair_theta_size() -> int:
    return int(_load().or_pair_theta_size())


def pair_forward(H, W, alpha, dt, a_ext, pin, theta, s_cur, pm=0.0, sphere=None):
    """The paper's pair cell, one frame: returns (s_next [6, n], dv [3, n])."""
    sc = _f64(s_cur).reshape(6, H * W)
    th, a, pn = _f64(theta), _f64(a_ext), _u8(pin)
    assert th.size == pair_theta_size()
    out, dv = np.empty((6, H * W)), np.empty((3, H * W))
    sph = _sphere(sphere)
    _load().or_pair_forward(H, W, alpha, dt, _ptr(a), float(pm), _ptr(pn), _ptr(th), _ptr(sc), _ptr(out), _ptr(dv),
                            _ptr(sph) if sph is not None else None)
    return out, dv


def pair_backward(H, W, alpha, dt, pin, theta, s_cur, g_next, pm=0.0, a_ext=(0.0, 0.0, 0.0), sphere=None):
    """Returns (g_cur, g_theta) for g_next = dLoss/dS^{k+1}. a_ext matters only with a sphere."""
    sc, gn = _f64(s_cur).reshape(6, H * W), _f64(g_next).reshape(6, H * W)
    th, pn, a = _f64(theta), _u8(pin), _f64(a_ext)
    gc, gt = np.zeros((6, H * W)), np.zeros(th.size)
    sph = _sphere(sphere)
    _load().or_pair_backward(H, W, alpha, dt, _ptr(a), float(pm), _ptr(pn), _ptr(th), _ptr(sc), _ptr(gn), _ptr(gc),
                             _ptr(gt), _ptr(sph) if sph is not None else None)
    return gc, gt


def loss_mse(pin, n_free, sx, sv, w, s_hat, s_true, want_grad=True):
    sh, st = _f64(s_hat).reshape(6, -1), _f64(s_true).reshape(6, -1)
    n = sh.shape[1]
    g = np.zeros_like(sh) if want_grad else None
    pn = _u8(pin)
    val = _load().or_loss_mse(n, _ptr(pn), int(n_free), sx, sv, w, _ptr(sh), _ptr(st),
                              _ptr(g) if g is not None else None)
    return val, g


def adam(theta, m, v, g, t, lr=1e-3, b1=0.9, b2=0.999, eps=1e-8):
    th, m, v, g = (_f64(x).copy() for x in (theta, m, v, g))
    _load().or_adam(th.size, lr, b1, b2, eps, int(t), _ptr(th), _ptr(m), _ptr(v), _ptr(g))
    return th, m, v


# ------------------------------------------------------------------ batch helpers
def _inst(batch, b):
    return (int(batch.H[b]), int(batch.W[b]), float(batch.h[b]), float(batch.mass[b]),
            np.asarray(batch.a_ext[b], np.float64), batch.pin[batch.instance(b)])


def _pressure(batch, b):
    p = getattr(batch, "pressure", None)
    return 0.0 if p is None else float(p[b])


def _batch_sphere(batch, b):
    sp = getattr(batch, "sphere", None)
    if sp is None or not float(sp[b][3]) > 0.0:
        return None
    return np.asarray(sp[b], np.float64)


def batch_ms_step(batch, s, mat, n_steps=1, dt=None):
    s = _f64(s)
    out = np.empty_like(s)
    for b in range(batch.n):
        H, W, h, m, a, pin = _inst(batch, b)
        sl = batch.instance(b)
        out[:, sl] = ms_run(H, W, h, m, a, pin, s[:, sl], mat, n_steps, dt, _pressure(batch, b), _batch_sphere(batch, b))
    return out


def batch_cnn_forward(batch, ch, alpha, dt, theta, s_prev, s_cur, emu=0):
    s_prev, s_cur = _f64(s_prev), _f64(s_cur)
    out = np.empty_like(s_cur)
    dv = np.empty((3, s_cur.shape[1]))
    for b in range(batch.n):
        H, W, h, m, a, pin = _inst(batch, b)
        sl = batch.instance(b)
        out[:, sl], dv[:, sl] = cnn_forward(H, W, ch, alpha, dt, a, pin, theta, s_prev[:, sl],
                                            s_cur[:, sl], emu, _pressure(batch, b) / m, _batch_sphere(batch, b))
    return out, dv


def batch_cnn_backward(batch, ch, alpha, dt, theta, s_prev, s_cur, g_next):
    gc = np.zeros((6, s_cur.shape[1]))
    gp = np.zeros_like(gc)
    gt = np.zeros(np.asarray(theta).size)
    for b in range(batch.n):
        H, W, h, m, a, pin = _inst(batch, b)
        sl = batch.instance(b)
        c, p, t = cnn_backward(H, W, ch, alpha, dt, pin, theta, s_prev[:, sl], s_cur[:, sl], g_next[:, sl],
                               _pressure(batch, b) / m, a, _batch_sphere(batch, b))
        gc[:, sl] += c
        gp[:, sl] += p
        gt += t
    return gc, gp, gt


def batch_pair_forward(batch, alpha, dt, theta, s_cur):
    s_cur = _f64(s_cur)
    out = np.empty_like(s_cur)
    dv = np.empty((3, s_cur.shape[1]))
    for b in range(batch.n):
        H, W, h, m, a, pin = _inst(batch, b)
        sl = batch.instance(b)
        out[:, sl], dv[:, sl] = pair_forward(H, W, alpha, dt, a, pin, theta, s_cur[:, sl], _pressure(batch, b) / m,
                                             _batch_sphere(batch, b))
    return out, dv


def batch_pair_backward(batch, alpha, dt, theta, s_cur, g_next):
    gc = np.zeros((6, s_cur.shape[1]))
    gt = np.zeros(np.asarray(theta).size)
    for b in range(batch.n):
        H, W, h, m, a, pin = _inst(batch, b)
        sl = batch.instance(b)
        c, t = pair_backward(H, W, alpha, dt, pin, theta, s_cur[:, sl], g_next[:, sl], _pressure(batch, b) / m,
                             a, _batch_sphere(batch, b))
        gc[:, sl] += c
        gt += t
    return gc, gt
