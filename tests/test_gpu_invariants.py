"""Invariants of the plain method re-run on the GPU (section 3.1, eqs. 1, 2, 4, 5), each against the
FP64 oracle, which the CPU pins fix:

  * energy drift without damping: the 32 x 32 two-corner scene with mu = d = 0 and no wind, 400
    steps of dt = 5e-4. The GPU energy curve (FP64 reduction of the FP32 state every 10 steps)
    follows the oracle's curve within 1e-5 of E_ref = M |g| width, and neither drifts;
  * momentum: no pins, no gravity, no drag and no wind, so the spring and spring-damping forces
    cancel in pairs and the total momentum stays at its start value;
  * translation invariance: every position (pins included) shifted by c gives the same motion
    shifted by c, for the mass-spring step and for the CNN frame.
"""
import numpy as np
import pytest

import oracle
from paper_2403_12820_amd import inputs as I
from tests.gpu_util import dev_tensor, perturbed_batch, rel_inf

pytestmark = pytest.mark.gpu

SHIFT = np.array([0.37, -1.25, 2.5])


@pytest.fixture(scope="module")
def L():
    from paper_2403_12820_amd import _lib
    _lib.lib()
    return _lib


def test_energy_drift_curve_matches_oracle(L):
    import torch
    mat = I.Material(mu=0.0, drag=0.0)
    sc = I.make_scene(32, 32, "two_top_corners", noise_sigma=1e-3, seed=0, mat=mat)
    batch = I.make_batch([sc])
    plan = L.Plan.from_batch(batch)
    P = L.ms_params(mat)
    ws = plan.workspace(L.WS_MS_STEP)
    a = dev_tensor(sc.state)
    b = torch.empty_like(a)
    out = torch.zeros(4, dtype=torch.float64, device="cuda")
    e_gpu = []
    for k in range(41):
        if k:
            L.cloth_ms_step(plan, P, a, b, 10, ws=ws)
            a, b = b, a
        L.cloth_reduce_fp64(plan, P, a, None, out)
        torch.cuda.synchronize()
        e_gpu.append(out[1].item())
    s = sc.state.astype(np.float64)
    e_ref = []
    for k in range(41):
        if k:
            s = oracle.ms_run(32, 32, sc.h, sc.mass, sc.a_ext, sc.pin, s, mat, 10)
        e_ref.append(oracle.energy(32, 32, sc.h, sc.mass, sc.a_ext, s, mat))
    e_gpu, e_ref = np.array(e_gpu), np.array(e_ref)
    E_ref = 1024 * sc.mass * 9.8 * 31 * sc.h
    dev = np.abs(e_gpu - e_ref).max() / E_ref
    assert dev <= 1e-5, dev
    # no secular drift in either curve over the 0.2 s
    assert np.abs(e_ref - e_ref[0]).max() <= 1e-3 * E_ref
    assert np.abs(e_gpu - e_gpu[0]).max() <= 1e-3 * E_ref


def _free_batch(seed):
    mat = I.Material(g=(0.0, 0.0, 0.0), drag=0.0)
    scenes = [I.make_scene(H, W, "none", noise_sigma=0.0, mat=mat) for H, W in [(20, 24), (7, 33), (1, 2)]]
    batch = I.make_batch(scenes)
    s = batch.state.astype(np.float64)
    s[:3] += I.random_array((3, batch.total), seed=seed, scale=0.05 * mat.h)
    s[3:] = I.random_array((3, batch.total), seed=seed + 1, scale=0.2)
    batch.state = s.astype(np.float32)
    return batch, mat


def test_momentum_conserved_gpu(L):
    """200 steps of free cloths: per instance, sum m v stays at its start value up to FP32
    rounding of the per-node updates, here held to 1e-4 of sum m |v|. A momentum-breaking
    error (a spring force applied to one end only) moves it by a fraction of order one."""
    import torch
    batch, mat = _free_batch(40)
    plan = L.Plan.from_batch(batch)
    P = L.ms_params(mat)
    a = dev_tensor(batch.state)
    b = torch.empty_like(a)
    L.cloth_ms_step(plan, P, a, b, 200, ws=plan.workspace(L.WS_MS_STEP))
    torch.cuda.synchronize()
    got = b.cpu().numpy().astype(np.float64)
    s0 = batch.state.astype(np.float64)
    for k in range(batch.n):
        sl = batch.instance(k)
        p0 = s0[3:, sl].sum(axis=1)
        p1 = got[3:, sl].sum(axis=1)
        scale = max(np.abs(s0[3:, sl]).sum(), np.abs(got[3:, sl]).sum())
        assert np.abs(p1 - p0).max() <= 1e-4 * scale, (k, p1 - p0, scale)
    # the oracle conserves it to FP64 rounding (the CPU pin), and the GPU run follows the oracle
    ref = oracle.batch_ms_step(batch, batch.state, mat, 200)
    width = max((w - 1) * h for w, h in zip(batch.W, batch.h))
    assert np.abs(got[:3] - ref[:3]).max() <= 1e-5 * width


def test_translation_invariance_ms_gpu(L):
    """10 steps of pinned, wind-blown cloths: shifting every position by c shifts the result by c
    (within FP32 rounding of the larger coordinates: 1e-5 of the width), and each run follows the
    oracle from its own (rounded) inputs. The run is kept short: the stiff springs amplify the
    FP32 rounding of positions (a few 1e-7 m at |x| ~ 2.5 m), and over 100 steps of the shifted
    cloth the state drifts about 1e-4 of the width from the FP64 run; the unshifted 400-step run
    of the plain-method scene is held to 1e-5 elsewhere."""
    import torch
    batch = perturbed_batch([(17, 23), (32, 32), (2, 9)], seed=41)
    mat = I.Material()
    plan = L.Plan.from_batch(batch)
    P = L.ms_params(mat)
    ws = plan.workspace(L.WS_MS_STEP)
    width = max((w - 1) * h for w, h in zip(batch.W, batch.h))
    res = []
    for c in (np.zeros(3), SHIFT):
        s = batch.state.astype(np.float64)
        s[:3] += c[:, None]
        s = s.astype(np.float32)
        a = dev_tensor(s)
        b = torch.empty_like(a)
        L.cloth_ms_step(plan, P, a, b, 10, ws=ws)
        torch.cuda.synchronize()
        out = b.cpu().numpy().astype(np.float64)
        ref = oracle.batch_ms_step(batch, s, mat, 10)
        assert np.abs(out[:3] - ref[:3]).max() <= 1e-5 * width
        out[:3] -= c[:, None]
        res.append(out)
    assert np.abs(res[1][:3] - res[0][:3]).max() <= 1e-5 * width


@pytest.mark.parametrize("prec", [0, 1])
def test_translation_invariance_cnn_gpu(L, prec):
    """The frame reads positions only through differences with the centre node (eq. 6 with the
    two-point correlations of section 3.2), so a shift of every position by c shifts S^{k+1} by c
    and leaves its velocities unchanged up to the rounding of the shifted FP32 inputs. Each run is
    also held to the oracle from its own inputs: 1e-5 relative in FP32, the bf16 bound (2^-8 of
    the output scale) against the emulated-bf16 oracle."""
    import torch
    batch = perturbed_batch([(17, 23), (33, 68), (2, 9)], seed=42, vel=0.1)
    s1 = batch.state.astype(np.float64)
    s0 = s1.copy()
    s0[:3] -= 5e-3 * s1[3:]
    th = (I.init_theta(32, seed=43).astype(np.float64) * 20).astype(np.float32)
    plan = L.Plan.from_batch(batch)
    model = L.make_model(dev_tensor(th), 32, prec, dt=5e-3)
    width = max((w - 1) * h for w, h in zip(batch.W, batch.h))
    res = []
    for c in (np.zeros(3), SHIFT):
        a, b = s0.copy(), s1.copy()
        a[:3] += c[:, None]
        b[:3] += c[:, None]
        a, b = a.astype(np.float32), b.astype(np.float32)
        ta, tb = dev_tensor(a), dev_tensor(b)
        out = torch.empty_like(tb)
        L.pecnn_forward(plan, model, ta, tb, out)
        torch.cuda.synchronize()
        o = out.cpu().numpy().astype(np.float64)
        ref, _ = oracle.batch_cnn_forward(batch, 32, 1.0, 5e-3, th.astype(np.float64), a, b, emu=7 if prec else 0)
        inc, inc_ref = o[3:] - b[3:], ref[3:] - b[3:]
        assert rel_inf(inc, inc_ref) <= (1e-5 if prec == 0 else 2.0 ** -8), rel_inf(inc, inc_ref)
        o[:3] -= c[:, None]
        res.append(o)
    assert np.abs(res[1][:3] - res[0][:3]).max() <= 1e-5 * width
