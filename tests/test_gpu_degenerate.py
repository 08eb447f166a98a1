"""Degenerate cases on the GPU against the oracle and against what eq. (5) fixes.

* A rollout of zero frames touches nothing.
* Cloths pinned at every node (a one-row cloth pinned along its top edge, 2 x 2 pinned at its
  four corners, a single spring with both ends pinned) keep their positions under the
  simulator step and every frame, with zero velocity. The reverse pass then gives theta no
  gradient. The input gradient is the direct term of eq. (5): the new position is the old one,
  and the new velocity is zero.
* These cloths sit beside ordinary ones in the same batch, which must be unaffected."""
import numpy as np
import pytest

import oracle
from paper_2403_12820_amd import inputs as I
from tests.gpu_util import dev_tensor, rel_inf

pytestmark = pytest.mark.gpu
MAT = I.Material()
DT = 5e-3


@pytest.fixture(scope="module")
def L():
    from paper_2403_12820_amd import _lib
    _lib.lib()
    return _lib


def _batch():
    """Pinned everywhere: 1 x 9 (top edge), 2 x 2 (four corners), 1 x 2 (top edge); and two
    ordinary cloths."""
    scenes = [I.make_scene(1, 9, "top_edge", wind=(0.5, 0.2, 0.0), seed=1),
              I.make_scene(12, 17, "two_top_corners", wind=(0.3, -0.4, 0.0), seed=2),
              I.make_scene(2, 2, "four_corners", seed=3),
              I.make_scene(1, 2, "top_edge", seed=4),
              I.make_scene(9, 8, "one_top_corner", seed=5)]
    batch = I.make_batch(scenes)
    s = batch.state.astype(np.float64)
    s[:3] += I.random_array((3, batch.total), seed=6, scale=0.004)
    s[3:] = I.random_array((3, batch.total), seed=7, scale=0.1)
    s[3:, batch.pin == 1] = 0.0  # a pinned node is at rest
    batch.state = s.astype(np.float32)
    return batch


ALL_PINNED = (0, 2, 3)


def test_zero_frame_rollout_touches_nothing(L):
    import torch
    batch = _batch()
    plan = L.Plan.from_batch(batch)
    th = I.init_theta(32, seed=1)
    model = L.make_model(dev_tensor(th), 32, L.PECNN_BF16, dt=DT)
    g = L.Guard()
    g.stretch_max, g.energy_gain_max, g.check_every, g.substeps = 2.0, 0.2, 1, 10
    a, b = dev_tensor(batch.state), dev_tensor(batch.state * 1.5)
    fb = torch.full((batch.n,), 7, dtype=torch.int32, device="cuda")
    stats = torch.full((4 * batch.n,), 3.0, dtype=torch.float64, device="cuda")
    L.pecnn_rollout(plan, model, L.ms_params(MAT), g, a, b, 0, fb, stats)
    torch.cuda.synchronize()
    assert np.array_equal(a.cpu().numpy(), batch.state)
    assert np.array_equal(b.cpu().numpy(), batch.state * np.float32(1.5))
    assert np.all(fb.cpu().numpy() == 7) and np.all(stats.cpu().numpy() == 3.0)


def _pinned_ok(batch, out, s):
    for b in ALL_PINNED:
        sl = batch.instance(b)
        assert np.array_equal(out[:3, sl], s[:3, sl]), b
        assert np.all(out[3:, sl] == 0.0), b


def test_pinned_cloths_stay_put_in_every_step(L):
    import torch
    batch = _batch()
    plan = L.Plan.from_batch(batch)
    s1 = batch.state
    s0 = s1.copy()
    s0[:3] -= np.float32(DT) * s1[3:]
    # simulator step
    out = torch.zeros(6, batch.total, device="cuda")
    L.cloth_ms_step(plan, L.ms_params(MAT), dev_tensor(s1), out, 1)
    torch.cuda.synchronize()
    got = out.cpu().numpy()
    _pinned_ok(batch, got, s1)
    ref = oracle.batch_ms_step(batch, s1, MAT, 1)
    width = max((w - 1) * h for w, h in zip(batch.W, batch.h))
    assert np.abs(got[:3] - ref[:3]).max() <= 1e-5 * width
    # the three frames
    th = (I.init_theta(32, seed=8).astype(np.float64) * 20).astype(np.float32)
    pth = I.init_pair_theta(seed=9)
    for prec, cell, theta, ch in ((L.PECNN_BF16, L.CELL_CONV, th, 32), (L.PECNN_FP32, L.CELL_CONV, th, 32),
                                  (L.PECNN_FP32, L.CELL_PAIR, pth, 12)):
        model = L.make_model(dev_tensor(theta), ch, prec, dt=DT, cell=cell)
        out.zero_()
        L.pecnn_forward(plan, model, dev_tensor(s0), dev_tensor(s1), out)
        torch.cuda.synchronize()
        got = out.cpu().numpy()
        _pinned_ok(batch, got, s1)
        if cell == L.CELL_PAIR:
            ref, _ = oracle.batch_pair_forward(batch, 1.0, DT, pth.astype(np.float64), s1)
        else:
            ref, _ = oracle.batch_cnn_forward(batch, 32, 1.0, DT, th.astype(np.float64), s0, s1,
                                              emu=7 if prec == L.PECNN_BF16 else 0)
        assert rel_inf(got[3:], ref[3:]) <= (2.0 ** -8 if prec == L.PECNN_BF16 else 1e-5), (prec, cell)


def test_pinned_cloths_backward(L):
    """Only pinned cloths: theta gets no gradient, and g_cur is the direct term of eq. (5)."""
    import torch
    scenes = [I.make_scene(1, 9, "top_edge", seed=1), I.make_scene(2, 2, "four_corners", seed=3),
              I.make_scene(1, 2, "top_edge", seed=4)]
    batch = I.make_batch(scenes)
    assert np.all(batch.pin == 1)
    plan = L.Plan.from_batch(batch)
    s1 = batch.state
    gn = I.random_array((6, batch.total), seed=10).astype(np.float32)
    for cell, theta, ch in ((L.CELL_CONV, I.init_theta(32, seed=8) * 20, 32), (L.CELL_PAIR, I.init_pair_theta(seed=9), 12)):
        theta = theta.astype(np.float32)
        model = L.make_model(dev_tensor(theta), ch, L.PECNN_FP32, dt=DT, cell=cell)
        gc = torch.zeros(6, batch.total, device="cuda")
        gp = torch.zeros_like(gc)
        gt = torch.zeros(theta.size, device="cuda")
        L.pecnn_backward(plan, model, dev_tensor(s1), dev_tensor(s1), dev_tensor(gn), gc, gp, gt)
        torch.cuda.synchronize()
        assert np.all(gt.cpu().numpy() == 0.0), cell
        # x' = x: the position adjoint passes straight through; v' = 0: nothing flows to v
        g = gc.cpu().numpy()
        np.testing.assert_array_equal(g[:3], gn[:3])
        assert np.all(g[3:] == 0.0)
        assert np.all(gp.cpu().numpy() == 0.0)
