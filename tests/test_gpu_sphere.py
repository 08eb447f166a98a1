"""GPU parity with a sphere in the constraint of eq. (5) (pecnn_plan_set_spheres) against the FP64
oracle: the mass-spring step and the three frames (bf16 and FP32 convolution cell, pair cell) on
ragged and aligned batches where a cap of each cloth penetrates its sphere, every tile
configuration bit for bit, the rollout, the reverse pass through the constraint (both cells, FP32)
and the error paths.

Whether a node is inside the sphere is decided in FP32 on the GPU and in FP64 in the oracle; nodes
whose updated position lies within a small margin of the surface (1e-5 of the radius for FP32
updates, 1e-3 for the bf16 frame) can be decided differently and are left out of the comparison;
the tests check that they are few and that many nodes were projected."""
import numpy as np
import pytest

import oracle
from paper_2403_12820_amd import inputs as I
from tests.gpu_util import SIZE_SETS, dev_tensor, ms_velocity_floor, perturbed_batch, rel_inf

pytestmark = pytest.mark.gpu
MAT = I.Material()


@pytest.fixture(scope="module")
def L():
    from paper_2403_12820_amd import _lib
    _lib.lib()
    return _lib


def _with_spheres(batch):
    """A ball under the middle of every instance but each fourth, its top 0.02 m above the flat
    cloth, with friction 0, 0.5 or 1."""
    sph = np.zeros((batch.n, 5), np.float32)
    for b in range(batch.n):
        if b % 4 == 3:
            continue
        h = float(batch.h[b])
        R = 0.3
        sph[b] = [(batch.W[b] - 1) * h / 2, (batch.H[b] - 1) * h / 2, -R + 0.02, R, (b % 3) / 2.0]
    batch.sphere = sph
    return batch


def _margin(batch, y):
    """|y - c| - R per node (inf where the instance has no sphere)."""
    m = np.full(batch.total, np.inf)
    for b in range(batch.n):
        if batch.sphere[b, 3] > 0:
            sl = batch.instance(b)
            c = batch.sphere[b, :3].astype(np.float64)
            m[sl] = np.linalg.norm(y[:, sl] - c[:, None], axis=0) - batch.sphere[b, 3]
    return m


def _ms(L, batch, s, cfg=None):
    import torch
    plan = L.Plan.from_batch(batch)
    if cfg is not None:
        plan.set_tiles(ms_cfg=cfg)
    a = dev_tensor(s)
    out = torch.zeros_like(a)
    L.cloth_ms_step(plan, L.ms_params(MAT), a, out, 1)
    torch.cuda.synchronize()
    return out.cpu().numpy().astype(np.float64)


@pytest.mark.parametrize("sizes_kind", ["ragged", "aligned"])
def test_ms_step_with_spheres_matches_oracle(L, sizes_kind):
    batch = _with_spheres(perturbed_batch(SIZE_SETS[sizes_kind]() + [(32, 32)], seed=900))
    got = _ms(L, batch, batch.state)
    ref = oracle.batch_ms_step(batch, batch.state, MAT, 1)
    free_y = oracle.batch_ms_step(_plain(batch), batch.state, MAT, 1)[:3]
    margin = _margin(batch, free_y)
    ok = np.abs(margin) > 1e-5 * 0.3
    inside = (margin < 0) & (batch.pin == 0)
    assert inside.sum() >= 20 and (~ok).sum() <= 2, (inside.sum(), (~ok).sum())
    width = max((w - 1) * h for w, h in zip(batch.W, batch.h))
    assert np.abs(got[:3, ok] - ref[:3, ok]).max() <= 1e-5 * width
    tol_v = max(1e-5 * np.abs(ref[3:]).max(), ms_velocity_floor(batch, MAT))
    assert np.abs(got[3:, ok] - ref[3:, ok]).max() <= tol_v
    # the projected nodes sit on their spheres
    assert np.abs(_margin(batch, got[:3])[inside & ok]).max() <= 1e-6


def _plain(batch):
    """The same batch without spheres."""
    import copy
    b = copy.copy(batch)
    b.sphere = None
    return b


def test_ms_sphere_tile_configs_bitwise_equal(L):
    batch = _with_spheres(perturbed_batch(SIZE_SETS["aligned"](), seed=901))
    outs = [_ms(L, batch, batch.state, cfg) for cfg in range(5)]
    for o in outs[1:]:
        assert np.array_equal(o, outs[0])


def _frame_inputs(sizes, seed, ch=32, scale=10.0):
    batch = _with_spheres(perturbed_batch(sizes, seed=seed, vel=0.05, pos=0.15))
    s1 = batch.state.astype(np.float64)
    s0 = s1.copy()
    s0[:3] -= 5e-3 * s1[3:]
    th = (I.init_theta(ch, seed=seed + 1).astype(np.float64) * scale).astype(np.float32)
    return batch, s0.astype(np.float32), s1.astype(np.float32), th


def _frame(L, batch, s0, s1, model_args, cfg=None):
    import torch
    plan = L.Plan.from_batch(batch)
    if cfg is not None:
        plan.set_tiles(cnn_cfg=cfg)
    th, ch, prec, cell = model_args
    model = L.make_model(dev_tensor(th), ch, prec, dt=5e-3, cell=cell)
    out = torch.zeros(6, batch.total, device="cuda")
    L.pecnn_forward(plan, model, dev_tensor(s0), dev_tensor(s1), out)
    torch.cuda.synchronize()
    return out.cpu().numpy().astype(np.float64)


@pytest.mark.parametrize("kind", ["fp32", "bf16", "pair"])
def test_frames_with_spheres_match_oracle(L, kind):
    batch, s0, s1, th = _frame_inputs(SIZE_SETS["aligned"]() + [(32, 32)], 910)
    if kind == "pair":
        th = I.init_pair_theta(seed=911)
        args = (th, 12, L.PECNN_FP32, L.CELL_PAIR)
        ref, _ = oracle.batch_pair_forward(batch, 1.0, 5e-3, th.astype(np.float64), s1)
        free, _ = oracle.batch_pair_forward(_plain(batch), 1.0, 5e-3, th.astype(np.float64), s1)
    else:
        prec = L.PECNN_BF16 if kind == "bf16" else L.PECNN_FP32
        args = (th, 32, prec, L.CELL_CONV)
        emu = 7 if kind == "bf16" else 0
        ref, _ = oracle.batch_cnn_forward(batch, 32, 1.0, 5e-3, th.astype(np.float64), s0, s1, emu=emu)
        free, _ = oracle.batch_cnn_forward(_plain(batch), 32, 1.0, 5e-3, th.astype(np.float64), s0, s1, emu=emu)
    got = _frame(L, batch, s0, s1, args)
    margin = _margin(batch, free[:3])
    ok = np.abs(margin) > (1e-3 if kind == "bf16" else 1e-5) * 0.3
    inside = (margin < 0) & (batch.pin == 0)
    assert inside.sum() >= 20 and (~ok).sum() <= 0.05 * max(inside.sum(), 1), (inside.sum(), (~ok).sum())
    tol = 2.0 ** -8 if kind == "bf16" else 1e-5
    assert rel_inf(got[3:, ok], ref[3:, ok]) <= tol
    assert np.abs(got[:3, ok] - ref[:3, ok]).max() <= (1e-4 if kind == "bf16" else 1e-6)
    assert np.abs(_margin(batch, got[:3])[inside & ok]).max() <= 1e-6


def test_rollout_with_spheres_equals_forward_loop(L):
    import torch
    batch, s0, s1, th = _frame_inputs([(40, 70), (16, 16), (3, 9), (20, 12)], 920, scale=5.0)
    plan = L.Plan.from_batch(batch)
    model = L.make_model(dev_tensor(th), 32, L.PECNN_BF16, dt=5e-3)
    bufs = [dev_tensor(s0), dev_tensor(s1), torch.zeros(6, batch.total, device="cuda")]
    for _ in range(6):
        L.pecnn_forward(plan, model, bufs[0], bufs[1], bufs[2])
        bufs = [bufs[1], bufs[2], bufs[0]]
    torch.cuda.synchronize()
    rp, rc = bufs[0].cpu().numpy(), bufs[1].cpu().numpy()
    g = L.Guard()
    g.stretch_max, g.energy_gain_max, g.check_every, g.substeps = 1e30, 1e30, 3, 10
    fb = torch.zeros(batch.n, dtype=torch.int32, device="cuda")
    for _ in range(2):
        a, b = dev_tensor(s0), dev_tensor(s1)
        L.pecnn_rollout(plan, model, L.ms_params(MAT), g, a, b, 6, fb, None)
        torch.cuda.synchronize()
        assert np.array_equal(a.cpu().numpy(), rp) and np.array_equal(b.cpu().numpy(), rc)


def test_sphere_errors(L):
    import torch
    batch = _with_spheres(perturbed_batch([(8, 8), (6, 6)], seed=930))
    plan = L.Plan.from_batch(batch)
    th = I.init_theta(16, seed=1)
    model = L.make_model(dev_tensor(th), 16, L.PECNN_FP32, dt=5e-3)
    s = dev_tensor(batch.state)
    with pytest.raises(L.PecnnError):
        plan.set_spheres([[0, 0, 0, 1.0, 1.5], [0, 0, 0, 1.0, 0.0]])   # friction above 1
    with pytest.raises(L.PecnnError):
        plan.set_spheres([[0, 0, 0, -1.0, 0.5], [0, 0, 0, 1.0, 0.0]])  # negative radius
    plan.set_spheres(np.zeros((2, 5)))
    small = plan.workspace(L.WS_BACKWARD, model)  # sized without spheres
    plan.set_spheres(batch.sphere)
    assert plan.workspace(L.WS_BACKWARD, model).numel() > small.numel()
    with pytest.raises(L.PecnnError):  # the reverse pass through spheres needs the larger workspace
        L.pecnn_backward(plan, model, s, s, torch.zeros_like(s), None, None, torch.zeros(th.size, device="cuda"),
                         ws=small)
    L.pecnn_backward(plan, model, s, s, torch.zeros_like(s), None, None, torch.zeros(th.size, device="cuda"))
    torch.cuda.synchronize()


def _sphere_pressures(n):
    """Zero on every third instance, otherwise +-20 or +-40 N/m^2."""
    return np.array([0.0 if b % 3 == 0 else 20.0 * (1 + b % 2) * (1 if b % 4 < 2 else -1) for b in range(n)],
                    np.float32)


@pytest.mark.parametrize("cell,pressure", [("conv", False), ("pair", False), ("conv", True), ("pair", True)])
def test_backward_with_spheres_matches_oracle(L, cell, pressure):
    """The reverse pass through each instance's sphere against the oracle's, FP32, without and
    with the pressure of eq. (3) on some instances (the frame recomputed without spheres then
    takes the kernels' pressure variant). The output adjoint is zeroed at nodes the two sides
    might send down different branches of the constraint: an updated position within 1e-5 R of
    the surface, or a normal velocity within 1e-4 of the speed of zero."""
    import torch
    batch, s0, s1, th = _frame_inputs(SIZE_SETS["aligned"]() + [(32, 32), (17, 23)], 940)
    if pressure:
        batch.pressure = _sphere_pressures(batch.n)
    if cell == "pair":
        th = I.init_pair_theta(seed=941).astype(np.float32)
        ch, c = 12, L.CELL_PAIR
        free, _ = oracle.batch_pair_forward(_plain(batch), 1.0, 5e-3, th.astype(np.float64), s1)
    else:
        ch, c = 32, L.CELL_CONV
        free, _ = oracle.batch_cnn_forward(_plain(batch), 32, 1.0, 5e-3, th.astype(np.float64), s0, s1)
    margin = _margin(batch, free[:3])
    vn = np.zeros(batch.total)
    for b in range(batch.n):
        if batch.sphere[b, 3] > 0:
            sl = batch.instance(b)
            d = free[:3, sl] - batch.sphere[b, :3].astype(np.float64)[:, None]
            vn[sl] = np.sum(free[3:, sl] * d, axis=0) / np.maximum(np.linalg.norm(d, axis=0), 1e-30)
    speed = np.linalg.norm(free[3:], axis=0)
    unsure = (np.abs(margin) <= 1e-5 * 0.3) | ((margin < 0) & (np.abs(vn) <= 1e-4 * speed))
    inside = (margin < 0) & (batch.pin == 0) & ~unsure
    assert inside.sum() >= 20 and unsure.sum() <= 0.05 * inside.sum(), (inside.sum(), unsure.sum())
    gn = I.random_array((6, batch.total), seed=942)
    gn[:, unsure] = 0.0
    gn = gn.astype(np.float32)
    plan = L.Plan.from_batch(batch)
    model = L.make_model(dev_tensor(th.astype(np.float32)), ch, L.PECNN_FP32, dt=5e-3, cell=c)
    gc = torch.zeros(6, batch.total, device="cuda")
    gp = torch.zeros_like(gc)
    gt = torch.zeros(th.size, device="cuda")
    L.pecnn_backward(plan, model, dev_tensor(s0), dev_tensor(s1), dev_tensor(gn), gc, gp, gt)
    torch.cuda.synchronize()
    args64 = [a.astype(np.float64) for a in (th, s0, s1, gn)]
    if cell == "pair":
        rc, rt = oracle.batch_pair_backward(batch, 1.0, 5e-3, args64[0], args64[2], args64[3])
        rp = np.zeros_like(rc)
        rt0 = oracle.batch_pair_backward(_plain(batch), 1.0, 5e-3, args64[0], args64[2], args64[3])[1]
    else:
        rc, rp, rt = oracle.batch_cnn_backward(batch, 32, 1.0, 5e-3, *args64)
        rt0 = oracle.batch_cnn_backward(_plain(batch), 32, 1.0, 5e-3, *args64)[2]
    got_t = gt.cpu().numpy()
    assert rel_inf(gc.cpu().numpy(), rc) <= 1e-5, rel_inf(gc.cpu().numpy(), rc)
    assert rel_inf(gp.cpu().numpy(), rp) <= 1e-5, rel_inf(gp.cpu().numpy(), rp)
    assert rel_inf(got_t, rt) <= 1e-5, rel_inf(got_t, rt)
    assert rel_inf(got_t, rt0) > 1e-2  # the spheres matter to the gradient
