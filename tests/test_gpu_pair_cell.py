"""GPU parity of the pair cell (section 3.2's own cell read literally, PECNN_CELL_PAIR) against the
FP64 oracle: one frame on ragged and 16-byte-aligned batches (some instances with a pressure),
every tile configuration bit for bit, the backward pass, the rollout, and the trainer's BPTT
gradient. Tolerances as for the FP32 convolution cell: 1e-5 relative on the state and on the
velocity increment, 1e-5 on gradients, also through a 3-frame BPTT chain."""
import numpy as np
import pytest

import oracle
from paper_2403_12820_amd import inputs as I
from tests.gpu_util import SIZE_SETS, dev_tensor, perturbed_batch, rel_inf

pytestmark = pytest.mark.gpu
MAT = I.Material()
DT = 5e-3


@pytest.fixture(scope="module")
def L():
    from paper_2403_12820_amd import _lib
    _lib.lib()
    return _lib


def _inputs(sizes, seed, pressure=True):
    batch = perturbed_batch(sizes, seed=seed, vel=0.3, pos=0.2)
    if pressure:
        batch.pressure = np.array([0.0 if b % 3 == 0 else 2.0 * (b % 5 - 2) for b in range(batch.n)], np.float32)
    th = I.init_pair_theta(seed=seed + 1).astype(np.float64)
    th[12:48] += I.random_array((36,), seed=seed + 2, scale=0.05)   # branch weights well away from 0
    th[48:51] = [0.01, -0.02, 0.03]
    return batch, th.astype(np.float32)


def _model(L, th):
    return L.make_model(dev_tensor(th), 12, L.PECNN_FP32, dt=DT, cell=L.CELL_PAIR)


def _forward(L, batch, th, cfg=None):
    import torch
    plan = L.Plan.from_batch(batch)
    if cfg is not None:
        plan.set_tiles(ms_cfg=cfg)
    out = torch.zeros(6, batch.total, device="cuda")
    s = dev_tensor(batch.state)
    L.pecnn_forward(plan, _model(L, th), torch.full_like(s, float("nan")), s, out)  # S^{k-1} is not read
    torch.cuda.synchronize()
    return out.cpu().numpy().astype(np.float64)


def _increment(batch, s, out):
    a = np.repeat(batch.a_ext.astype(np.float64), np.diff(batch.node_off), axis=0).T
    d = out[3:] - s[3:].astype(np.float64) - DT * a
    d[:, batch.pin == 1] = 0.0
    return d


@pytest.mark.parametrize("sizes_kind", ["ragged", "aligned", "wide"])
def test_pair_forward_matches_oracle(L, sizes_kind):
    batch, th = _inputs(SIZE_SETS[sizes_kind]() + [(32, 32)], 800)
    got = _forward(L, batch, th)
    ref, _ = oracle.batch_pair_forward(batch, 1.0, DT, th.astype(np.float64), batch.state)
    assert rel_inf(got[3:], ref[3:]) <= 1e-5
    assert rel_inf(got[:3], ref[:3]) <= 1e-6
    assert rel_inf(_increment(batch, batch.state, got), _increment(batch, batch.state, ref)) <= 1e-5


def test_pair_tile_configs_bitwise_equal(L):
    batch, th = _inputs(SIZE_SETS["aligned"](), 801)
    outs = [_forward(L, batch, th, cfg) for cfg in range(5)]
    for o in outs[1:]:
        assert np.array_equal(o, outs[0])


def test_pair_backward_matches_oracle(L):
    import torch
    batch, th = _inputs([(8, 8), (17, 23), (1, 2), (5, 3), (6, 9)], 802)
    gn = I.random_array((6, batch.total), seed=803).astype(np.float32)
    plan = L.Plan.from_batch(batch)
    model = _model(L, th)
    s = dev_tensor(batch.state)
    gc = torch.zeros(6, batch.total, device="cuda")
    gp = torch.zeros_like(gc)
    gt = torch.zeros(51, device="cuda")
    L.pecnn_backward(plan, model, s, s, dev_tensor(gn), gc, gp, gt)
    torch.cuda.synchronize()
    rc, rt = oracle.batch_pair_backward(batch, 1.0, DT, th.astype(np.float64), batch.state.astype(np.float64),
                                        gn.astype(np.float64))
    assert rel_inf(gc.cpu().numpy(), rc) <= 1e-5, rel_inf(gc.cpu().numpy(), rc)
    assert rel_inf(gt.cpu().numpy(), rt) <= 1e-5, rel_inf(gt.cpu().numpy(), rt)
    assert np.all(gp.cpu().numpy() == 0.0)  # the cell does not read S^{k-1}
    # deterministic, and accumulating
    L.pecnn_backward(plan, model, s, s, dev_tensor(gn), gc, None, gt)
    torch.cuda.synchronize()
    assert rel_inf(gt.cpu().numpy(), 2 * rt) <= 1e-5, rel_inf(gt.cpu().numpy(), 2 * rt)


def test_pair_rollout_equals_forward_loop(L):
    import torch
    batch, th = _inputs([(40, 70), (16, 16), (3, 9), (20, 12)], 804)
    plan = L.Plan.from_batch(batch)
    model = _model(L, th)
    s0 = dev_tensor(batch.state)
    bufs = [s0.clone(), s0.clone(), torch.zeros_like(s0)]
    for _ in range(7):
        L.pecnn_forward(plan, model, bufs[0], bufs[1], bufs[2])
        bufs = [bufs[1], bufs[2], bufs[0]]
    torch.cuda.synchronize()
    rp, rc = bufs[0].cpu().numpy(), bufs[1].cpu().numpy()
    g = L.Guard()
    # bounds no instance reaches: the checks (and their reductions) run, nothing falls back
    g.stretch_max, g.energy_gain_max, g.check_every, g.substeps = 1e30, 1e30, 3, 10
    fb = torch.zeros(batch.n, dtype=torch.int32, device="cuda")
    for _ in range(2):  # the second call replays cached graphs
        a, b = s0.clone(), s0.clone()
        L.pecnn_rollout(plan, model, L.ms_params(MAT), g, a, b, 7, fb, None)
        torch.cuda.synchronize()
        assert np.array_equal(a.cpu().numpy(), rp) and np.array_equal(b.cpu().numpy(), rc)
        assert np.all(fb.cpu().numpy() == 0)


def test_pair_trainer_gradient_matches_oracle_chain(L):
    """The trainer's loss and theta gradient over a 3-frame unroll (one-step weight 1) equal the
    oracle's chain of pair-cell frames and reverse passes."""
    import torch
    from paper_2403_12820_amd.train import Trainer
    U = 3
    batch, th = _inputs([(8, 8), (6, 10)], 805, pressure=False)
    s1 = batch.state.astype(np.float64)
    targets = [s1 + I.random_array(s1.shape, seed=810 + t, scale=0.01) for t in range(U)]
    frames = np.stack([s1, s1] + targets).astype(np.float32)
    sx, sv = 0.01, 0.05
    n_free = int((batch.pin == 0).sum())
    plan = L.Plan.from_batch(batch)
    tr = Trainer(dt_nn=DT, theta=th, cell="pair")
    tr.gradient(torch.tensor(frames, device="cuda"), plan, n_free, sx, sv)
    torch.cuda.synchronize()
    th64 = th.astype(np.float64)
    states = [frames[1].astype(np.float64)]
    og = [np.zeros_like(s1) for _ in range(U + 1)]
    lv = 0.0
    for t in range(U):
        sn, _ = oracle.batch_pair_forward(batch, 1.0, DT, th64, states[-1])
        states.append(sn)
        v, gg = oracle.loss_mse(batch.pin, n_free, sx, sv, 1.0 / U + (1.0 if t == 0 else 0.0), sn,
                                frames[t + 2].astype(np.float64))
        lv += v
        og[t + 1] += gg
    gt = np.zeros(51)
    for t in range(U - 1, -1, -1):
        gc, g_t = oracle.batch_pair_backward(batch, 1.0, DT, th64, states[t], og[t + 1])
        if t >= 1:
            og[t] += gc
        gt += g_t
    assert abs(tr.loss.item() - lv) <= 1e-5 * abs(lv)
    assert rel_inf(tr.g.cpu().numpy(), gt) <= 1e-5, rel_inf(tr.g.cpu().numpy(), gt)


def test_pair_model_validation(L):
    import torch
    batch, th = _inputs([(8, 8)], 806, pressure=False)
    plan = L.Plan.from_batch(batch)
    s = dev_tensor(batch.state)
    out = torch.zeros_like(s)
    bad = L.make_model(dev_tensor(th), 16, L.PECNN_FP32, dt=DT, cell=L.CELL_PAIR)
    with pytest.raises(L.PecnnError):
        L.pecnn_forward(plan, bad, s, s, out)
    bad = L.make_model(dev_tensor(th), 12, L.PECNN_BF16, dt=DT, cell=L.CELL_PAIR)
    with pytest.raises(L.PecnnError):
        L.pecnn_forward(plan, bad, s, s, out)
    assert L.lib().pecnn_cell_theta_size(L.CELL_PAIR, 12) == 51
    assert L.lib().pecnn_cell_theta_size(L.CELL_CONV, 32) == I.theta_size(32)
