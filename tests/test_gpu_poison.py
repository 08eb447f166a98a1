"""GPU: NaN-poisoned workspaces and outputs. Every entry point that takes a workspace runs twice
on the same inputs, once with the workspace zero-filled and once with every byte 0xFF (NaN as
FP32 and FP64); outputs that the call overwrites are NaN-filled before both runs. The results must
agree bit for bit and be finite: a read of workspace memory the call did not write first, or an
output element it did not write, would show as a NaN or a difference."""
import numpy as np
import pytest

from paper_2403_12820_amd import inputs as I
from tests.gpu_util import aligned_sizes, dev_tensor, perturbed_batch, ragged_sizes

pytestmark = pytest.mark.gpu

MAT = I.Material()


@pytest.fixture(scope="module")
def L():
    from paper_2403_12820_amd import _lib
    _lib.lib()
    return _lib


def _twice(torch, ws, run):
    """run(ws) -> list of tensors; ws zero-filled, then 0xFF-filled."""
    outs = []
    for fill in (0, 255):
        if ws is not None:
            ws.fill_(fill)
        res = run(ws)
        torch.cuda.synchronize()
        outs.append([t.detach().cpu().numpy().copy() for t in res])
    for a, b in zip(*outs):
        assert np.all(np.isfinite(a)), "non-finite output"
        np.testing.assert_array_equal(a, b)
    return outs[0]


@pytest.mark.parametrize("sizes", [ragged_sizes, aligned_sizes])
def test_poisoned_workspaces_and_outputs(L, sizes):
    import torch
    batch = perturbed_batch(sizes() + [(64, 64)], seed=1500)
    plan = L.Plan.from_batch(batch)
    sim = L.ms_params(MAT)
    s0 = dev_tensor(batch.state)
    s1 = s0.clone()
    s1[3:] += dev_tensor(I.random_array((3, batch.total), seed=1501, scale=0.02).astype(np.float32))
    s1[:3] += 5e-3 * s1[3:]
    nan = float("nan")

    # mass-spring step, three steps through the workspace's intermediate state
    def ms(ws):
        out = torch.full_like(s0, nan)
        L.cloth_ms_step(plan, sim, s1, out, 3, ws=ws)
        return [out]
    _twice(torch, plan.workspace(L.WS_MS_STEP), ms)

    # both frames (no workspace): every node of s_next is written
    for ch, prec in ((16, L.PECNN_FP32), (32, L.PECNN_BF16)):
        th = torch.tensor(I.init_theta(ch, seed=3) * 5, device="cuda")
        model = L.make_model(th, ch, prec, dt=5e-3)

        def fwd(ws):
            out = torch.full_like(s0, nan)
            L.pecnn_forward(plan, model, s0, s1, out)
            return [out]
        _twice(torch, None, fwd)

    # backward: the factor table and the partial sums come from the workspace
    th = torch.tensor(I.init_theta(32, seed=4) * 5, device="cuda")
    model = L.make_model(th, 32, L.PECNN_FP32, dt=5e-3)
    gn = dev_tensor(I.random_array((6, batch.total), seed=1502).astype(np.float32))

    def bwd(ws):
        gc, gp = torch.zeros_like(s0), torch.zeros_like(s0)
        gt = torch.zeros(th.numel(), device="cuda")
        L.pecnn_backward(plan, model, s0, s1, gn, gc, gp, gt, ws=ws)
        return [gc, gp, gt]
    _twice(torch, plan.workspace(L.WS_BACKWARD, model), bwd)

    # FP64 diagnostics and the loss: partial sums in the workspace
    def red(ws):
        out = torch.full((4 * batch.n,), nan, dtype=torch.float64, device="cuda")
        L.cloth_reduce_fp64(plan, sim, s1, s0, out, ws=ws)
        return [out]
    _twice(torch, plan.workspace(L.WS_REDUCE), red)

    n_free = int((batch.pin == 0).sum())

    def loss(ws):
        lv = torch.zeros(1, dtype=torch.float64, device="cuda")
        g = torch.zeros_like(s0)
        L.pecnn_loss_mse(plan, s1, s0, 0.01, 0.1, 1.0, n_free, lv, g, ws=ws)
        return [lv, g]
    _twice(torch, plan.workspace(L.WS_REDUCE), loss)

    # the guarded rollout: graph-captured chunks, the guard's FP64 state and the third buffer
    model_b = L.make_model(torch.tensor(I.init_theta(32, seed=5) * 5, device="cuda"), 32, L.PECNN_BF16, dt=5e-3)
    g = L.Guard()
    g.stretch_max, g.energy_gain_max, g.check_every, g.substeps, g.frame_err_max = 1.05, 1e30, 2, 10, 0.0

    def roll(ws):
        a, b = s0.clone(), s1.clone()
        fb = torch.zeros(batch.n, dtype=torch.int32, device="cuda")
        st = torch.full((4 * batch.n,), nan, dtype=torch.float64, device="cuda")
        L.pecnn_rollout(plan, model_b, sim, g, a, b, 5, fb, st, ws=ws)
        return [a, b, fb, st]
    out = _twice(torch, plan.workspace(L.WS_ROLLOUT), roll)
    assert out[2].sum() > 0, "the guard was meant to hand some cloth to the simulator"
    plan.close()
