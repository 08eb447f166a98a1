"""GPU tests of the learned part: trajectory generation, BPTT through the C ABI against the
FP64 oracle's unrolled gradient, and the gain of training over the untrained network."""
import numpy as np
import pytest

import oracle
from paper_2403_12820_amd import inputs as I
from tests.gpu_util import dev_tensor, rel_inf

pytestmark = pytest.mark.gpu
MAT = I.Material()


@pytest.fixture(scope="module")
def L():
    from paper_2403_12820_amd import _lib
    _lib.lib()
    return _lib


def test_trajectory_frames_match_oracle(L):
    """Saved frames are stride-step mass-spring runs: frame 3 of a 16 x 20 scene equals 30 oracle steps."""
    from paper_2403_12820_amd.train import Trajectories
    scenes = I.random_scenes([(16, 20), (9, 9)], seed=7)
    tr = Trajectories(scenes, MAT, 4, 10)
    got = tr.frames[3].cpu().numpy().astype(np.float64)
    ref = oracle.batch_ms_step(tr.batch, tr.batch.state, MAT, 30)
    width = 19 * float(tr.batch.h[0])
    assert np.abs(got[:3] - ref[:3]).max() <= 1e-5 * width


@pytest.mark.parametrize("unroll", [1, 3])
def test_bptt_gradient_matches_oracle(L, unroll):
    """Loss = sum_t w_t * MSE(pred_t, target_t) over an unrolled rollout; the theta gradient from the
    library chain (forward, loss, backward in reverse order) equals the oracle's (pinned by finite
    differences)."""
    import torch
    from paper_2403_12820_amd.train import Trainer
    ch, dt = 16, 5e-3
    scenes = I.random_scenes([(8, 8), (6, 10)], seed=11)
    batch = I.make_batch(scenes)
    s1 = batch.state.astype(np.float64)
    s1[3:] = I.random_array((3, batch.total), seed=12, scale=0.1)
    s0 = s1.copy()
    s0[:3] -= dt * s1[3:]
    targets = [s1 + I.random_array(s1.shape, seed=20 + t, scale=0.01) for t in range(unroll)]
    th = (I.init_theta(ch, seed=13).astype(np.float64) * 10).astype(np.float32)
    sx, sv = 0.01, 0.05
    n_free = int((batch.pin == 0).sum())
    weights = [1.0 / unroll + (1.0 if t == 0 else 0.0) for t in range(unroll)]

    # library chain
    plan = L.Plan.from_batch(batch)
    tr = Trainer(ch=ch, dt_nn=dt, theta=th)
    S = [dev_tensor(s0), dev_tensor(s1)]
    pred = [torch.zeros_like(S[0]) for _ in range(unroll)]
    for t in range(unroll):
        L.pecnn_forward(plan, tr.model, S[-2], S[-1], pred[t])
        S.append(pred[t])
    grads = [torch.zeros_like(S[0]) for _ in range(unroll)]
    loss = torch.zeros(1, dtype=torch.float64, device="cuda")
    for t in range(unroll):
        L.pecnn_loss_mse(plan, pred[t], dev_tensor(targets[t]), sx, sv, weights[t], n_free, loss, grads[t])
    gth = torch.zeros(th.size, device="cuda")
    for t in range(unroll - 1, -1, -1):
        L.pecnn_backward(plan, tr.model, S[t], S[t + 1], grads[t], grads[t - 1] if t >= 1 else None,
                         grads[t - 2] if t >= 2 else None, gth)
    torch.cuda.synchronize()

    # oracle chain
    th64 = th.astype(np.float64)
    states = [s0.astype(np.float32).astype(np.float64), s1.astype(np.float32).astype(np.float64)]
    for t in range(unroll):
        sn, _ = oracle.batch_cnn_forward(batch, ch, 1.0, dt, th64, states[-2], states[-1])
        states.append(sn)
    og = [None, None] + [np.zeros_like(s0) for _ in range(unroll)]
    lv = 0.0
    for t in range(unroll):
        tg = targets[t].astype(np.float32).astype(np.float64)
        v, g = oracle.loss_mse(batch.pin, n_free, sx, sv, weights[t], states[t + 2], tg)
        lv += v
        og[t + 2] += g
    ogt = np.zeros(th.size)
    for t in range(unroll - 1, -1, -1):
        gc, gp, gt = oracle.batch_cnn_backward(batch, ch, 1.0, dt, th64, states[t], states[t + 1], og[t + 2])
        if t >= 1:
            og[t + 1] += gc
        if t >= 2:
            og[t] += gp
        ogt += gt
    assert abs(loss.item() - lv) <= 1e-5 * abs(lv)
    assert rel_inf(gth.cpu().numpy(), ogt) <= 1e-5, rel_inf(gth.cpu().numpy(), ogt)


@pytest.mark.parametrize("alpha", [0.0, 0.5, 1.0])
def test_trainer_gradient_with_physics_term_matches_oracle(L, alpha):
    """Eq. (8) with both terms: (1 - alpha) x the data term plus alpha x the physics term, whose
    target is the simulator's velocity after one frame (10 steps) from each frame's own input state,
    held constant. The trainer's loss and theta gradient over a 3-frame unroll equal the oracle's
    chain, which runs its own FP64 simulator for the targets."""
    import torch
    from paper_2403_12820_amd.train import NO_POSITIONS, Trainer
    ch, dt, stride, U = 16, 5e-3, 10, 3
    scenes = I.random_scenes([(8, 8), (6, 10)], seed=11)
    batch = I.make_batch(scenes)
    s1 = batch.state.astype(np.float64)
    s1[3:] = I.random_array((3, batch.total), seed=12, scale=0.1)
    s0 = s1.copy()
    s0[:3] -= dt * s1[3:]
    targets = [s1 + I.random_array(s1.shape, seed=20 + t, scale=0.01) for t in range(U)]
    th = (I.init_theta(ch, seed=13).astype(np.float64) * 10).astype(np.float32)
    sx, sv = 0.01, 0.05
    n_free = int((batch.pin == 0).sum())
    plan = L.Plan.from_batch(batch)
    tr = Trainer(ch=ch, dt_nn=dt, theta=th)
    frames = np.stack([s0, s1] + targets).astype(np.float32)
    tr.gradient(torch.tensor(frames, device="cuda"), plan, n_free, sx, sv, 1.0, alpha, L.ms_params(MAT), stride)
    torch.cuda.synchronize()
    loss, gth = tr.loss.item(), tr.g.cpu().numpy()

    th64 = th.astype(np.float64)
    states = [frames[0].astype(np.float64), frames[1].astype(np.float64)]
    og = [None, None] + [np.zeros_like(s0) for _ in range(U)]
    lv = 0.0
    for t in range(U):
        sn, _ = oracle.batch_cnn_forward(batch, ch, 1.0, dt, th64, states[-2], states[-1])
        phys = oracle.batch_ms_step(batch, states[-1], MAT, stride)
        states.append(sn)
        w = 1.0 / U + (1.0 if t == 0 else 0.0)
        for tgt, sxx, wt in ((frames[t + 2].astype(np.float64), sx, (1 - alpha) * w), (phys, NO_POSITIONS, alpha * w)):
            if wt > 0:
                v, g = oracle.loss_mse(batch.pin, n_free, sxx, sv, wt, sn, tgt)
                lv += v
                og[t + 2] += g
    ogt = np.zeros(th.size)
    for t in range(U - 1, -1, -1):
        gc, gp, gt = oracle.batch_cnn_backward(batch, ch, 1.0, dt, th64, states[t], states[t + 1], og[t + 2])
        if t >= 1:
            og[t + 1] += gc
        if t >= 2:
            og[t] += gp
        ogt += gt
    assert abs(loss - lv) <= 1e-5 * abs(lv), (loss, lv)
    assert rel_inf(gth, ogt) <= 1e-5, rel_inf(gth, ogt)


def test_trainer_rejects_bad_alpha(L):
    from paper_2403_12820_amd.train import Trainer
    import torch
    tr = Trainer(ch=16, dt_nn=5e-3)
    batch = I.make_batch(I.random_scenes([(8, 8)], seed=1))
    plan = L.Plan.from_batch(batch)
    buf = torch.zeros(3, 6, batch.total, device="cuda")
    with pytest.raises(ValueError):
        tr.gradient(buf, plan, 10, 0.01, 0.05, alpha=1.5, sim=L.ms_params(MAT))
    with pytest.raises(ValueError):
        tr.gradient(buf, plan, 10, 0.01, 0.05, alpha=0.5, sim=None)


def test_training_reduces_loss_and_beats_untrained(L):
    """A short training run on small synthetic trajectories: the held-out loss of the final
    parameters is below that of the initial ones, and on test scenes that neither training nor
    the choice of the kept parameters saw, the kept network's 20-frame rollout error is below 0.97
    of the untrained network's (600 iterations at 24 x 24 learn little more than gravity; the
    committed weights are held to a larger gain below)."""
    from paper_2403_12820_amd.train import train
    theta, rep = train(n_scenes=15, size=24, n_val=3, n_test=3, iters=600, n_win=8, n_unroll=4, ch=16, lr=1e-3,
                       seed=3, n_frames=41, stride=10, log_every=200, eval_frames=20, verbose=False, lr_final=1e-4)
    print("test-scene rms: trained %.4g untrained %.4g; selection scenes: %.4g %.4g" % (
        rep["test_rms_trained_mean"], rep["test_rms_untrained_mean"], rep["val_rms_trained_mean"],
        rep["val_rms_untrained_mean"]))
    assert rep["val_loss_final_theta"] < rep["val_loss_first"], rep["loss_curve"]
    assert rep["test_rms_trained_mean"] < 0.97 * rep["test_rms_untrained_mean"], rep
    assert np.all(np.isfinite(theta))


def test_checkpoint_resume_matches_straight_run(L, tmp_path):
    """Training stopped at a checkpoint and resumed from it (theta, Adam moments and step, the
    sampler's RNG state, the best parameters so far) ends bit for bit where an uninterrupted run
    ends."""
    from paper_2403_12820_amd.train import train
    kw = dict(n_scenes=6, size=16, n_val=1, n_test=1, iters=30, n_win=4, n_unroll=3, ch=16, lr=1e-3, seed=5,
              n_frames=21, stride=10, log_every=10, eval_frames=10, verbose=False, lr_final=1e-4)
    a, b = str(tmp_path / "straight.npz"), str(tmp_path / "resumed.npz")
    th_a, _ = train(**kw, checkpoint=a, checkpoint_every=15)
    assert train(**kw, checkpoint=b, checkpoint_every=15, stop_after=15) == (None, None)
    with np.load(b, allow_pickle=False) as z:
        assert int(z["t"]) == 15
    th_b, _ = train(**kw, checkpoint=b, checkpoint_every=15, resume=b)
    np.testing.assert_array_equal(th_a, th_b)
    with np.load(a, allow_pickle=False) as za, np.load(b, allow_pickle=False) as zb:
        assert int(za["t"]) == int(zb["t"]) == 30
        for k in ("theta", "m", "v", "best_theta"):
            np.testing.assert_array_equal(za[k], zb[k])
        assert str(za["rng"]) == str(zb["rng"])


def test_committed_weights_gain_on_unseen_scenes(L):
    """The committed Ch = 32 weights against the untrained initial weights on the eight 64 x 64
    test scenes of the training draw (scenes 64..71 of seed 4: the committed run trained on
    scenes 0..55 and chose its kept parameters on 56..63), 100 frames of 10 simulator steps: the
    trained network's mean position RMS is at most 0.6 of the untrained one's (measured: 0.165
    against 0.520). Scene by scene it is lower on seven of the eight; on one cloth pinned at its four
    corners it is higher (0.43 against 0.25), so no per-scene bound is asserted."""
    import os
    from paper_2403_12820_amd.train import Trajectories, rollout_rms
    w = os.path.join(os.path.dirname(os.path.dirname(os.path.abspath(__file__))), "paper_2403_12820_amd", "weights",
                     "pecnn_ch32.npy")
    theta = np.load(w, allow_pickle=False).astype(np.float32)
    scenes = I.random_scenes([(64, 64)] * 72, seed=4)[64:]
    traj = Trajectories(scenes, MAT, 101, 10)
    ids = list(range(len(scenes)))
    rms_t, _ = rollout_rms(traj, ids, theta, 32, 100)
    rms_u, _ = rollout_rms(traj, ids, I.init_theta(32, seed=1), 32, 100)
    print("unseen 64x64 scenes, 100 frames: trained %s, untrained %s" % (np.round(rms_t, 4), np.round(rms_u, 4)))
    assert rms_t.mean() <= 0.6 * rms_u.mean(), (rms_t, rms_u)
    assert np.all(np.isfinite(rms_t)), rms_t