"""Parity at the largest sizes a plan accepts.

* One cloth of 4097 x 4095 nodes, 2^24 - 1: the most one instance may have. Its width is odd, so
  the scalar-load path runs. It sits beside the smallest cloth (1 x 2) and a tiny one. The
  simulator step, the three frames (bf16 and FP32 convolution cell, pair cell) and both reverse
  passes are checked.
* Eleven cloths of 4096 columns that fill the batch up to its node limit (24 N < 2^32):
  178,954,240 nodes and 4.3 GB per state, with 16-byte row pieces. Every tile configuration must
  give the same bits. The FP64 diagnostics and a guarded rollout are checked there too.

The oracle computes windows of the large cloths: corners, edge midpoints and the centre. A
window node whose stencil lies inside the window sees the same inputs as in the whole cloth. That
means two nodes from a cut edge for the simulator and the pair cell, and one for the convolution
cell. Only those nodes are compared. The reverse passes take an output gradient that is zero
outside the windows' inner nodes, so the whole-cloth gradients are the sums of the windows'."""
import dataclasses

import numpy as np
import pytest

import oracle
from paper_2403_12820_amd import inputs as I
from tests.gpu_util import U32, dev_tensor, ms_velocity_floor, rel_inf

pytestmark = [pytest.mark.gpu, pytest.mark.timeout(600)]
MAT = I.Material()
# the oracle takes the material with the values the library receives (its parameters are FP32):
# with cloths 1.25 m above the plane, gravity's FP32 rounding alone moves the energy by 3e-9
MAT32 = dataclasses.replace(MAT, **{f.name: float(np.float32(getattr(MAT, f.name)))
                                    for f in dataclasses.fields(MAT) if f.name != "g"},
                            g=tuple(float(np.float32(x)) for x in MAT.g))
DT = 5e-3
BIG = (4097, 4095)                        # 2^24 - 1 nodes
NODE_LIMIT = (1 << 32) // 24              # a plan holds fewer nodes than this
FULL = [(4095, 4096)] * 10 + [(2740, 4096)]
WIN = 20


def _windows(H, W, n=WIN):
    """(r0, r1, c0, c1) of the corners, the edge midpoints and the centre; the whole grid if small."""
    if H < 4 * n or W < 4 * n:
        return [(0, H, 0, W)]
    rs, cs = (0, H // 2 - n // 2, H - n), (0, W // 2 - n // 2, W - n)
    return [(r, r + n, c, c + n) for r in rs for c in cs]


def _idx(W, off, w):
    r0, r1, c0, c1 = w
    return (off + np.arange(r0, r1)[:, None] * W + np.arange(c0, c1)[None, :]).ravel()


def _inner(H, W, w, m):
    """Window nodes at least m nodes from every window edge that is not a grid edge."""
    r0, r1, c0, c1 = w
    rr, cc = np.arange(r0, r1)[:, None], np.arange(c0, c1)[None, :]
    ok = np.ones((r1 - r0, c1 - c0), bool)
    if r0 > 0:
        ok &= rr >= r0 + m
    if r1 < H:
        ok &= rr < r1 - m
    if c0 > 0:
        ok &= cc >= c0 + m
    if c1 < W:
        ok &= cc < c1 - m
    return ok.ravel()


def _cases(batch, instances):
    """(instance, H, W, window, node indices) for every window of the chosen instances."""
    out = []
    for b in instances:
        H, W, off = int(batch.H[b]), int(batch.W[b]), int(batch.node_off[b])
        for w in _windows(H, W):
            out.append((b, H, W, w, _idx(W, off, w)))
    return out


def _fetch(t, idx):
    import torch
    return t[:, torch.from_numpy(idx).to(t.device)].cpu().numpy().astype(np.float64)


def _frame_dv(a, s1w, out, pin):
    dv = out[3:] - s1w[3:].astype(np.float64) - DT * a[:, None]
    dv[:, pin == 1] = 0.0
    return dv


def _check_ms(batch, s1, out, instances):
    tol_floor = ms_velocity_floor(batch, MAT)
    for b, H, W, w, idx in _cases(batch, instances):
        r0, r1, c0, c1 = w
        ref = oracle.ms_run(r1 - r0, c1 - c0, float(batch.h[b]), float(batch.mass[b]),
                            batch.a_ext[b].astype(np.float64), batch.pin[idx], s1[:, idx], MAT32, 1)
        got = _fetch(out, idx)
        ok = _inner(H, W, w, 2)
        xmax = np.abs(ref[:3]).max()
        assert np.abs(got[:3, ok] - ref[:3, ok]).max() <= 4 * U32 * xmax + MAT.dt * tol_floor, (b, w)
        tol_v = max(1e-5 * np.abs(ref[3:, ok]).max(), tol_floor)
        assert np.abs(got[3:, ok] - ref[3:, ok]).max() <= tol_v, (b, w)


def _check_conv_frame(batch, s0, s1, th, out, bf16, instances):
    for b, H, W, w, idx in _cases(batch, instances):
        r0, r1, c0, c1 = w
        a = batch.a_ext[b].astype(np.float64)
        pin = batch.pin[idx]
        ref, dv_ref = oracle.cnn_forward(r1 - r0, c1 - c0, 32, 1.0, DT, a, pin, th.astype(np.float64), s0[:, idx],
                                         s1[:, idx], emu=7 if bf16 else 0)
        dv_ref[:, pin == 1] = 0.0
        got = _fetch(out, idx)
        dv = _frame_dv(a, s1[:, idx], got, pin)
        ok = _inner(H, W, w, 1)
        assert rel_inf(dv[:, ok], dv_ref[:, ok]) <= (2.0 ** -8 if bf16 else 1e-5), (b, w)
        tol_x = 4 * U32 * np.abs(ref[:3]).max() + DT * (2.0 ** -8 if bf16 else 1e-5) * np.abs(dv_ref).max()
        assert np.abs(got[:3, ok] - ref[:3, ok]).max() <= tol_x, (b, w)


def _batch(sizes, seed):
    """Cloths at their rest grid plus a random displacement (0.15 h rms per axis) and random
    velocities (0.1 m/s rms), shifted by half a metre per cloth, with pins and wind drawn per
    cloth; returns the batch (state S^k) and S^{k-1} = S^k less one frame of motion, velocities
    scaled by 0.98. The random fields are drawn once for 2^20 nodes; each cloth takes them rolled
    by its own amount and repeated, which keeps the generation of 1.8e8 nodes to seconds."""
    mat = I.Material()
    h = float(np.float32(mat.h))
    P = I.random_array((3, 1 << 20), seed, scale=0.15 * h)
    V = I.random_array((3, 1 << 20), seed + 1, scale=0.1)
    kinds, winds = I.random_scene_params(len(sizes), seed + 2)
    off = np.zeros(len(sizes) + 1, np.int64)
    off[1:] = np.cumsum([H * W for H, W in sizes])
    s1 = np.empty((6, int(off[-1])), np.float32)
    s0 = np.empty_like(s1)
    pin = np.empty(int(off[-1]), np.uint8)
    for b, (H, W) in enumerate(sizes):
        o, n = int(off[b]), H * W
        rest = (np.arange(W)[None, :] * h, np.arange(H)[:, None] * h, 0.0)
        for c in range(3):
            x = s1[c, o:o + n]
            x.reshape(H, W)[:] = rest[c] + (0.5, -0.25, 0.125)[c] * b + np.resize(np.roll(P[c], 7919 * b), n).reshape(H, W)
            v = s1[3 + c, o:o + n]
            v[:] = np.resize(np.roll(V[c], 104729 * b), n)
            s0[c, o:o + n] = x - np.float32(DT) * v
            s0[3 + c, o:o + n] = np.float32(0.98) * v
        pin[o:o + n] = I.pin_mask(H, W, kinds[b])
    nb = len(sizes)
    batch = I.Batch(np.array([s[0] for s in sizes], np.int32), np.array([s[1] for s in sizes], np.int32),
                    np.full(nb, h, np.float32), np.full(nb, float(np.float32(mat.mass)), np.float32),
                    winds.astype(np.float32), pin, s1, off, np.zeros(nb, np.float32))
    return batch, s0


# ------------------------------------------------------------------ the largest cloth
@pytest.fixture(scope="module")
def big():
    from paper_2403_12820_amd import _lib as L
    batch, s0 = _batch([BIG, (1, 2), (2, 3)], 1700)
    s1 = batch.state
    assert int(batch.H[0]) * int(batch.W[0]) == (1 << 24) - 1
    plan = L.Plan.from_batch(batch)
    th = (I.init_theta(32, seed=1701).astype(np.float64) * 20).astype(np.float32)
    return L, batch, plan, s0, s1, dev_tensor(s0), dev_tensor(s1), th


def test_largest_cloth_ms_step_and_frames(big):
    import torch
    L, batch, plan, s0, s1, d0, d1, th = big
    everything = range(batch.n)
    out = torch.zeros_like(d1)
    L.cloth_ms_step(plan, L.ms_params(MAT), d1, out, 1)
    torch.cuda.synchronize()
    _check_ms(batch, s1, out, everything)
    for prec in (L.PECNN_BF16, L.PECNN_FP32):
        model = L.make_model(dev_tensor(th), 32, prec, dt=DT)
        L.pecnn_forward(plan, model, d0, d1, out)
        torch.cuda.synchronize()
        _check_conv_frame(batch, s0, s1, th, out, prec == L.PECNN_BF16, everything)
    pth = I.init_pair_theta(seed=1702).astype(np.float64)
    pth[12:48] += I.random_array((36,), seed=1703, scale=0.05)
    pth = pth.astype(np.float32)
    L.pecnn_forward(plan, L.make_model(dev_tensor(pth), 12, L.PECNN_FP32, dt=DT, cell=L.CELL_PAIR), d0, d1, out)
    torch.cuda.synchronize()
    for b, H, W, w, idx in _cases(batch, everything):
        r0, r1, c0, c1 = w
        a = batch.a_ext[b].astype(np.float64)
        ref, _ = oracle.pair_forward(r1 - r0, c1 - c0, 1.0, DT, a, batch.pin[idx], pth.astype(np.float64), s1[:, idx])
        got = _fetch(out, idx)
        ok = _inner(H, W, w, 2)
        d_got = _frame_dv(a, s1[:, idx], got, batch.pin[idx])
        d_ref = _frame_dv(a, s1[:, idx], ref, batch.pin[idx])
        assert rel_inf(d_got[:, ok], d_ref[:, ok]) <= 1e-5, (b, w)


def _sparse_gradient(batch, margin, seed):
    """An output gradient that is random on the inner nodes of every window and zero elsewhere."""
    gn = np.zeros((6, batch.total), np.float32)
    cases = _cases(batch, range(batch.n))
    for k, (b, H, W, w, idx) in enumerate(cases):
        ok = _inner(H, W, w, margin)
        gn[:, idx[ok]] = I.random_array((6, int(ok.sum())), seed=seed + k).astype(np.float32)
    return gn, cases


def _zero_outside(t, cases):
    import torch
    rest = t.clone()
    for *_, idx in cases:
        rest[:, torch.from_numpy(idx).to(t.device)] = 0.0
    return int(torch.count_nonzero(rest))


def test_largest_cloth_backward(big):
    """Both cells' reverse passes over 2^24 - 1 nodes: input gradients on every window node,
    zero elsewhere, and the theta gradient summed over the whole batch."""
    import torch
    L, batch, plan, s0, s1, d0, d1, th = big
    # convolution cell: a window's inner nodes (one from a cut edge) depend only on window nodes
    gn, cases = _sparse_gradient(batch, 1, 1710)
    model = L.make_model(dev_tensor(th), 32, L.PECNN_FP32, dt=DT)
    gc, gp = torch.zeros_like(d1), torch.zeros_like(d1)
    gt = torch.zeros(th.size, device="cuda")
    L.pecnn_backward(plan, model, d0, d1, dev_tensor(gn), gc, gp, gt)
    torch.cuda.synchronize()
    rt = np.zeros(th.size)
    got_c, got_p, ref_c, ref_p = [], [], [], []
    for b, H, W, w, idx in cases:
        r0, r1, c0, c1 = w
        c, p, t = oracle.cnn_backward(r1 - r0, c1 - c0, 32, 1.0, DT, batch.pin[idx], th.astype(np.float64),
                                      s0[:, idx], s1[:, idx], gn[:, idx])
        rt += t
        got_c.append(_fetch(gc, idx))
        got_p.append(_fetch(gp, idx))
        ref_c.append(c)
        ref_p.append(p)
    e = [rel_inf(np.concatenate(got_c, 1), np.concatenate(ref_c, 1)),
         rel_inf(np.concatenate(got_p, 1), np.concatenate(ref_p, 1)), rel_inf(gt.cpu().numpy(), rt)]
    assert max(e) <= 1e-5, e
    assert _zero_outside(gc, cases) == 0 and _zero_outside(gp, cases) == 0
    del gc, gp

    # pair cell: its links reach two nodes
    pth = I.init_pair_theta(seed=1711).astype(np.float64)
    pth[12:48] += I.random_array((36,), seed=1712, scale=0.05)
    pth = pth.astype(np.float32)
    gn, cases = _sparse_gradient(batch, 2, 1720)
    model = L.make_model(dev_tensor(pth), 12, L.PECNN_FP32, dt=DT, cell=L.CELL_PAIR)
    gc = torch.zeros_like(d1)
    gt = torch.zeros(pth.size, device="cuda")
    L.pecnn_backward(plan, model, d1, d1, dev_tensor(gn), gc, None, gt)
    torch.cuda.synchronize()
    rt = np.zeros(pth.size)
    got_c, ref_c = [], []
    for b, H, W, w, idx in cases:
        r0, r1, c0, c1 = w
        c, t = oracle.pair_backward(r1 - r0, c1 - c0, 1.0, DT, batch.pin[idx], pth.astype(np.float64), s1[:, idx],
                                    gn[:, idx])
        rt += t
        got_c.append(_fetch(gc, idx))
        ref_c.append(c)
    e = [rel_inf(np.concatenate(got_c, 1), np.concatenate(ref_c, 1)), rel_inf(gt.cpu().numpy(), rt)]
    assert max(e) <= 1e-5, e
    assert _zero_outside(gc, cases) == 0


# ------------------------------------------------------------------ the batch at its node limit
@pytest.fixture(scope="module")
def full():
    from paper_2403_12820_amd import _lib as L
    total = sum(h * w for h, w in FULL)
    assert total < NODE_LIMIT and NODE_LIMIT - total < 4096
    batch, s0 = _batch(FULL, 1800)
    s1 = batch.state
    plan = L.Plan.from_batch(batch)
    th = (I.init_theta(32, seed=1802).astype(np.float64) * 20).astype(np.float32)
    return L, batch, plan, s0, s1, dev_tensor(s0), dev_tensor(s1), th


SAMPLED = (0, 5, 10)


def test_node_limit_every_tile_config_same_bits(full):
    import torch
    L, batch, plan, s0, s1, d0, d1, th = full
    assert batch.total == 178_954_240
    ref, out = torch.zeros_like(d1), torch.zeros_like(d1)
    for cfg in range(5):
        plan.set_tiles(ms_cfg=cfg)
        L.cloth_ms_step(plan, L.ms_params(MAT), d1, ref if cfg == 0 else out, 1)
        torch.cuda.synchronize()
        if cfg:
            assert torch.equal(out, ref), cfg
    _check_ms(batch, s1, ref, SAMPLED)
    model = L.make_model(dev_tensor(th), 32, L.PECNN_BF16, dt=DT)
    for cfg in range(4):
        plan.set_tiles(cnn_cfg=cfg)
        L.pecnn_forward(plan, model, d0, d1, ref if cfg == 0 else out)
        torch.cuda.synchronize()
        if cfg:
            assert torch.equal(out, ref), cfg
    _check_conv_frame(batch, s0, s1, th, ref, True, SAMPLED)


def test_node_limit_diagnostics_and_rollout(full):
    import torch
    L, batch, plan, s0, s1, d0, d1, th = full
    out = torch.zeros(4 * batch.n, dtype=torch.float64, device="cuda")
    L.cloth_reduce_fp64(plan, L.ms_params(MAT), d1, d0, out)
    torch.cuda.synchronize()
    o = out.cpu().numpy().reshape(-1, 4)
    for b in (0, batch.n - 1):  # the first and the last cloth, whole
        H, W = int(batch.H[b]), int(batch.W[b])
        sl = batch.instance(b)
        h, m = float(batch.h[b]), float(batch.mass[b])
        # sums over 1.7e7 nodes in two orders: relative rounding about eps sqrt(N) = 5e-13
        err = oracle.sq_pos_err(H, W, s1[:, sl], s0[:, sl])
        assert abs(o[b, 0] - err) <= 1e-11 * err
        a = batch.a_ext[b].astype(np.float64)
        e = oracle.energy(H, W, h, m, a, s1[:, sl], MAT32)
        # the potential terms can cancel: the bound is taken on their magnitudes
        r = np.linalg.norm(s1[:3, sl].astype(np.float64), axis=0).sum()
        scale = abs(e) + m * (np.linalg.norm(MAT32.g) + np.linalg.norm(a)) * r
        assert abs(o[b, 1] - e) <= 1e-10 * scale
        assert abs(o[b, 2] - oracle.max_stretch(H, W, h, s1[:, sl], 1)) <= 1e-12
        assert abs(o[b, 3] - oracle.max_stretch(H, W, h, s1[:, sl], 7)) <= 1e-12
    del out

    # three guarded frames (a check after each, bounds no cloth reaches) equal three forward calls
    plan.set_tiles(cnn_cfg=0)
    model = L.make_model(dev_tensor(th), 32, L.PECNN_BF16, dt=DT)
    bufs = [d0.clone(), d1.clone(), torch.zeros_like(d1)]
    for _ in range(3):
        L.pecnn_forward(plan, model, bufs[0], bufs[1], bufs[2])
        bufs = [bufs[1], bufs[2], bufs[0]]
    torch.cuda.synchronize()
    g = L.Guard()
    g.stretch_max, g.energy_gain_max, g.check_every, g.substeps = 1e30, 1e30, 1, 10
    fb = torch.zeros(batch.n, dtype=torch.int32, device="cuda")
    stats = torch.zeros(4 * batch.n, dtype=torch.float64, device="cuda")
    a, b = d0.clone(), d1.clone()
    L.pecnn_rollout(plan, model, L.ms_params(MAT), g, a, b, 3, fb, stats)
    torch.cuda.synchronize()
    assert torch.equal(a, bufs[0]) and torch.equal(b, bufs[1])
    assert int(fb.sum()) == 0
    # the energy at the start, as the diagnostics computed it
    st = stats.cpu().numpy().reshape(-1, 4)
    np.testing.assert_allclose(st[:, 0], o[:, 1], rtol=1e-14, atol=0)
