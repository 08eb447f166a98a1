"""Pins of the oracle's pressure force (eq. 3) and of its place in the mass-spring step and the
CNN frame, against closed forms, invariants and brute force.

The reading: the four nearest neighbours, taken round the node in the order right, down, left,
up, form four consecutive pairs (j1, j2); a pair counts when both nodes lie on the grid and adds
p (x_j1 - x_i) x (x_j2 - x_i). On the flat rest grid each pair gives +h^2 along z.
"""
import math

import numpy as np
import pytest

import oracle
from paper_2403_12820_amd import inputs as I


def _only_pressure():
    m = I.Material()
    m.k_struct = m.k_shear = m.k_bend = 0.0
    m.mu = m.drag = 0.0
    m.g = (0.0, 0.0, 0.0)
    return m


def _state(x):
    s = np.zeros((6, x.shape[1]))
    s[:3] = x
    return s


def _force(H, W, x, pr, h=0.1):
    return oracle.ms_force(H, W, h, 1.0, np.zeros(3), np.zeros(H * W, np.uint8), _state(x),
                           _only_pressure(), pressure=pr)


def test_flat_grid_closed_form():
    """Flat grid: every complete pair adds pr h^2 along +z; interior nodes have 4 pairs, edge
    nodes 2, corners 1."""
    H, W, h, pr = 5, 7, 0.1, 3.0
    f = _force(H, W, I.flat_grid(H, W, h), pr, h).reshape(3, H, W)
    count = np.full((H, W), 4.0)
    count[0, :] = count[-1, :] = 2.0
    count[:, 0] = count[:, -1] = 2.0
    count[0, 0] = count[0, -1] = count[-1, 0] = count[-1, -1] = 1.0
    np.testing.assert_allclose(f[2], pr * h * h * count, rtol=1e-14, atol=0)
    assert np.abs(f[:2]).max() < 1e-15


def test_cylinder_closed_form():
    """A sheet wrapped round a cylinder of radius R (axis along y, columns along the arc):
    x = (R sin t, y, R cos t), t = j h / R. For interior nodes the four pairs sum to
    4 pr h R sin(h / R) times the outward unit normal (sin t, 0, cos t)."""
    H, W, h, R, pr = 6, 9, 0.1, 0.35, 2.5
    i, j = np.meshgrid(np.arange(H, dtype=float), np.arange(W, dtype=float), indexing="ij")
    t = j * h / R
    x = np.stack([R * np.sin(t), i * h, R * np.cos(t)]).reshape(3, -1)
    f = _force(H, W, x, pr, h).reshape(3, H, W)
    mag = 4 * pr * h * R * math.sin(h / R)
    exp = np.stack([mag * np.sin(t), np.zeros_like(t), mag * np.cos(t)])
    np.testing.assert_allclose(f[:, 1:-1, 1:-1], exp[:, 1:-1, 1:-1], rtol=0, atol=1e-13 * mag)


def _random_config(H, W, h, seed):
    x = I.flat_grid(H, W, h) + I.random_array((3, H * W), seed=seed, scale=0.3 * h)
    return x


def test_interior_force_does_not_depend_on_own_position():
    """Round a complete ring of four pairs the node's own position cancels out of the sum
    (each neighbour appears once as j1 and once as j2), so moving an interior node leaves its
    own pressure force unchanged."""
    H, W, h = 5, 5, 0.1
    x = _random_config(H, W, h, 5)
    p = 2 * W + 2
    f0 = _force(H, W, x, 1.7, h)
    x2 = x.copy()
    x2[:, p] += np.array([0.03, -0.02, 0.05])
    f1 = _force(H, W, x2, 1.7, h)
    np.testing.assert_allclose(f1[:, p], f0[:, p], rtol=0, atol=1e-15)
    assert np.abs(f1[:, p + 1] - f0[:, p + 1]).max() > 1e-4  # a neighbour's force does change


def test_rotation_translation_and_scaling():
    """Cross products of differences: rotating the cloth rotates the forces, a translation
    changes nothing, scaling all positions by s scales the forces by s^2."""
    H, W, h = 4, 6, 0.1
    x = _random_config(H, W, h, 7)
    f = _force(H, W, x, 1.3, h)
    a, b, c = 0.3, -1.1, 0.7
    Rz = np.array([[math.cos(a), -math.sin(a), 0], [math.sin(a), math.cos(a), 0], [0, 0, 1]])
    Rx = np.array([[1, 0, 0], [0, math.cos(b), -math.sin(b)], [0, math.sin(b), math.cos(b)]])
    Ry = np.array([[math.cos(c), 0, math.sin(c)], [0, 1, 0], [-math.sin(c), 0, math.cos(c)]])
    R = Rz @ Rx @ Ry
    np.testing.assert_allclose(_force(H, W, R @ x, 1.3, h), R @ f, rtol=0, atol=1e-15)
    np.testing.assert_allclose(_force(H, W, x + np.array([[5.0], [-2.0], [0.5]]), 1.3, h), f, rtol=0, atol=1e-14)
    np.testing.assert_allclose(_force(H, W, 2.5 * x, 1.3, h), 6.25 * f, rtol=1e-13, atol=0)


def test_mass_spring_step_applies_pressure_on_free_nodes():
    """Eq. (5) with only pressure acting on a flat grid at rest: free interior nodes gain
    dt pr 4 h^2 / m along z, pinned nodes stay at rest."""
    H, W = 6, 6
    mat = _only_pressure()
    h, m, pr = mat.h, mat.mass, 2.0
    pin = I.pin_mask(H, W, "four_corners")
    s = _state(I.flat_grid(H, W, h))
    out = oracle.ms_step(H, W, h, m, np.zeros(3), pin, s, mat, pressure=pr).reshape(6, H, W)
    np.testing.assert_allclose(out[5, 1:-1, 1:-1], mat.dt * pr * 4 * h * h / m, rtol=1e-13)
    assert out[5].reshape(-1)[pin == 1].max() == 0.0


def test_cnn_frame_adds_pressure_like_the_simulator():
    """With theta = 0 the cell adds nothing, so the frame's velocity change is dt (a_ext +
    f_p / m), with f_p the simulator's pressure force at S^k."""
    H, W, ch, dt = 5, 6, 16, 5e-3
    h, m, pr = 0.1, 0.02, 1.5
    x = _random_config(H, W, h, 9)
    sk = _state(x)
    sk[3:] = I.random_array((3, H * W), seed=10, scale=0.1)
    pin = np.zeros(H * W, np.uint8)
    a = np.array([0.2, -0.1, 0.0])
    th = np.zeros(oracle.theta_size(ch))
    out, dv = oracle.cnn_forward(H, W, ch, 1.0, dt, a, pin, th, sk, sk, pm=pr / m)
    assert np.abs(dv).max() == 0.0
    fp = _force(H, W, x, pr, h)
    np.testing.assert_allclose(out[3:] - sk[3:], dt * (a[:, None] + fp / m), rtol=1e-13, atol=1e-15)


@pytest.mark.parametrize("ch", [16])
def test_backward_with_pressure_finite_differences(ch):
    """Brute force: central differences of a random linear functional of one frame with
    pressure, with respect to theta and to entries of S^k and S^{k-1}."""
    H, W, dt, pm = 6, 7, 5e-3, 40.0
    th = I.init_theta(ch, seed=71).astype(np.float64) * 10
    pin = I.pin_mask(H, W, "two_top_corners")
    a_ext = np.array([0.4, -0.3, 0.0])
    x = _random_config(H, W, 1.0 / 31, 11)
    s1 = _state(x)
    s1[3:] = I.random_array((3, H * W), seed=12, scale=0.2)
    s0 = s1.copy()
    s0[:3] -= dt * s1[3:]
    tg = I.random_array((6, H * W), seed=13)

    def L(a=s0, b=s1):
        sn, _ = oracle.cnn_forward(H, W, ch, 1.0, dt, a_ext, pin, th, a, b, pm=pm)
        return float(np.sum(tg * sn))

    g1, g0, _ = oracle.cnn_backward(H, W, ch, 1.0, dt, pin, th, s0, s1, tg, pm=pm)
    scale = max(1.0, np.abs(g1).max())
    rs = np.random.RandomState(1)
    for which, g in ((0, g0), (1, g1)):
        for flat in rs.choice(3 * H * W, 40, replace=False):  # positions, where pressure acts
            c, p = divmod(int(flat), H * W)
            base = s0 if which == 0 else s1
            e = 1e-6
            bp, bm = base.copy(), base.copy()
            bp[c, p] += e
            bm[c, p] -= e
            fd = (L(a=bp) - L(a=bm)) / (2 * e) if which == 0 else (L(b=bp) - L(b=bm)) / (2 * e)
            assert abs(fd - g[c, p]) <= 1e-6 * scale, (which, c, p, fd, g[c, p])
    # the pressure part of the gradient is not small here
    g1n, _, _ = oracle.cnn_backward(H, W, ch, 1.0, dt, pin, th, s0, s1, tg, pm=0.0)
    assert np.abs(g1 - g1n)[:3].max() > 1e-3 * np.abs(g1[:3]).max()
