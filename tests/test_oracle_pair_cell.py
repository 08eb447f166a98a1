"""Pins of the oracle's pair cell: section 3.2 read literally. Twelve channels, one per stencil
neighbour, phi_c = s_c (x_j - x_i) and xi_c = s_c (v_j - v_i) (frozen +-s_c filters shared by the
three axes; zero off the grid), then per axis dv = sum_c [wL_c phi_c + wN_c sigma(phi_c) +
wD_c xi_c sigma(phi_c)] + b_L.

Checked against a library graph Laplacian, closed forms, invariants and central differences."""
import math

import numpy as np
import pytest
import scipy.sparse as sp
from scipy.sparse.csgraph import laplacian

import oracle
from paper_2403_12820_amd import inputs as I

PS, PWL, PWN, PWD, PBL = 0, 12, 24, 36, 48


def _theta(**blocks):
    th = np.zeros(51)
    for k, v in blocks.items():
        off = {"s": PS, "wL": PWL, "wN": PWN, "wD": PWD, "bL": PBL}[k]
        v = np.atleast_1d(np.asarray(v, float))
        th[off:off + v.size] = v
    return th


def _state(H, W, seed, h=1.0 / 31, pos=0.2, vel=0.3):
    s = np.zeros((6, H * W))
    s[:3] = I.flat_grid(H, W, h) + I.random_array((3, H * W), seed=seed, scale=pos * h)
    s[3:] = I.random_array((3, H * W), seed=seed + 1, scale=vel)
    return s


def _grid_laplacian(H, W, offsets):
    """Graph Laplacian D - A of the grid with edges along the given (dy, dx) offsets (scipy)."""
    n = H * W
    rows, cols = [], []
    for i in range(H):
        for j in range(W):
            for dy, dx in offsets:
                ii, jj = i + dy, j + dx
                if 0 <= ii < H and 0 <= jj < W:
                    rows.append(i * W + j)
                    cols.append(ii * W + jj)
    A = sp.coo_matrix((np.ones(len(rows)), (rows, cols)), shape=(n, n)).tocsr()
    return laplacian(A)


@pytest.mark.parametrize("fam,offsets", [
    (0, [(0, 1), (0, -1), (1, 0), (-1, 0)]),
    (1, [(1, 1), (1, -1), (-1, 1), (-1, -1)]),
    (2, [(0, 2), (0, -2), (2, 0), (-2, 0)]),
])
def test_linear_branch_is_a_graph_laplacian(fam, offsets):
    """With only the linear weights of one spring family (w), unit filters and no bias, dv is
    -w times the graph Laplacian of that family's links applied to the positions, axis by
    axis."""
    H, W, w = 7, 9, 0.37
    wl = np.zeros(12)
    wl[4 * fam:4 * fam + 4] = w
    th = _theta(s=np.ones(12), wL=wl)
    s = _state(H, W, 3)
    _, dv = oracle.pair_forward(H, W, 1.0, 5e-3, np.zeros(3), np.zeros(H * W, np.uint8), th, s)
    Lap = _grid_laplacian(H, W, offsets)
    np.testing.assert_allclose(dv, -w * (Lap @ s[:3].T).T, rtol=0, atol=1e-13)


def test_isru_and_derivative_branches_closed_form():
    """A 1 x 2 cloth: node 0 sees only its right neighbour (channel 0), node 1 only its left one
    (channel 1). Differences placed at Pythagorean points give sigma = 3/5 and 4/5 exactly."""
    s = np.zeros((6, 2))
    s[:3, 1] = [0.75, 4.0 / 3.0, 0.0]       # x_1 - x_0
    s[3:, 1] = [2.0, -1.0, 0.5]             # v_1 - v_0
    wn, wd = 0.9, -1.3
    th = _theta(s=np.ones(12), wN=[wn] * 12, wD=[wd] * 12, bL=[0.1, 0.2, 0.3])
    _, dv = oracle.pair_forward(1, 2, 1.0, 5e-3, np.zeros(3), np.zeros(2, np.uint8), th, s)
    sig = np.array([0.6, 0.8, 0.0])
    e = np.array([2.0, -1.0, 0.5])
    np.testing.assert_allclose(dv[:, 0], [0.1, 0.2, 0.3] + wn * sig + wd * e * sig, rtol=0, atol=1e-15)
    # node 1: differences change sign; sigma is odd and xi changes sign too
    np.testing.assert_allclose(dv[:, 1], [0.1, 0.2, 0.3] - wn * sig + wd * e * sig, rtol=0, atol=1e-15)


def test_filter_scale_enters_the_activation():
    """phi = s (x_j - x_i): doubling s with wN halved is not the same map (the ISRU saturates),
    while for the linear branch it is."""
    s = np.zeros((6, 2))
    s[:3, 1] = [1.0, 0.0, 0.0]
    a = oracle.pair_forward(1, 2, 1.0, 5e-3, np.zeros(3), np.zeros(2, np.uint8), _theta(s=[1.0] * 12, wL=[1.0] * 12), s)[1]
    b = oracle.pair_forward(1, 2, 1.0, 5e-3, np.zeros(3), np.zeros(2, np.uint8), _theta(s=[2.0] * 12, wL=[0.5] * 12), s)[1]
    np.testing.assert_allclose(a, b, rtol=1e-15)
    c = oracle.pair_forward(1, 2, 1.0, 5e-3, np.zeros(3), np.zeros(2, np.uint8), _theta(s=[1.0] * 12, wN=[1.0] * 12), s)[1]
    d = oracle.pair_forward(1, 2, 1.0, 5e-3, np.zeros(3), np.zeros(2, np.uint8), _theta(s=[2.0] * 12, wN=[0.5] * 12), s)[1]
    assert abs(c[0, 0] - 1 / math.sqrt(2)) < 1e-15 and abs(d[0, 0] - 0.5 * 2 / math.sqrt(5)) < 1e-15


def test_translation_invariance_in_position_and_velocity():
    """Every feature is a difference with the centre: shifting all positions, or all velocities,
    by a constant leaves dv unchanged."""
    H, W = 6, 5
    th = I.random_array((51,), seed=5, scale=0.8)
    s = _state(H, W, 7)
    pin = np.zeros(H * W, np.uint8)
    _, d0 = oracle.pair_forward(H, W, 1.0, 5e-3, np.zeros(3), pin, th, s)
    s2 = s.copy()
    s2[:3] += np.array([[3.0], [-1.0], [0.25]])
    s2[3:] += np.array([[0.5], [0.5], [-2.0]])
    _, d1 = oracle.pair_forward(H, W, 1.0, 5e-3, np.zeros(3), pin, th, s2)
    np.testing.assert_allclose(d1, d0, rtol=0, atol=1e-13)


def test_frame_applies_eq5_with_pins_wind_and_pressure():
    H, W, dt = 4, 5, 5e-3
    th = I.random_array((51,), seed=9, scale=0.5)
    s = _state(H, W, 11)
    pin = I.pin_mask(H, W, "two_top_corners")
    a = np.array([0.3, -0.2, 0.1])
    out, dv = oracle.pair_forward(H, W, 1.0, dt, a, pin, th, s)
    v = s[3:] + dv + dt * a[:, None]
    v[:, pin == 1] = 0.0
    np.testing.assert_allclose(out[3:], v, rtol=0, atol=1e-15)
    np.testing.assert_allclose(out[:3], s[:3] + dt * v, rtol=0, atol=1e-15)
    # pressure adds dt pm f_p at the positions of S^k (f_p from the simulator's force with only p)
    m = I.Material()
    m.k_struct = m.k_shear = m.k_bend = m.mu = m.drag = 0.0
    m.g = (0.0, 0.0, 0.0)
    fp = oracle.ms_force(H, W, 0.1, 1.0, np.zeros(3), np.zeros(H * W, np.uint8), s, m, pressure=2.0)
    outp, _ = oracle.pair_forward(H, W, 1.0, dt, a, pin, th, s, pm=2.0)
    v2 = v + dt * fp
    v2[:, pin == 1] = 0.0
    np.testing.assert_allclose(outp[3:], v2, rtol=0, atol=1e-14)


@pytest.mark.parametrize("pm", [0.0, 30.0])
def test_backward_finite_differences(pm):
    """Central differences of a random linear functional of one frame, with respect to every
    parameter and to sampled state entries."""
    H, W, dt = 6, 7, 5e-3
    th = I.random_array((51,), seed=21, scale=0.6)
    th[PS:PS + 12] = 20.0 + I.random_array((12,), seed=22, scale=5.0)  # phi of order 1
    pin = I.pin_mask(H, W, "two_top_corners")
    a = np.array([0.4, -0.3, 0.0])
    s = _state(H, W, 23)
    tg = I.random_array((6, H * W), seed=24)

    def L(th_=th, s_=s):
        out, _ = oracle.pair_forward(H, W, 1.0, dt, a, pin, th_, s_, pm=pm)
        return float(np.sum(tg * out))

    gc, gt = oracle.pair_backward(H, W, 1.0, dt, pin, th, s, tg, pm=pm)
    fd = np.zeros(51)
    for k in range(51):
        e = 1e-6 * max(1.0, abs(th[k]))
        tp, tm = th.copy(), th.copy()
        tp[k] += e
        tm[k] -= e
        fd[k] = (L(th_=tp) - L(th_=tm)) / (2 * e)
    np.testing.assert_allclose(gt, fd, rtol=0, atol=1e-6 * np.abs(gt).max())
    rs = np.random.RandomState(2)
    scale = max(1.0, np.abs(gc).max())
    for flat in rs.choice(6 * H * W, 50, replace=False):
        c, p = divmod(int(flat), H * W)
        e = 1e-6
        sp_, sm_ = s.copy(), s.copy()
        sp_[c, p] += e
        sm_[c, p] -= e
        fdv = (L(s_=sp_) - L(s_=sm_)) / (2 * e)
        assert abs(fdv - gc[c, p]) <= 1e-6 * scale, (c, p, fdv, gc[c, p])
