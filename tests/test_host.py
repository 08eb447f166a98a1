"""Host-side logic that needs no GPU: the seeded input generator against the published
splitmix64 sequence, scene helpers, the library's host-only entry points, the benchmark's
refusal of several GPUs, and the profile summaries the benchmark reads."""
import ctypes as C
import os
import subprocess
import sys

import numpy as np

from paper_2403_12820_amd import _lib as L
from paper_2403_12820_amd import inputs as I

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


def test_splitmix64_matches_the_published_sequence():
    """Seed 0: the first outputs of splitmix64 (Steele, Lea and Flood; reference code by Vigna)."""
    got = [int(x) for x in I.Stream(0, 0).u64(4)]
    assert got == [0xE220A8397B1DCDAF, 0x6E789E6AA1B965F4, 0x06C45D188009454F, 0xF88BB8A8724C81EC]
    # counter-based: drawing in two pieces gives the same values
    s = I.Stream(7, 3)
    a = np.concatenate([s.u64(5), s.u64(6)])
    assert np.array_equal(a, I.Stream(7, 3).u64(11))


def test_uniform_and_normal_draws():
    u = I.Stream(1, 2).uniform(200_000)
    assert u.min() >= 0.0 and u.max() < 1.0 and abs(u.mean() - 0.5) < 0.005
    z = I.Stream(1, 3).normal(200_000)
    assert abs(z.mean()) < 0.01 and abs(z.std() - 1.0) < 0.01
    assert abs(np.mean(z ** 4) - 3.0) < 0.1  # Gaussian kurtosis


def test_scene_helpers():
    H, W = 6, 9
    counts = {k: int(I.pin_mask(H, W, k).sum()) for k in I.PIN_KINDS}
    assert counts == {"two_top_corners": 2, "four_corners": 4, "one_top_corner": 1, "top_edge": W, "none": 0}
    sizes = I.loguniform_sizes(512, 16, 256, seed=2)
    sides = np.array([s[0] for s in sizes])
    assert sides.min() >= 16 and sides.max() <= 256 and len(set(sides)) > 100
    sc = I.make_scene(5, 7, "four_corners", noise_sigma=1e-3, seed=0)
    assert np.all(sc.state[2][sc.pin == 1] == 0.0) and np.any(sc.state[2][sc.pin == 0] != 0.0)
    th = I.init_pair_theta(seed=1)
    assert th.size == I.PAIR_THETA_SIZE and abs(th[0] * I.Material().h - 1.0) < 1e-6


def test_host_only_entry_points():
    lib = L.lib()
    assert lib.pecnn_cell_theta_size(L.CELL_PAIR, 12) == 51
    assert lib.pecnn_cell_theta_size(L.CELL_PAIR, 16) == -1
    assert lib.pecnn_cell_theta_size(L.CELL_CONV, 16) == I.theta_size(16)
    assert lib.pecnn_cell_theta_size(7, 16) == -1
    p = np.zeros(4, np.float32)
    assert lib.pecnn_plan_set_pressure(None, p.ctypes.data, None) == -1
    assert lib.pecnn_plan_set_spheres(None, p.ctypes.data, None) == -1
    assert lib.pecnn_backward(None, None, None, None, None, None, None, None, None, 0, None) == -1


def test_position_exclusion_scale_vanishes_in_fp32():
    """The trainer's physics term passes a position scale whose inverse square is 0 in FP32."""
    from paper_2403_12820_amd.train import NO_POSITIONS
    sx = np.float32(NO_POSITIONS)
    with np.errstate(over="ignore"):
        assert np.float32(1.0) / (sx * sx) == 0.0
    assert np.isfinite(sx)


def test_bench_refuses_several_gpus():
    r = subprocess.run([sys.executable, os.path.join(ROOT, "bench.py"), "--gpus", "2"], capture_output=True,
                       text=True, timeout=120)
    assert r.returncode == 2 and "one GPU" in r.stderr


def test_profile_summaries_parse():
    from paper_2403_12820_amd import profile_summary as PS
    tr = PS.read_summary(os.path.join(ROOT, "profiles", "cnn_fwd_bf16_128x256x256_traffic.txt"))
    assert int(tr["nodes"]) == 8388608
    # measured bytes per node at or above the 73 algorithmic ones
    assert 73.0 <= float(tr["bytes_per_node"]) < 100.0
    ms = PS.read_summary(os.path.join(ROOT, "profiles", "ms_step_128x256x256_traffic.txt"))
    assert 49.0 <= float(ms["bytes_per_node"]) < 70.0
