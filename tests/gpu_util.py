"""Shared helpers of the GPU tests (inputs and tolerances; no method arithmetic)."""
import math

import numpy as np

from paper_2403_12820_amd import inputs as I

U32 = 2.0 ** -24


def dev_tensor(a, dtype=None):
    import torch
    a = np.ascontiguousarray(a)
    t = torch.from_numpy(a.astype(np.float32) if dtype is None and a.dtype == np.float64 else a)
    return t.to("cuda")


def ragged_sizes():
    """Tile-edge coverage: single spring, tiny, prime, one-row and wide, several tiles with a ragged tail."""
    return [(1, 2), (2, 2), (17, 23), (2, 257), (33, 65), (5, 3), (64, 64), (3, 70)]


def aligned_sizes():
    """Every width a multiple of 4 (16-byte row pieces), with tiles crossing the right and bottom
    grid edges: tiny, one-row, tall, and several tiles with ragged tails."""
    return [(4, 4), (9, 20), (33, 68), (2, 132), (17, 36), (64, 64), (3, 100), (40, 12)]


def wide_sizes():
    """Every width at least 4, most not a multiple of 4 (16-byte row pieces at 4-byte alignment):
    widths 4 to 7 (one piece crossing the right edge by 0 to 3 columns), several tiles with
    ragged tails, and instance offsets that are not multiples of 4."""
    return [(5, 4), (3, 5), (7, 6), (2, 7), (17, 23), (33, 65), (64, 64), (9, 130), (40, 13), (3, 70)]


SIZE_SETS = {"ragged": ragged_sizes, "aligned": aligned_sizes, "wide": wide_sizes}


def perturbed_batch(sizes, seed, vel=0.05, pos=0.15, mat=None):
    """Random scenes with deformed positions and random velocities (float32 state)."""
    scenes = I.random_scenes(sizes, seed, noise_sigma=1e-3, mat=mat)
    batch = I.make_batch(scenes)
    s = batch.state.astype(np.float64)
    h = float(batch.h[0])
    s[:3] += I.random_array((3, batch.total), seed=seed + 11, scale=pos * h)
    s[3:] = I.random_array((3, batch.total), seed=seed + 12, scale=vel)
    batch.state = s.astype(np.float32)
    return batch


def ms_velocity_floor(batch, mat, strain=0.3):
    """Worst-case FP32 rounding of one step's velocity: each spring length r is formed with a few
    roundings (|dr| <= 4 u r), so |df| <= 4 u sum_j k_j r_j over the 12 springs, times dt/m."""
    h = float(np.max(batch.h))
    m = float(np.min(batch.mass))
    ksum = 4 * (mat.k_struct * h + mat.k_shear * math.sqrt(2) * h + mat.k_bend * 2 * h) * (1 + strain)
    return 4 * U32 * ksum * mat.dt / m


def rel_inf(a, b):
    return float(np.abs(a - b).max() / max(np.abs(b).max(), 1e-300))
