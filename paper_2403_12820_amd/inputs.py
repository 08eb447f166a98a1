"""Seeded synthetic inputs for cloth scenes.

This module is the only code that the oracle tests, the GPU parity tests and
the benchmark have in common. It holds none of the method's arithmetic: a
counter-based random stream (splitmix64, Steele/Lea/Flood 2014, with the
Box-Muller transform for normals), the flat rest grid of a mass-spring cloth
(section 3.1: a regular grid of mass points), pin sets, wind draws, z-noise and
the random initial network weights.

State layout used everywhere: six float planes [x0, x1, x2, v0, v1, v2], each a
row-major H x W grid; several cloths are concatenated along the node axis, so a
batch state is a [6, N_total] float32 array.
"""
from __future__ import annotations

from dataclasses import dataclass, field
import math

import numpy as np

_M64 = (1 << 64) - 1
_GAMMA = 0x9E3779B97F4A7C15

# Tags that separate independent streams drawn from one seed.
TAG_NOISE, TAG_THETA, TAG_SCENE, TAG_SIZE, TAG_WINDOW, TAG_MISC = 1, 2, 3, 4, 5, 6


def _mix64_np(z: np.ndarray) -> np.ndarray:
    """The splitmix64 output function on a uint64 array (wrapping arithmetic)."""
    z = z.astype(np.uint64, copy=True)
    with np.errstate(over="ignore"):
        z = (z ^ (z >> np.uint64(30))) * np.uint64(0xBF58476D1CE4E5B9)
        z = (z ^ (z >> np.uint64(27))) * np.uint64(0x94D049BB133111EB)
        z = z ^ (z >> np.uint64(31))
    return z


def _mix64_int(z: int) -> int:
    z &= _M64
    z = ((z ^ (z >> 30)) * 0xBF58476D1CE4E5B9) & _M64
    z = ((z ^ (z >> 27)) * 0x94D049BB133111EB) & _M64
    return z ^ (z >> 31)


_CHUNK = 1 << 20


class Stream:
    """Counter-based splitmix64 stream: value n is mix64(base + (n+1)*gamma)."""

    def __init__(self, seed: int, tag: int = 0):
        self.base = _mix64_int((seed & _M64) ^ ((tag * 0xD1B54A32D192ED03) & _M64))
        self.pos = 0

    def u64(self, n: int) -> np.ndarray:
        idx = np.arange(self.pos + 1, self.pos + n + 1, dtype=np.uint64)
        self.pos += n
        with np.errstate(over="ignore"):
            z = np.uint64(self.base) + idx * np.uint64(_GAMMA)
        return _mix64_np(z)

    def uniform(self, n: int) -> np.ndarray:
        """Doubles in [0, 1) from the top 53 bits."""
        out = np.empty(n, np.float64)
        for a in range(0, n, _CHUNK):  # in cache-sized pieces: same values, far fewer page faults
            m = min(_CHUNK, n - a)
            out[a:a + m] = (self.u64(m) >> np.uint64(11)).astype(np.float64) * (1.0 / 9007199254740992.0)
        return out

    def normal(self, n: int) -> np.ndarray:
        """Standard normals by Box-Muller, one pair of uniforms per value (cosine branch)."""
        out = np.empty(n, np.float64)
        for a in range(0, n, _CHUNK):
            m = min(_CHUNK, n - a)
            u = self.uniform(2 * m).reshape(m, 2)
            out[a:a + m] = np.sqrt(-2.0 * np.log1p(-u[:, 0])) * np.cos(2.0 * math.pi * u[:, 1])
        return out


# --------------------------------------------------------------------------- material
@dataclass
class Material:
    """Cloth material of the mass-spring model (eqs. 1, 2, 4, 5).

    Defaults: 32 x 32 nodes span a unit square (h = 1/31), node mass 1/1024,
    spring constants structural/shear/bend = 1000/500/100, spring damping 0.01,
    no air drag, gravity 9.8 perpendicular to the flat cloth, dt = 5e-4.
    """
    h: float = 1.0 / 31.0
    mass: float = 1.0 / 1024.0
    k_struct: float = 1000.0
    k_shear: float = 500.0
    k_bend: float = 100.0
    mu: float = 0.01
    drag: float = 0.0
    g: tuple = (0.0, 0.0, -9.8)
    dt: float = 5e-4


PIN_KINDS = ("two_top_corners", "four_corners", "one_top_corner", "top_edge", "none")


def pin_mask(H: int, W: int, kind: str) -> np.ndarray:
    """uint8 [H*W]; row 0 is the top edge."""
    m = np.zeros((H, W), np.uint8)
    if kind == "two_top_corners":
        m[0, 0] = m[0, W - 1] = 1
    elif kind == "four_corners":
        m[0, 0] = m[0, W - 1] = m[H - 1, 0] = m[H - 1, W - 1] = 1
    elif kind == "one_top_corner":
        m[0, 0] = 1
    elif kind == "top_edge":
        m[0, :] = 1
    elif kind == "none":
        pass
    else:
        raise ValueError(kind)
    return m.reshape(-1)


def flat_grid(H: int, W: int, h: float) -> np.ndarray:
    """Rest positions X_ij = (j h, i h, 0), float64 [3, H*W]."""
    i, j = np.meshgrid(np.arange(H, dtype=np.float64), np.arange(W, dtype=np.float64), indexing="ij")
    return np.stack([j * h, i * h, np.zeros_like(i)]).reshape(3, H * W)


@dataclass
class Scene:
    H: int
    W: int
    h: float
    mass: float
    a_ext: np.ndarray           # float64 [3], constant wind acceleration
    pin: np.ndarray             # uint8 [H*W]
    state: np.ndarray           # float32 [6, H*W]
    pin_kind: str = ""
    pressure: float = 0.0       # uniform pressure of eq. (3), N/m^2 (float32 value)

    @property
    def n(self) -> int:
        return self.H * self.W


def make_scene(H: int, W: int, pin_kind: str = "two_top_corners", wind=(0.0, 0.0, 0.0),
               noise_sigma: float = 1e-3, seed: int = 0, mat: Material | None = None,
               v0=None, pressure: float = 0.0) -> Scene:
    """Flat cloth at rest plus z-noise N(0, sigma^2) on unpinned nodes (one draw per node, p = i*W + j)."""
    mat = mat or Material()
    X = flat_grid(H, W, mat.h)
    pin = pin_mask(H, W, pin_kind)
    if noise_sigma > 0:
        z = Stream(seed, TAG_NOISE).normal(H * W) * noise_sigma
        X[2] += np.where(pin == 1, 0.0, z)
    s = np.zeros((6, H * W), np.float32)
    s[:3] = X.astype(np.float32)
    if v0 is not None:
        s[3:] = np.asarray(v0, np.float32).reshape(3, -1)
    return Scene(H, W, float(np.float32(mat.h)), float(np.float32(mat.mass)),
                 np.asarray(wind, np.float64), pin, s, pin_kind, float(np.float32(pressure)))


def random_scene_params(n: int, seed: int):
    """Per scene: pin set uniform over the four pinned kinds, wind |a| ~ U[0, 2] m/s^2 along a
    horizontal direction angle ~ U[0, 2 pi) (horizontal = perpendicular to gravity along -z)."""
    st = Stream(seed, TAG_SCENE)
    u = st.uniform(3 * n).reshape(n, 3)
    kinds = [PIN_KINDS[min(int(x * 4), 3)] for x in u[:, 0]]
    mag = 2.0 * u[:, 1]
    ang = 2.0 * math.pi * u[:, 2]
    winds = np.stack([mag * np.cos(ang), mag * np.sin(ang), np.zeros(n)], 1)
    return kinds, winds


def random_scenes(sizes, seed: int, noise_sigma: float = 1e-3, mat: Material | None = None):
    """A list of scenes with the given (H, W) sizes, random pins and wind, z-noise seeded per scene."""
    kinds, winds = random_scene_params(len(sizes), seed)
    out = []
    for b, (H, W) in enumerate(sizes):
        out.append(make_scene(H, W, kinds[b], winds[b], noise_sigma, seed=seed * 1000003 + b, mat=mat))
    return out


def loguniform_sizes(n: int, lo: int = 16, hi: int = 256, seed: int = 2):
    """Square side N = round(exp(U(ln lo, ln hi)))."""
    u = Stream(seed, TAG_SIZE).uniform(n)
    N = np.rint(np.exp(math.log(lo) + u * (math.log(hi) - math.log(lo)))).astype(int)
    return [(int(x), int(x)) for x in N]


# --------------------------------------------------------------------------- batches
@dataclass
class Batch:
    """Several scenes concatenated along the node axis."""
    H: np.ndarray               # int32 [n]
    W: np.ndarray               # int32 [n]
    h: np.ndarray               # float32 [n]
    mass: np.ndarray            # float32 [n]
    a_ext: np.ndarray           # float32 [n, 3]
    pin: np.ndarray             # uint8 [N_total]
    state: np.ndarray           # float32 [6, N_total]
    node_off: np.ndarray = field(default=None)  # int64 [n+1]
    pressure: np.ndarray = field(default=None)  # float32 [n], eq. (3)
    sphere: np.ndarray = field(default=None)    # float32 [n, 5]: centre, radius (0: none), friction

    @property
    def n(self) -> int:
        return len(self.H)

    @property
    def total(self) -> int:
        return int(self.node_off[-1])

    def instance(self, b: int):
        a, e = int(self.node_off[b]), int(self.node_off[b + 1])
        return slice(a, e)


def make_batch(scenes) -> Batch:
    H = np.array([s.H for s in scenes], np.int32)
    W = np.array([s.W for s in scenes], np.int32)
    off = np.zeros(len(scenes) + 1, np.int64)
    off[1:] = np.cumsum(H.astype(np.int64) * W)
    return Batch(H, W,
                 np.array([s.h for s in scenes], np.float32),
                 np.array([s.mass for s in scenes], np.float32),
                 np.array([s.a_ext for s in scenes], np.float32).reshape(-1, 3),
                 np.concatenate([s.pin for s in scenes]).astype(np.uint8),
                 np.concatenate([s.state for s in scenes], axis=1).astype(np.float32),
                 off,
                 np.array([getattr(s, "pressure", 0.0) for s in scenes], np.float32))


# --------------------------------------------------------------------------- weights
def theta_size(ch: int) -> int:
    """Parameter count of the cell: conv Ch*6*3*3, two Ch x Ch maps, three 3 x Ch heads, bias 3."""
    return ch * 54 + 2 * ch * ch + 9 * ch + 3


def init_theta(ch: int, seed: int = 1, std: float = 0.02) -> np.ndarray:
    """Every entry N(0, std^2), drawn in flat parameter order."""
    return (Stream(seed, TAG_THETA).normal(theta_size(ch)) * std).astype(np.float32)


PAIR_THETA_SIZE = 51  # pair cell: s[12] | wL[12] | wN[12] | wD[12] | b_L[3]


def init_pair_theta(seed: int = 1, std: float = 0.02, h: float = 1.0 / 31.0) -> np.ndarray:
    """Pair cell: filter scales s_c = 1 / rest length of the channel's link (so that a link at
    rest gives |phi| = 1 along it), branch weights N(0, std^2) in flat order, bias 0."""
    th = Stream(seed, TAG_THETA).normal(PAIR_THETA_SIZE) * std
    rest = np.array([1.0] * 4 + [math.sqrt(2.0)] * 4 + [2.0] * 4) * h
    th[0:12] = 1.0 / rest
    th[48:51] = 0.0
    return th.astype(np.float32)


def random_array(shape, seed: int, scale: float = 1.0, tag: int = TAG_MISC) -> np.ndarray:
    n = int(np.prod(shape))
    return (Stream(seed, tag).normal(n) * scale).reshape(shape)
