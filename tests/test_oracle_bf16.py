"""Pins of the oracle's bf16 emulation (the expected values of every bf16 parity check).

bf16_round: hand-derived IEEE cases (ties to even in both directions, values just off a tie,
negatives, subnormals, a carry into the exponent, overflow to infinity, specials) and agreement
with torch's own float32 -> bfloat16 conversion (round to nearest even) over random encodings.

cnn_forward(emu=...): each flag rounds exactly the operands it names. Tiny cells on a 1 x 2
cloth where every value is picked so that the rounded and unrounded paths give different,
hand-derivable velocity increments.
"""
import numpy as np
import pytest

import oracle

E = 2.0 ** -8


def test_bf16_round_hand_cases():
    cases = [
        (1.0, 1.0),
        (1 + E, 1.0),                       # tie, lower neighbour even
        (1 + 3 * E, 1 + 2 * 2 * E),         # tie, upper neighbour (1 + 2^-6) even
        (1 + E + 2.0 ** -20, 1 + 2 * E),    # just above a tie: up
        (1 + E - 2.0 ** -20, 1.0),          # just below a tie: down
        (-(1 + 3 * E), -(1 + 4 * E)),       # sign kept, magnitude rounded
        (-(1 + E), -1.0),
        (2 - E, 2.0),                       # tie at the top of the binade: carry into the exponent
        (2 - 2 * E, 2 - 2 * E),             # largest bf16 below 2 is kept
        (0.6, 0.6015625),                   # 0.10011001100..b -> 0.1001101b
        (3.0 * 2.0 ** -134, 2.0 ** -132),   # subnormal tie: 0x18000 -> even 0x20000
        (2.0 ** -134, 0.0),                 # subnormal tie: 0x08000 -> even 0x00000
        (2.0 ** -133, 2.0 ** -133),         # a bf16 subnormal is kept
        (2.0 ** -149, 0.0),                 # the smallest float32 subnormal rounds to zero
        ((2.0 ** 23 - 1) * 2.0 ** -149, 2.0 ** -126),  # largest subnormal -> smallest normal
        (np.float32(3.4028234663852886e38), np.inf),   # largest float32 -> past bf16's largest
        (3.3895313892515355e38, 3.3895313892515355e38),  # bf16's largest finite value is kept
        (0.0, 0.0),
        (np.inf, np.inf),
        (-np.inf, -np.inf),
    ]
    x = np.array([c[0] for c in cases], dtype=np.float64)
    want = np.array([c[1] for c in cases], dtype=np.float64)
    got = oracle.bf16_round(x)
    for xi, gi, wi in zip(x, got, want):
        assert gi == wi, (xi, gi, wi)
    z = oracle.bf16_round(np.array([-0.0, np.nan]))
    assert z[0] == 0.0 and np.signbit(z[0]) and np.isnan(z[1])


def test_bf16_round_matches_torch_conversion():
    """Against torch's CPU float32 -> bfloat16 conversion (round to nearest even) on random
    float32 encodings of every exponent, including subnormals (NaNs left out)."""
    torch = pytest.importorskip("torch")
    rng = np.random.default_rng(12)
    bits = rng.integers(0, 2 ** 32, size=1 << 20, dtype=np.uint64).astype(np.uint32)
    # plus encodings whose lower 16 bits sit at, just below and just above the halfway point
    hi = rng.integers(0, 2 ** 16, size=1 << 14, dtype=np.uint64).astype(np.uint32) << 16
    bits = np.concatenate([bits, hi | 0x8000, hi | 0x7FFF, hi | 0x8001, hi])
    f = bits.view(np.float32)
    f = f[~np.isnan(f)]
    ref = torch.from_numpy(f.copy()).to(torch.bfloat16).to(torch.float32).numpy().astype(np.float64)
    got = oracle.bf16_round(f.astype(np.float64))
    same = (got == ref) | (np.isnan(got) & np.isnan(ref))
    assert same.all(), f[~same][:8]


def _pair_inputs():
    """1 x 2 cloth: node 0 at the origin, node 1 one unit east, at rest (S^{k-1} = S^k)."""
    s = np.zeros((6, 2))
    s[0, 1] = 1.0
    return s


def _theta(ch=16, kw=1.0, A=0.0, B=0.0, wl=0.0, wn=0.0):
    th = np.zeros(oracle.theta_size(ch))
    K, Ao = 0, ch * 54
    Bo = Ao + ch * ch
    WL = Bo + ch * ch
    WN = WL + 3 * ch
    th[K + 0 * 54 + 0 * 9 + 5] = kw      # K[0][x][dy = 0][dx = +1]: the east neighbour's x difference
    th[Ao + 0] = A                       # A[0][0]
    th[Bo + 0] = B                       # B[0][0]
    th[WL + 0] = wl                      # W_L[x][0]
    th[WN + 0] = wn                      # W_N[x][0]
    return th


def _dvx(th, s, emu):
    _, dv = oracle.cnn_forward(1, 2, 16, 1.0, 5e-3, np.zeros(3), np.zeros(2, np.uint8), th, s, s, emu=emu)
    return dv[0, 0]


def test_emu_bit0_rounds_conv_operands():
    """Bit 0 rounds the conv weights and the im2col entries. L branch only: dv_x = W_L phi_0 with
    phi_0 = K (x_1 - x_0). K = 1 - 2^-9 rounds to 1 (tie, even) and x_1 - x_0 = 1 + 3 2^-8 rounds
    to 1 + 2^-6; unrounded, the product 1 + 2.5 2^-8 - ... lies below the midpoint 1 + 3 2^-8, so
    bit 2 alone (the head operand) takes it to 1 + 2^-7 instead."""
    s = _pair_inputs()
    s[0, 1] = 1 + 3 * E
    th = _theta(kw=1 - E / 2, wl=1.0)
    assert _dvx(th, s, 1) == 1 + 4 * E
    assert _dvx(th, s, 5) == 1 + 4 * E
    assert _dvx(th, s, 4) == 1 + 2 * E
    assert _dvx(th, s, 0) == (1 - E / 2) * (1 + 3 * E)


def test_emu_bit1_rounds_mix_operands():
    """Bit 1 rounds A, B and phi in the two Ch x Ch maps. phi_0 = 1 exactly; A = 1 + 2^-8 rounds to
    1 and B = 0.75 (1 + 2^-9) rounds to 0.75, so z = a b = 3/4 and n = sigma(3/4) = 3/5."""
    s = _pair_inputs()
    th = _theta(kw=1.0, A=1 + E, B=0.75 * (1 + E / 2), wn=1.0)
    assert _dvx(th, s, 2) == 0.6
    z = (1 + E) * 0.75 * (1 + E / 2)
    assert abs(_dvx(th, s, 0) - z / np.sqrt(1 + z * z)) <= 1e-15
    assert _dvx(th, s, 0) != 0.6


def test_emu_bit2_rounds_head_operands():
    """Bit 2 rounds the head weights and the features they multiply. With phi_0 = 1, A = 1,
    B = 0.75: n = 3/5, which rounds to 0.6015625; W_L = 1 + 2^-8 + 2^-12 rounds up to 1 + 2^-7."""
    s = _pair_inputs()
    th = _theta(kw=1.0, A=1.0, B=0.75, wl=1 + E + 2.0 ** -12, wn=1.0)
    assert _dvx(th, s, 4) == (1 + 2 * E) + 0.6015625
    assert abs(_dvx(th, s, 0) - ((1 + E + 2.0 ** -12) + 0.6)) <= 1e-15
    # all three flags: the conv and mix operands here are already bf16 values
    assert _dvx(th, s, 7) == (1 + 2 * E) + 0.6015625
