"""Pins of the oracle's 8-bit frame output (the "Image I/O" phase, Table 5):
floor(clamp(v, 0, 1) * 255 + 1/2), NaN -> 0.  Checked against exact rational
arithmetic and hand-worked values."""
import math
from fractions import Fraction

import numpy as np


def _exact(v: float) -> int:
    if math.isnan(v) or v <= 0.0:
        return 0
    if v >= 1.0:
        return 255
    return math.floor(Fraction(v) * 255 + Fraction(1, 2))


def test_quantize_hand_values(oracle_mod):
    v = np.array([0.0, -0.0, 1.0, 0.5, 0.25, 0.75, 1.0 / 256, 3.0 / 512, -1.0, 2.0,
                  np.inf, -np.inf, np.nan, 1e-30], dtype=np.float32)
    # 0.5 * 255 = 127.5 rounds up; 0.25 -> 63.75; 0.75 -> 191.25; 1/256 -> 0.996;
    # 3/512 -> 1.494
    want = [0, 0, 255, 128, 64, 191, 1, 1, 0, 255, 255, 0, 0, 0]
    assert oracle_mod.quantize_rgb8(v).tolist() == want


def test_quantize_levels_round_trip(oracle_mod):
    k = np.arange(256)
    v = (k / 255.0).astype(np.float32)
    assert np.array_equal(oracle_mod.quantize_rgb8(v), k.astype(np.uint8))


def test_quantize_matches_exact_rationals(oracle_mod):
    rng = np.random.default_rng(3)
    v = rng.uniform(-0.1, 1.1, 4000).astype(np.float32)
    # values next to every rounding boundary (k + 1/2) / 255, both sides
    b = ((np.arange(255) + 0.5) / 255.0).astype(np.float32)
    v = np.concatenate([v, b, np.nextafter(b, np.float32(0)), np.nextafter(b, np.float32(1))])
    got = oracle_mod.quantize_rgb8(v)
    assert got.tolist() == [_exact(float(x)) for x in v]
