"""The complex64 phase's fp32 argument reduction (tile_device.h, phase_cs for
float cost entries), emulated step by step in numpy with the constants read
from the kernel source: pi/2 split into two 12-bit parts and a remainder, so
that k * P1 and k * P2 are exact for |k| < 2^12, and the reduced argument within
1.5 fp32 ulps of pi/4 of the exact one for every product with |g1 C| < 4096."""
import os
import re

import numpy as np

SRC = os.path.join(os.path.dirname(__file__), "..", "paper_2407_13012_amd", "csrc", "tile_device.h")
f32 = np.float32


def _constants():
    text = open(SRC).read()
    body = text[text.index("void phase_cs(double g, float cval"):]
    body = body[:body.index("} else {")]
    two_over_pi = float.fromhex(re.search(r"rintf\(p \* (0x[0-9a-fp.+-]+)f\)", body).group(1))
    parts = [float.fromhex(h) for h in re.findall(r"fmaf\(-k, (-?0x[0-9a-fp.+-]+)f", body)]
    assert len(parts) == 3
    return two_over_pi, parts


def _fma32(a, b, c):
    # a * b is exact in fp64 for fp32 operands; one rounding to fp32, as an FMA
    return f32(np.float64(a) * np.float64(b) + np.float64(c))


def _significant_bits(x):
    m, _ = np.frexp(abs(x))
    bits = 0
    while m != int(m):
        m *= 2
        bits += 1
    return bits


def test_split_of_half_pi():
    two_over_pi, (p1, p2, p3) = _constants()
    assert float(f32(two_over_pi)) == two_over_pi and abs(two_over_pi - 2 / np.pi) < 1e-7
    assert _significant_bits(p1) <= 12 and _significant_bits(p2) <= 12
    assert float(f32(p3)) == p3
    assert abs((p1 + p2 + p3) - np.pi / 2) < 1e-15


def test_reduced_argument_error_bound():
    two_over_pi, (p1, p2, p3) = _constants()
    rng = np.random.default_rng(7)
    worst = 0.0
    for _ in range(40000):
        g = rng.uniform(-np.pi, np.pi)
        c = f32(rng.uniform(-1300.0, 1300.0) if rng.random() < 0.5 else rng.normal(0.0, 50.0))
        g1 = f32(g)
        g2 = f32(g - np.float64(g1))
        p = f32(g1 * c)
        if abs(p) >= 4096:
            continue
        pe = _fma32(g1, c, -p)
        k = f32(np.rint(f32(p * f32(two_over_pi))))
        r = _fma32(-k, f32(p1), p)
        r = _fma32(-k, f32(p2), r)
        r = _fma32(-k, f32(p3), r)
        r = f32(r + f32(pe + f32(g2 * c)))
        exact = g * np.float64(c) - np.float64(k) * (np.pi / 2)
        worst = max(worst, abs(float(r) - exact))
        assert abs(float(r)) < np.pi / 4 + 1e-3
    assert worst <= 1.5 * float(np.spacing(f32(np.pi / 4))), worst
