"""The FP32 arc-length polynomial of the cut kernels against asin.

The kernels evaluate asin(x) / x for 0 <= x <= 0.8 as a polynomial in x^2
(lst_device.h, asin_over_x_f). This reads its coefficients from the header,
evaluates it the way the kernel does (FP32 Horner with fused multiply-add
emulated in FP64 then rounded), and checks it against numpy's FP64 arcsin.
"""
import os
import re

import numpy as np

HDR = os.path.join(os.path.dirname(__file__), "..", "paper_2403_13166_amd", "csrc", "lst_device.h")


def _coefs():
    src = open(HDR).read()
    body = src[src.index("float asin_over_x_f(float t)"):]
    body = body[:body.index("}")]
    vals = [float(v) for v in re.findall(r"([-+]?\d\.\d+e[-+]\d+)f", body)]
    # Horner order in the source: highest degree first, then the constant 1.0f
    return vals + [1.0]


def _horner_f32(coefs, t):
    t = np.asarray(t, np.float32).astype(np.float64)
    g = np.full_like(t, np.float32(coefs[0]))
    for c in coefs[1:]:
        g = (g * t + np.float64(np.float32(c))).astype(np.float32).astype(np.float64)   # one rounding per fma
    return g


def test_polynomial_matches_asin_over_x():
    coefs = _coefs()
    assert len(coefs) == 11
    x = np.linspace(0.0, 0.8, 200001)
    t = (x * x).astype(np.float32)
    g = _horner_f32(coefs, t)
    xs = np.sqrt(t.astype(np.float64))
    ref = np.where(xs > 0, np.arcsin(xs) / np.where(xs > 0, xs, 1.0), 1.0)
    assert np.max(np.abs(g - ref) / ref) < 1.5e-7


def test_arc_length_limits():
    coefs = _coefs()
    # straight line: the arc length is the radius
    assert _horner_f32(coefs, [0.0])[0] == 1.0
    # a known value: asin(0.5) / 0.5 = pi / 3
    assert abs(_horner_f32(coefs, [0.25])[0] - np.pi / 3) < 2e-7
