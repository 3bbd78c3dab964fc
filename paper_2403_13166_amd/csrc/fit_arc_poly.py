"""Coefficients of the arc-length polynomial used by the FP32 cuts.

The arc length of a helix from the beam line to radius r at half-curvature c
is asin(c r) / c = r * g((c r)^2) with g(t) = asin(sqrt(t)) / sqrt(t). For
c r <= 0.8 the kernels evaluate g as a degree-10 polynomial in t by Horner's
rule. This script fits it (least squares on Chebyshev nodes, reweighted toward
equal-ripple relative error) and prints the coefficients (constant first) and
the worst relative error of the FP32 evaluation on a dense grid.
"""
import numpy as np

T_MAX = 0.64          # t = x^2 for x <= 0.8
DEGREE = 10


def g(t):
    x = np.sqrt(t)
    return np.where(t > 0, np.arcsin(x) / np.where(x > 0, x, 1.0), 1.0)


def fit(degree=DEGREE, t_max=T_MAX):
    k = np.arange(4 * degree)
    nodes = 0.5 * t_max * (1 - np.cos(np.pi * (k + 0.5) / len(k)))
    A = np.vander(nodes, degree + 1, increasing=True)
    w = np.ones_like(nodes)
    for _ in range(30):
        coef, *_ = np.linalg.lstsq(A * w[:, None], g(nodes) * w, rcond=None)
        err = np.abs(A @ coef - g(nodes))
        w = w * (err / err.max() + 1e-3) ** 0.5
        w /= w.max()
    return coef


def horner_f32(coef, t):
    c = np.asarray(coef, np.float32)
    t = np.asarray(t, np.float32)
    acc = np.full_like(t, c[-1])
    for ck in c[-2::-1]:
        acc = (acc * t + ck).astype(np.float32)
    return acc


if __name__ == "__main__":
    coef = fit()
    grid = np.linspace(0.0, T_MAX, 400001)
    rel = np.max(np.abs(horner_f32(coef, grid).astype(np.float64) - g(grid.astype(np.float32).astype(np.float64)))
                 / g(grid))
    print(", ".join(f"{float(np.float32(c)):.9e}f" for c in coef))
    print(f"max relative error (FP32 Horner): {rel:.2e}")
