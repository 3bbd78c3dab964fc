"""Exact (FP64, noise-free) helix crossings for the oracle pins.

Independent of both implementations of the method: positions come from the
helix parametrisation of the event generator with smearing off.
"""
import math

import numpy as np

from paper_2403_13166_amd.synth import events


def crossings(geo, q, pt, eta, phi0, zv):
    """Noise-free hits of one track, ordered outward: list of (x, y, z, sensor)."""
    rng = np.random.default_rng(0)
    tr = np.array([[q, pt, eta, phi0, zv]], dtype=np.float64)
    xs, ys, zs, sens, _ = events._track_hits(geo, tr[:, 0], tr[:, 1], tr[:, 2], tr[:, 3], tr[:, 4],
                                             0.0, rng)
    order = np.argsort(np.hypot(xs, ys) + 1e-3 * np.abs(zs), kind="stable")
    return [(xs[i], ys[i], zs[i], int(sens[i])) for i in order]


def md_pairs(geo, hits):
    """Group crossings into (anchor, other) pairs of the same module, by layer."""
    by_mod = {}
    for h in hits:
        by_mod.setdefault(h[3] // 2, {})[h[3] % 2] = h
    out = []
    for m, d in by_mod.items():
        if 0 in d and 1 in d:
            out.append((int(geo.layer[m]), d[0], d[1]))
    out.sort(key=lambda t: t[0])
    return out


def layers_crossed(geo, hits):
    """Logical layers whose anchor sensor was crossed (module-edge splits included)."""
    return sorted({int(geo.layer[h[3] // 2]) for h in hits if h[3] % 2 == 0})


def half_curvature(geo, pt):
    return geo.params["k_b"] / (2.0 * pt)
