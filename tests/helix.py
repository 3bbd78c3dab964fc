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


def threshold_event(geo, seed, n_min=300, n_high=60, n_noise=400):
    """Noise-free tracks at pT_min with z_v = +-Z on the side of their eta
    (on the selection envelope), tracks of pT 5-20 GeV from the origin (far
    from every threshold), and noise hits on the outer sensors of modules
    those tracks cross (candidates far outside the cuts). Hits are FP32."""
    rng = np.random.default_rng(seed)
    Z, pmin = geo.params["z_lum"], geo.params["pt_min"]
    eta1 = rng.uniform(-2.3, 2.3, n_min)
    t1 = np.stack([np.where(rng.random(n_min) < 0.5, -1.0, 1.0), np.full(n_min, pmin), eta1,
                   rng.uniform(0, 2 * math.pi, n_min), np.where(eta1 >= 0, Z, -Z)], axis=1)
    t2 = np.stack([np.where(rng.random(n_high) < 0.5, -1.0, 1.0), rng.uniform(5.0, 20.0, n_high),
                   rng.uniform(-2.3, 2.3, n_high), rng.uniform(0, 2 * math.pi, n_high), np.zeros(n_high)], axis=1)
    ev = events.make_event_from_tracks(geo, np.concatenate([t1, t2]), 0, 0.0, rng, shuffle=False)
    mods = np.unique(ev.sensor // 2)
    nm = rng.choice(mods, n_noise)
    p = geo.p[nm]
    phi = rng.uniform(p[:, 4], p[:, 5])
    bar = geo.kind[nm] == 0
    r = np.where(bar, p[:, 1], rng.uniform(p[:, 2], p[:, 3]))
    zz = np.where(bar, rng.uniform(p[:, 2], p[:, 3]), p[:, 1])
    x = np.concatenate([ev.x, (r * np.cos(phi)).astype(np.float32)])
    y = np.concatenate([ev.y, (r * np.sin(phi)).astype(np.float32)])
    z = np.concatenate([ev.z, zz.astype(np.float32)])
    s = np.concatenate([ev.sensor, (2 * nm + 1).astype(np.int32)])
    tr = np.concatenate([ev.truth, np.full(n_noise, -1, np.int32)])
    return events.Event(x, y, z, s, tr, ev.tracks)
