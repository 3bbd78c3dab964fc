"""Seeded synthetic events: helical tracks from the beam line plus uniform noise.

Input generation only (no object-building arithmetic). A track of transverse
momentum pT and charge q in the solenoid field is a helix whose transverse
projection is a circle of radius R = pT / k_b through its vertex. With
transverse arc length s and direction angle psi(s) = phi0 - q s / R:

    x(s) = (R/q) (sin phi0 - sin(phi0 - q s/R))
    y(s) = (R/q) (cos(phi0 - q s/R) - cos phi0)
    z(s) = z_v + s sinh(eta)

Hits are recorded where the helix crosses a sensor surface (barrel cylinders,
endcap planes), smeared, and assigned to the module containing the smeared
point. Events mimic the workloads of the paper's Sec. 3 (HL-LHC pile-up)
with synthetic numbers: PU200-like occupancy is 6000 tracks + 100k noise hits.

Displaced workload (Sec. 3, the "muon-cube" sample): muons from vertices
uniform in a 5 cm cube centred on the nominal interaction point, so their
helices start at (x_v, y_v, z_v) instead of the beam line; each track then
carries x_v and y_v as two more truth columns.
"""
from __future__ import annotations

import math
from dataclasses import dataclass

import numpy as np

from .geometry import (BARREL_RADII, DISK_Z, RING_EDGES, BARREL_HALF_LENGTH, Geometry,
                       barrel_nphi, TWO_PI)


@dataclass
class EventConfig:
    """Workload recipe (all values in GeV, cm)."""
    name: str
    n_tracks: int
    invpt_lo: float
    invpt_hi: float
    eta_max: float
    zv_sigma: float        # 0 -> vertex at the origin
    n_noise: int
    with_endcap: bool
    sigma_scale: float = 1.0   # 0 -> noise-free hit positions
    cube: float = 0.0          # side of the vertex cube (x, y, z uniform); 0 -> vertices on the beam line


# Single barrel-only event of 100 tracks, pT in [1, 10] GeV, |eta| < 0.8.
SMALL_BARREL = EventConfig("small-barrel-100trk", 100, 0.1, 1.0, 0.8, 0.0, 0, False)
# PU200-like event: 6000 tracks, pT in [0.8, 50], |eta| < 2.4, z_v ~ N(0, 5 cm), 100k noise.
PU200 = EventConfig("pu200-6000trk-100knoise", 6000, 1 / 50.0, 1 / 0.8, 2.4, 5.0, 100_000, True)


def batch_event_config(rng: np.random.Generator) -> EventConfig:
    """Per-event occupancy of the 64-event batch: tracks U{1500..6000}, noise U{25k..100k}."""
    nt = int(rng.integers(1500, 6001))
    nn = int(rng.integers(25_000, 100_001))
    return EventConfig(f"batch-{nt}trk-{nn}noise", nt, 1 / 50.0, 1 / 0.8, 2.4, 5.0, nn, True)


def muon_cube_config(n_muons: int = 50, side: float = 5.0, n_noise: int = 0) -> EventConfig:
    """Displaced workload: n_muons muons, pT in [0.8, 50] GeV (1/pT uniform),
    |eta| < 2.4, vertices uniform in a cube of the given side (cm)."""
    return EventConfig(f"muon-cube-{n_muons}mu-{side:g}cm", n_muons, 1 / 50.0, 1 / 0.8, 2.4, 0.0, n_noise, True,
                       cube=side)


def pileup_event_config(pu: float) -> EventConfig:
    """Serving workload: 30 tracks and 500 noise hits per unit of pile-up."""
    return EventConfig(f"pu{pu:.0f}", int(round(30 * pu)), 1 / 50.0, 1 / 0.8, 2.4, 5.0,
                       int(round(500 * pu)), True)


@dataclass
class Event:
    x: np.ndarray        # f32
    y: np.ndarray
    z: np.ndarray
    sensor: np.ndarray   # i32
    truth: np.ndarray    # i32 track id, -1 noise
    # per-track truth (f64): q, pt, eta, phi0, zv (and x_v, y_v for displaced vertices)
    tracks: np.ndarray

    @property
    def n(self) -> int:
        return int(self.x.shape[0])


def helix_point(q, R, phi0, zv, lam, s):
    """Helix position at transverse arc length s (vectorised).

    Same curve as the parametrisation in the module docstring, written with
    the product-to-sum identities so that straight (R -> inf) tracks keep full
    precision: the point lies at distance 2R sin(s / 2R) from the vertex, at
    polar angle phi0 - q s / (2R)."""
    h = s / (2.0 * R)
    chord = 2.0 * R * np.sin(h)
    ang = phi0 - q * h
    return chord * np.cos(ang), chord * np.sin(ang), zv + s * lam


def _first_cylinder_crossing(q, R, phi0, xv, yv, rr):
    """Transverse arc length of the first crossing of radius rr by helices
    starting at (xv, yv) inside it, and whether there is one within half a
    turn: the first sign change of |V + P(s)|^2 - rr^2 on a grid of 512 steps
    in s / 2R over (0, pi / 2], refined by 60 bisections."""
    def f(h, q, R, phi0, xv, yv):
        ch = 2.0 * R * np.sin(h)
        ang = phi0 - q * h
        return (xv + ch * np.cos(ang)) ** 2 + (yv + ch * np.sin(ang)) ** 2 - rr * rr

    hs = np.linspace(0.0, 0.5 * math.pi, 513)[1:]
    col = lambda a: a[:, None]
    vals = f(hs[None, :], col(q), col(R), col(phi0), col(xv), col(yv))
    pos = vals >= 0.0
    ok = pos.any(axis=1)
    k = np.argmax(pos, axis=1)
    hi = hs[k]
    lo = np.where(k > 0, hs[np.maximum(k - 1, 0)], 0.0)
    for _ in range(60):
        mid = 0.5 * (lo + hi)
        up = f(mid, q, R, phi0, xv, yv) >= 0.0
        hi = np.where(up, mid, hi)
        lo = np.where(up, lo, mid)
    return np.where(ok, 2.0 * R * hi, 0.0), ok


def _track_hits(geo: Geometry, q, pt, eta, phi0, zv, sigma_scale, rng, xv=None, yv=None):
    """All sensor crossings of the given tracks -> (x, y, z, sensor, track_index).
    xv, yv: transverse vertex positions (None: on the beam line)."""
    displaced = xv is not None
    prm = geo.params
    kb = prm["k_b"]
    g = prm["gap"]
    R = pt / kb
    c = 1.0 / (2.0 * R)
    lam = np.sinh(eta)
    s_rphi = prm["sigma_rphi"] * sigma_scale
    s_z = prm["sigma_z"] * sigma_scale
    s_r = prm["sigma_r"] * sigma_scale
    out = []
    idx = np.arange(pt.shape[0])
    # barrel cylinders: anchor (r) and other (r + gap)
    for li, rk in enumerate(BARREL_RADII):
        for which, rr in ((0, rk), (1, rk + g)):
            if displaced:
                s, ok = _first_cylinder_crossing(q, R, phi0, xv, yv, rr)
                x, y, z = helix_point(q, R, phi0, zv, lam, s)
                x, y = x + xv, y + yv
            else:
                ok = c * rr < 1.0
                s = np.where(ok, np.arcsin(np.minimum(1.0, c * rr)) / c, 0.0)
                x, y, z = helix_point(q, R, phi0, zv, lam, s)
            phi = np.arctan2(y, x) + rng.normal(0.0, 1.0, pt.shape) * (s_rphi / rr)
            zz = z + rng.normal(0.0, 1.0, pt.shape) * s_z
            mod = geo.barrel_module(np.full(pt.shape, li), zz, phi)
            keep = ok & (mod >= 0)
            out.append((rr * np.cos(phi[keep]), rr * np.sin(phi[keep]), zz[keep],
                        2 * mod[keep] + which, idx[keep]))
    if geo.with_endcap:
        for si, sgn in enumerate((+1, -1)):
            for di, zd in enumerate(DISK_Z):
                for which, zz0 in ((0, zd), (1, zd + g)):
                    Zp = sgn * zz0
                    with np.errstate(divide="ignore", invalid="ignore"):
                        s = (Zp - zv) / lam
                    ok = np.isfinite(s) & (s > 0) & (c * s <= math.pi / 2)
                    s = np.where(ok, s, 0.0)
                    x, y, _ = helix_point(q, R, phi0, zv, lam, s)
                    if displaced:
                        x, y = x + xv, y + yv
                    r = np.hypot(x, y)
                    phi = np.arctan2(y, x)
                    rr = r + rng.normal(0.0, 1.0, pt.shape) * s_r
                    phi = phi + rng.normal(0.0, 1.0, pt.shape) * (s_rphi / np.maximum(rr, 1.0))
                    mod = geo.endcap_module(np.full(pt.shape, si), np.full(pt.shape, di), rr, phi)
                    keep = ok & (mod >= 0)
                    out.append((rr[keep] * np.cos(phi[keep]), rr[keep] * np.sin(phi[keep]),
                                np.full(int(keep.sum()), Zp), 2 * mod[keep] + which, idx[keep]))
    xs = np.concatenate([o[0] for o in out])
    ys = np.concatenate([o[1] for o in out])
    zs = np.concatenate([o[2] for o in out])
    sens = np.concatenate([o[3] for o in out])
    tid = np.concatenate([o[4] for o in out])
    return xs, ys, zs, sens, tid


def _sensor_surface_areas(geo: Geometry):
    p = geo.p
    dphi = p[:, 5] - p[:, 4]
    area = np.empty(geo.n_sensors)
    b = geo.kind == 0
    # barrel: cylinder patch at the sensor radius
    area[0::2][b] = p[b, 0] * dphi[b] * (p[b, 3] - p[b, 2])
    area[1::2][b] = p[b, 1] * dphi[b] * (p[b, 3] - p[b, 2])
    e = ~b
    ae = 0.5 * dphi[e] * (p[e, 3] ** 2 - p[e, 2] ** 2)
    area[0::2][e] = ae
    area[1::2][e] = ae
    return area


def _noise_hits(geo: Geometry, n: int, rng: np.random.Generator):
    area = _sensor_surface_areas(geo)
    sens = rng.choice(geo.n_sensors, size=n, p=area / area.sum())
    mod = sens // 2
    which = sens % 2
    p = geo.p[mod]
    phi = rng.uniform(p[:, 4], p[:, 5])
    barrel = geo.kind[mod] == 0
    x = np.empty(n); y = np.empty(n); z = np.empty(n)
    rb = np.where(which == 0, p[:, 0], p[:, 1])
    zb = rng.uniform(p[:, 2], p[:, 3])
    u = rng.random(n)
    re = np.sqrt(p[:, 2] ** 2 + u * (p[:, 3] ** 2 - p[:, 2] ** 2))
    ze = np.where(which == 0, p[:, 0], p[:, 1])
    r = np.where(barrel, rb, re)
    x = r * np.cos(phi)
    y = r * np.sin(phi)
    z = np.where(barrel, zb, ze)
    return x, y, z, sens


def make_tracks(cfg: EventConfig, rng: np.random.Generator, n: int | None = None):
    n = cfg.n_tracks if n is None else n
    q = np.where(rng.random(n) < 0.5, -1.0, 1.0)
    invpt = rng.uniform(cfg.invpt_lo, cfg.invpt_hi, n)
    eta = rng.uniform(-cfg.eta_max, cfg.eta_max, n)
    phi0 = rng.uniform(0.0, TWO_PI, n)
    if cfg.cube > 0:
        v = rng.uniform(-0.5 * cfg.cube, 0.5 * cfg.cube, (n, 3))
        return np.stack([q, 1.0 / invpt, eta, phi0, v[:, 2], v[:, 0], v[:, 1]], axis=1)
    zv = rng.normal(0.0, cfg.zv_sigma, n) if cfg.zv_sigma > 0 else np.zeros(n)
    return np.stack([q, 1.0 / invpt, eta, phi0, zv], axis=1)


def make_event_from_tracks(geo: Geometry, tracks: np.ndarray, n_noise: int, sigma_scale: float,
                           rng: np.random.Generator, shuffle: bool = True) -> Event:
    q, pt, eta, phi0, zv = (tracks[:, i] for i in range(5))
    xv, yv = (tracks[:, 5], tracks[:, 6]) if tracks.shape[1] > 5 else (None, None)
    xs, ys, zs, sens, tid = _track_hits(geo, q, pt, eta, phi0, zv, sigma_scale, rng, xv, yv)
    if n_noise > 0:
        nx, ny, nz, ns = _noise_hits(geo, n_noise, rng)
        xs = np.concatenate([xs, nx]); ys = np.concatenate([ys, ny]); zs = np.concatenate([zs, nz])
        sens = np.concatenate([sens, ns]); tid = np.concatenate([tid, np.full(n_noise, -1)])
    order = rng.permutation(xs.shape[0]) if shuffle else np.arange(xs.shape[0])
    return Event(xs[order].astype(np.float32), ys[order].astype(np.float32),
                 zs[order].astype(np.float32), sens[order].astype(np.int32),
                 tid[order].astype(np.int32), tracks)


def event_rng(*key: int) -> np.random.Generator:
    return np.random.Generator(np.random.PCG64(np.random.SeedSequence(list(key))))


def make_event(geo: Geometry, cfg: EventConfig, seed_key) -> Event:
    """One seeded event: seed_key is the SeedSequence entropy, e.g. (1, event_id)."""
    rng = event_rng(*seed_key)
    tracks = make_tracks(cfg, rng)
    return make_event_from_tracks(geo, tracks, cfg.n_noise, cfg.sigma_scale, rng)


def concat_events(events):
    """Concatenate events into batch arrays plus int64 event offsets."""
    off = np.zeros(len(events) + 1, np.int64)
    for i, e in enumerate(events):
        off[i + 1] = off[i] + e.n
    cat = lambda a: np.concatenate([getattr(e, a) for e in events]) if events else np.zeros(0)
    return (cat("x").astype(np.float32), cat("y").astype(np.float32), cat("z").astype(np.float32),
            cat("sensor").astype(np.int32), off)
