"""Synthetic doublet-module tracker geometry and its module map.

This module is input generation: it describes a detector (where the sensors
are, which module pairs count as "adjacent"), the way a real tracker ships a
geometry file and a module-map file. It holds none of the object-building
arithmetic; the oracle and the GPU library each parse the blob it writes with
their own code.

Paper anchor (Sec. 1): outer-tracker "pT-modules" are two silicon sensors a few
millimetres apart; mini-doublets pair a hit on each sensor of one module; line
segments join mini-doublets on adjacent modules that pass geometric criteria.
The paper gives no detector numbers, so every dimension below is a reading:

* barrel: 6 cylinders at r = 23, 36, 51, 68, 86, 108 cm, half-length 120 cm;
  each layer is a doublet, anchor (inner) sensor at r, other sensor at r + 0.26;
  modules are cylinder patches ~5 cm in r-phi by 10 cm in z.
* endcap: 5 disks per side at |z| = 131, 155, 185, 220, 265 cm, anchor sensor
  at |z|, other at |z| + 0.26; annulus r in [23, 110] cut in 9 rings of 10 cm
  (the last 7 cm), each ring split into ceil(2 pi r_in / 5) phi sectors.

Blob v1 (little endian)::

    0   char[4]  magic "LSTG"
    4   u32      version (1)
    8   u32      n_modules
    12  u32      n_barrel_modules
    16  u32      n_map (number of module-map entries)
    20  u32      n_params (16)
    24  f64[16]  cut/physics parameters, order of PARAM_NAMES
    152 module records, 64 B each:
            i32 kind (0 barrel, 1 endcap), i32 layer (1..6 barrel, 7..11 disks),
            i32 side (0 barrel, +1 / -1 endcap), i32 nphi,
            f64 p[6]: barrel (r_anchor, r_other, z_min, z_max, phi_min, phi_max)
                      endcap (z_anchor, z_other, r_min, r_max, phi_min, phi_max)
    ... u32 map_offsets[n_modules + 1], u32 map_targets[n_map]

Sensor id = 2 * module + (0 anchor sensor, 1 other sensor).
"""
from __future__ import annotations

import math
import struct
from dataclasses import dataclass, field

import numpy as np

BARREL_RADII = (23.0, 36.0, 51.0, 68.0, 86.0, 108.0)
BARREL_HALF_LENGTH = 120.0
BARREL_Z_TILE = 10.0
DISK_Z = (131.0, 155.0, 185.0, 220.0, 265.0)
RING_EDGES = (23.0, 33.0, 43.0, 53.0, 63.0, 73.0, 83.0, 93.0, 103.0, 110.0)
SENSOR_GAP = 0.26
MODULE_RPHI = 5.0

# Physics and selection parameters stored in the blob (all readings except
# pt_min = 0.8 GeV, which is the mini-doublet requirement of Sec. 1).
PARAM_NAMES = (
    "k_b",          # GeV per cm of radius: pT = k_b * R; 0.3 * 3.8 T / 100
    "pt_min",       # GeV
    "z_lum",        # cm, luminous-region half length allowed for z0
    "n_sigma",      # resolution multiplier in every tolerance
    "sigma_rphi",   # cm
    "sigma_z",      # cm (barrel z resolution)
    "sigma_r",      # cm (endcap r resolution)
    "gap",          # cm, sensor separation inside a module
    "chi2_rz_max",  # quintuplet r-z line-fit cut
    "chi2_rphi_max",  # quintuplet r-phi circle-fit cut (pre-DNN mode only)
    "md_e2_slack",  # cm, second-order allowance in the endcap radial window
    "ls3_slack",    # rad, floor of the mini-doublet direction tolerance
    "reserved0", "reserved1", "reserved2", "reserved3",
)
DEFAULT_PARAMS = {
    "k_b": 0.3 * 3.8 / 100.0,
    "pt_min": 0.8,
    "z_lum": 15.0,
    "n_sigma": 5.0,
    "sigma_rphi": 0.003,
    "sigma_z": 0.05,
    "sigma_r": 0.05,
    "gap": SENSOR_GAP,
    "chi2_rz_max": 30.0,
    "chi2_rphi_max": 25.0,
    "md_e2_slack": 1e-3,
    "ls3_slack": 1e-4,
    "reserved0": 0.0, "reserved1": 0.0, "reserved2": 0.0, "reserved3": 0.0,
}

# Relaxed beam constraints for the displaced workload (vertices in a 5 cm
# cube, so transverse displacements d0 up to 2.5 sqrt 2 = 3.5 cm). Every cut
# that ties a pair of points to the beam line does so through a circle through
# the origin, whose half-curvature for a straight track of impact parameter d0
# through points at radii r_A < r_B is d0 / (r_A r_B). The pT threshold sets
# c_max = k_b / (2 pT_min); the lowest threshold at which every circle with
# c <= c_max still reaches the outermost sensors (c_max r < 1 at r = 110 cm)
# is 0.63 GeV. At 0.65 GeV (c_max = 0.0088 / cm) a track of pT p passes the
# innermost barrel pair (23, 36 cm) up to d0 = (c_max - k_b / 2p) * 23 * 36:
# 1.4 cm at 0.8 GeV, 4.9 cm at 2 GeV, more at larger radii. The z0
# extrapolation of a track starting at r_v <= 3.5 cm misses its vertex z by
# up to |cot theta| r_v (5.5 * 3.5 = 19 cm at |eta| = 2.4) on top of
# |z_v| <= 2.5 cm: z_lum 25 cm. The module map, the windows and the fits all
# follow from these parameters.
DISPLACED_PARAMS = {"pt_min": 0.65, "z_lum": 25.0}

# Map-building tolerances: beyond the selection envelope, windows are widened
# by 5 sigma of the hit resolution plus this many cm.
MAP_EXTRA_CM = 0.5

TWO_PI = 2.0 * math.pi


def barrel_nphi(r: float) -> int:
    return int(math.ceil(TWO_PI * r / MODULE_RPHI))


@dataclass
class Geometry:
    """Module table plus map; arrays are indexed by module id."""
    with_endcap: bool
    params: dict
    kind: np.ndarray      # i32
    layer: np.ndarray     # i32 (1..11)
    side: np.ndarray      # i32
    nphi: np.ndarray      # i32
    p: np.ndarray         # f64 [n, 6]
    map_off: np.ndarray = field(default=None)   # u32 [n+1]
    map_tgt: np.ndarray = field(default=None)   # u32 [n_map]
    # lookup helpers (input side only)
    barrel_layer_off: tuple = ()
    ring_off: tuple = ()

    @property
    def n_modules(self) -> int:
        return int(self.kind.shape[0])

    @property
    def n_barrel(self) -> int:
        return int(np.count_nonzero(self.kind == 0))

    @property
    def n_sensors(self) -> int:
        return 2 * self.n_modules

    def c_max(self) -> float:
        return self.params["k_b"] / (2.0 * self.params["pt_min"])

    # ---- position -> module (input side: used to assign generated hits) ----
    def barrel_module(self, layer_idx: np.ndarray, z: np.ndarray, phi: np.ndarray) -> np.ndarray:
        """Module id of barrel points (layer_idx 0..5); -1 outside |z| <= half length."""
        out = np.full(z.shape, -1, dtype=np.int64)
        nph = np.array([barrel_nphi(r) for r in BARREL_RADII])[layer_idx]
        nz = int(round(2 * BARREL_HALF_LENGTH / BARREL_Z_TILE))
        iz = np.floor((z + BARREL_HALF_LENGTH) / BARREL_Z_TILE).astype(np.int64)
        ph = np.mod(phi, TWO_PI)
        ip = np.minimum(np.floor(ph / (TWO_PI / nph)).astype(np.int64), nph - 1)
        ok = (z >= -BARREL_HALF_LENGTH) & (z < BARREL_HALF_LENGTH) & (iz >= 0) & (iz < nz)
        off = np.array(self.barrel_layer_off)[layer_idx]
        out[ok] = (off + iz * nph + ip)[ok]
        return out

    def endcap_module(self, side_idx: np.ndarray, disk_idx: np.ndarray, r: np.ndarray,
                      phi: np.ndarray) -> np.ndarray:
        """Module id of endcap points (side_idx 0 for +z, 1 for -z); -1 off the annulus."""
        out = np.full(r.shape, -1, dtype=np.int64)
        if not self.with_endcap:
            return out
        edges = np.array(RING_EDGES)
        ring = np.searchsorted(edges, r, side="right") - 1
        ok = (r >= edges[0]) & (r < edges[-1])
        ring = np.clip(ring, 0, len(edges) - 2)
        nph = np.array([barrel_nphi(e) for e in RING_EDGES[:-1]])[ring]
        ph = np.mod(phi, TWO_PI)
        ip = np.minimum(np.floor(ph / (TWO_PI / nph)).astype(np.int64), nph - 1)
        per_disk = self.ring_off[-1]
        base = self.n_barrel + (side_idx * len(DISK_Z) + disk_idx) * per_disk
        out[ok] = (base + np.array(self.ring_off[:-1])[ring] + ip)[ok]
        return out

    # ---- serialisation ----
    def to_blob(self) -> bytes:
        n = self.n_modules
        head = struct.pack("<4sIIIII", b"LSTG", 1, n, self.n_barrel, int(self.map_tgt.shape[0]),
                           len(PARAM_NAMES))
        par = struct.pack("<16d", *[float(self.params[k]) for k in PARAM_NAMES])
        rec = np.zeros(n, dtype=np.dtype([("kind", "<i4"), ("layer", "<i4"), ("side", "<i4"),
                                          ("nphi", "<i4"), ("p", "<f8", (6,))]))
        rec["kind"], rec["layer"], rec["side"], rec["nphi"], rec["p"] = (
            self.kind, self.layer, self.side, self.nphi, self.p)
        return b"".join([head, par, rec.tobytes(),
                         self.map_off.astype("<u4").tobytes(),
                         self.map_tgt.astype("<u4").tobytes()])


def build_modules(with_endcap: bool = True, params: dict | None = None) -> Geometry:
    """Tile the barrel (and optionally the endcaps) into modules, no map yet."""
    prm = dict(DEFAULT_PARAMS)
    if params:
        prm.update(params)
    g = prm["gap"]
    kind, layer, side, nphi, p = [], [], [], [], []
    nz = int(round(2 * BARREL_HALF_LENGTH / BARREL_Z_TILE))
    layer_off = []
    count = 0
    for li, r in enumerate(BARREL_RADII):
        layer_off.append(count)
        nph = barrel_nphi(r)
        dphi = TWO_PI / nph
        for iz in range(nz):
            z0 = -BARREL_HALF_LENGTH + iz * BARREL_Z_TILE
            for ip in range(nph):
                kind.append(0); layer.append(li + 1); side.append(0); nphi.append(nph)
                p.append((r, r + g, z0, z0 + BARREL_Z_TILE, ip * dphi, (ip + 1) * dphi))
        count += nz * nph
    ring_off = [0]
    for e in RING_EDGES[:-1]:
        ring_off.append(ring_off[-1] + barrel_nphi(e))
    if with_endcap:
        for si, sgn in enumerate((+1, -1)):
            for di, zd in enumerate(DISK_Z):
                for ri in range(len(RING_EDGES) - 1):
                    nph = barrel_nphi(RING_EDGES[ri])
                    dphi = TWO_PI / nph
                    for ip in range(nph):
                        kind.append(1); layer.append(7 + di); side.append(sgn); nphi.append(nph)
                        p.append((sgn * zd, sgn * (zd + g), RING_EDGES[ri], RING_EDGES[ri + 1],
                                  ip * dphi, (ip + 1) * dphi))
    geo = Geometry(with_endcap=with_endcap, params=prm,
                   kind=np.array(kind, np.int32), layer=np.array(layer, np.int32),
                   side=np.array(side, np.int32), nphi=np.array(nphi, np.int32),
                   p=np.array(p, np.float64),
                   barrel_layer_off=tuple(layer_off), ring_off=tuple(ring_off))
    return geo


# ---------------------------------------------------------------------------
# Module map: conservative reachability between anchor sensors of adjacent
# logical layers for tracks from the beam line (|z_v| <= z_lum, |c| <= c_max).
# ---------------------------------------------------------------------------

def _arc(c: float, r):
    """Transverse arc length from the origin to radius r on a circle of half-curvature c."""
    r = np.asarray(r, dtype=np.float64)
    if c == 0.0:
        return r
    return np.arcsin(np.minimum(1.0, c * r)) / c


def _phi_sectors(lo: float, hi: float, n: int) -> list:
    w = TWO_PI / n
    i0 = int(math.floor(lo / w))
    i1 = int(math.floor(hi / w))
    if i1 - i0 + 1 >= n:
        return list(range(n))
    return sorted({i % n for i in range(i0, i1 + 1)})


def build_map(geo: Geometry) -> Geometry:
    """Fill geo.map_off / geo.map_tgt (sorted targets per source module)."""
    prm = geo.params
    cmax = geo.c_max()
    Z = prm["z_lum"]
    ns = prm["n_sigma"]
    s_rphi, s_z, s_r = prm["sigma_rphi"], prm["sigma_z"], prm["sigma_r"]
    wid = MAP_EXTRA_CM
    nz = int(round(2 * BARREL_HALF_LENGTH / BARREL_Z_TILE))
    nb = len(BARREL_RADII)
    per_disk = geo.ring_off[-1]

    def barrel_id(li, iz, ip):
        return geo.barrel_layer_off[li] + iz * barrel_nphi(BARREL_RADII[li]) + ip

    def endcap_id(si, di, ri, ip):
        return geo.n_barrel + (si * len(DISK_Z) + di) * per_disk + geo.ring_off[ri] + ip

    targets = [[] for _ in range(geo.n_modules)]
    for m in range(geo.n_modules):
        k, lay, sd = int(geo.kind[m]), int(geo.layer[m]), int(geo.side[m])
        pp = geo.p[m]
        phi0, phi1 = pp[4], pp[5]
        if k == 0:
            ra = pp[0]
            za0, za1 = pp[2] - ns * s_z - 0.25, pp[3] + ns * s_z + 0.25
            li = lay - 1
            # barrel -> next barrel layer
            if li + 1 < nb:
                rb = BARREL_RADII[li + 1]
                rho0 = rb / ra
                rho1 = float(_arc(cmax, rb) / _arc(cmax, ra))
                cand = [zv * (1 - rho) + za * rho for zv in (-Z, Z) for za in (za0, za1)
                        for rho in (rho0, rho1)]
                zlo, zhi = min(cand) - wid - ns * s_z, max(cand) + wid + ns * s_z
                dphi = math.asin(cmax * rb) - math.asin(cmax * ra)
                wphi = dphi + (wid + ns * s_rphi) / rb + ns * s_rphi / ra
                izs = [iz for iz in range(nz)
                       if -BARREL_HALF_LENGTH + (iz + 1) * BARREL_Z_TILE > zlo
                       and -BARREL_HALF_LENGTH + iz * BARREL_Z_TILE < zhi]
                ips = _phi_sectors(phi0 - wphi, phi1 + wphi, barrel_nphi(rb))
                targets[m].extend(barrel_id(li + 1, iz, ip) for iz in izs for ip in ips)
            # barrel -> first disk, either side
            if geo.with_endcap:
                theta = math.asin(cmax * ra)
                for si, sgn in enumerate((+1, -1)):
                    zd = DISK_Z[0]
                    # signed coordinate along the side: u = sgn * z
                    ua1 = max(sgn * za0, sgn * za1)
                    if ua1 + Z <= 0:
                        continue
                    kmin = (zd + Z) / (ua1 + Z)
                    if kmin * theta >= math.pi / 2:
                        continue
                    rb_lo = ra * math.sin(kmin * theta) / math.sin(theta) - wid - ns * s_r
                    ua0 = min(sgn * za0, sgn * za1)
                    if ua0 - Z > 0:
                        kmax = (zd - Z) / (ua0 - Z)
                        rb_hi = ra * kmax + wid + ns * s_r
                    else:
                        rb_hi = RING_EDGES[-1]
                    if li + 1 < nb:
                        # a track that reaches the disk without crossing the next
                        # barrel layer leaves the barrel (|z| >= half length)
                        # before radius r_{k+1}
                        kex = (zd - Z) / (BARREL_HALF_LENGTH - ns * s_z - 0.25 - Z)
                        rb_hi = min(rb_hi, kex * float(_arc(cmax, BARREL_RADII[li + 1]))
                                    + wid + ns * s_r)
                    for ri in range(len(RING_EDGES) - 1):
                        r0, r1 = RING_EDGES[ri], RING_EDGES[ri + 1]
                        if r1 <= rb_lo or r0 > rb_hi:
                            continue
                        dphi = math.asin(min(1.0, cmax * min(r1, rb_hi))) - math.asin(cmax * ra)
                        wphi = dphi + (wid + ns * s_rphi) / r0 + ns * s_rphi / ra
                        for ip in _phi_sectors(phi0 - wphi, phi1 + wphi, barrel_nphi(r0)):
                            targets[m].append(endcap_id(si, 0, ri, ip))
        else:
            di = lay - 7
            if di + 1 >= len(DISK_Z):
                continue
            si = 0 if sd > 0 else 1
            zda, zdb = DISK_Z[di], DISK_Z[di + 1]
            ra0, ra1 = pp[2] - ns * s_r - 0.25, pp[3] + ns * s_r + 0.25
            kmin = (zdb - Z) / (zda - Z)
            kmax = (zdb + Z) / (zda + Z)
            kmin, kmax = min(kmin, kmax), max(kmin, kmax)
            th0 = math.asin(cmax * ra0)
            if kmin * th0 >= math.pi / 2:
                rb_lo = 0.0
            else:
                rb_lo = ra0 * math.sin(kmin * th0) / math.sin(th0)
            rb_lo -= wid + ns * s_r
            rb_hi = ra1 * kmax + wid + ns * s_r
            for ri in range(len(RING_EDGES) - 1):
                r0, r1 = RING_EDGES[ri], RING_EDGES[ri + 1]
                if r1 <= rb_lo or r0 > rb_hi:
                    continue
                rtop = min(r1, rb_hi)
                dphi = math.asin(min(1.0, cmax * rtop)) - math.asin(min(1.0, cmax * max(ra0, 1e-9)))
                dphi = max(dphi, 0.0)
                wphi = dphi + (wid + ns * s_rphi) / r0 + ns * s_rphi / max(ra0, 1.0)
                for ip in _phi_sectors(phi0 - wphi, phi1 + wphi, barrel_nphi(r0)):
                    targets[m].append(endcap_id(si, di + 1, ri, ip))
    off = np.zeros(geo.n_modules + 1, np.uint32)
    flat = []
    for m, t in enumerate(targets):
        t = sorted(set(t))
        flat.extend(t)
        off[m + 1] = off[m] + len(t)
    geo.map_off = off
    geo.map_tgt = np.array(flat, np.uint32)
    return geo


_CACHE: dict = {}


def make_geometry(with_endcap: bool = True, params: dict | None = None) -> Geometry:
    """Geometry plus module map; cached per (with_endcap, params)."""
    key = (with_endcap, tuple(sorted((params or {}).items())))
    if key not in _CACHE:
        _CACHE[key] = build_map(build_modules(with_endcap, params))
    return _CACHE[key]
