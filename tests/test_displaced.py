"""Displaced-track workload (Sec. 3, the muon-cube sample: muons from points
uniform in a 5 cm cube) and the relaxed cut set for it, on the CPU.

Pins, none of which comes from the oracle itself:
* the generator: noise-free displaced hits lie on the circle through their
  vertex with radius pT / k_b, on their sensor surfaces, and the crossing
  solver reduces to the beam-line closed form asin(c r) / c at V = 0;
* closed forms of the cuts for a straight track with impact parameter d0:
  the beam-line circle through two points at radii r_A < r_B has
  half-curvature d0 / (r_A r_B) (twice the triangle's area over the product
  of its sides), and the opening angle of an MD at radii r < r' is
  asin(d0 / r) - asin(d0 / r');
* the reading of the relaxed constraints: on seeded muon-cube events the
  relaxed set keeps displaced muons (r_v >= 2.5 cm) that the default set
  loses, and finds every muon the default set finds;
* the line-segment windows hold for every oracle segment under the relaxed
  set (curvatures up to c r = 0.96, where most runs are not trimmed in phi).
"""
import math

import numpy as np
import pytest

from oracle import oracle as O
from paper_2403_13166_amd import train as TR
from paper_2403_13166_amd.synth import events as E, geometry as G, model as M
from tests import helix as H


@pytest.fixture(scope="module")
def geo_d():
    return G.make_geometry(True, G.DISPLACED_PARAMS)


@pytest.fixture(scope="module")
def og_d(geo_d):
    return O.Geom(geo_d.to_blob())


@pytest.fixture(scope="module")
def om():
    return O.Model(M.make_model().to_blob())


def _circle(tr, kb):
    """Centre and radius of the transverse circle of tracks [q, pt, eta, phi0, zv, xv, yv]."""
    q, pt, phi0, xv, yv = tr[:, 0], tr[:, 1], tr[:, 3], tr[:, 5], tr[:, 6]
    R = pt / kb
    return xv + q * R * np.sin(phi0), yv - q * R * np.cos(phi0), R


def test_cube_vertices_and_hits_on_their_circles(geo_d):
    cfg = E.EventConfig("cube-noise-free", 300, 1 / 50.0, 1 / 0.8, 2.4, 0.0, 0, True, sigma_scale=0.0, cube=5.0)
    ev = E.make_event(geo_d, cfg, (9, 1))
    tr = ev.tracks
    assert tr.shape == (300, 7)
    assert np.all(np.abs(tr[:, 4:7]) <= 2.5)
    # the cube is filled: each coordinate spans most of [-2.5, 2.5]
    assert np.all(tr[:, 4:7].max(axis=0) > 2.3) and np.all(tr[:, 4:7].min(axis=0) < -2.3)
    cx, cy, R = _circle(tr[ev.truth], geo_d.params["k_b"])
    d = np.hypot(ev.x.astype(np.float64) - cx, ev.y.astype(np.float64) - cy) - R
    assert np.max(np.abs(d)) < 2e-5 * np.maximum(1.0, R / 1000).max()
    # barrel hits on their sensor radius, endcap hits on their disk
    mod = ev.sensor // 2
    which = ev.sensor % 2
    b = geo_d.kind[mod] == 0
    r = np.hypot(ev.x, ev.y).astype(np.float64)
    assert np.max(np.abs(r[b] - geo_d.p[mod[b], which[b]])) < 2e-5
    assert np.max(np.abs(ev.z[~b] - geo_d.p[mod[~b], which[~b]])) < 2e-5
    # z grows linearly with the arc length from the vertex: z = z_v + s sinh(eta)
    t = ev.truth
    ang = np.arctan2(ev.y - cy, ev.x - cx) - np.arctan2(tr[t, 6] - cy, tr[t, 5] - cx)
    s = R * np.abs((ang + math.pi) % (2 * math.pi) - math.pi)
    assert np.max(np.abs(tr[t, 4] + s * np.sinh(tr[t, 2]) - ev.z)) < 1e-4


def test_crossing_solver_reduces_to_the_beam_line_closed_form():
    rng = np.random.default_rng(2)
    n = 400
    q = rng.choice([-1.0, 1.0], n)
    pt = rng.uniform(0.8, 50, n)
    R = pt / (0.3 * 3.8 / 100)
    phi0 = rng.uniform(0, 2 * math.pi, n)
    z = np.zeros(n)
    for rr in (23.0, 51.0, 108.26):
        s, ok = E._first_cylinder_crossing(q, R, phi0, z, z, rr)
        c = 1 / (2 * R)
        exp_ok = c * rr < 1
        assert np.array_equal(ok, exp_ok)
        assert np.allclose(s[ok], np.arcsin(c[ok] * rr) / c[ok], rtol=1e-12, atol=1e-9)


def _straight_displaced(geo, d0_sign, d0, phi_n, eta=0.1):
    """Noise-free hits of a straight (pT = 1e7 GeV) track whose closest point
    to the beam line is d0 from it at polar angle phi_n, grouped into MD pairs."""
    pt = 1e7
    # vertex at the closest approach point, direction perpendicular to it
    xv, yv = d0 * math.cos(phi_n), d0 * math.sin(phi_n)
    phi0 = phi_n + d0_sign * 0.5 * math.pi
    tr = np.array([[1.0, pt, eta, phi0, 0.0, xv, yv]])
    xs, ys, zs, sens, _ = E._track_hits(geo, tr[:, 0], tr[:, 1], tr[:, 2], tr[:, 3], tr[:, 4], 0.0,
                                        np.random.default_rng(0), tr[:, 5], tr[:, 6])
    hits = [(xs[i], ys[i], zs[i], int(sens[i])) for i in np.argsort(np.hypot(xs, ys))]
    return H.md_pairs(geo, hits)


def test_cut_values_of_a_displaced_straight_track(geo_d, og_d, om):
    rng = np.random.default_rng(7)
    n_md = n_ls = 0
    for _ in range(60):
        d0 = rng.uniform(0.2, 3.5)
        pairs = _straight_displaced(geo_d, rng.choice([-1, 1]), d0, rng.uniform(0, 2 * math.pi))
        pairs = [p for p in pairs if geo_d.kind[p[1][3] // 2] == 0]
        for lay, a, o in pairs:
            r_lo, r_up = geo_d.p[a[3] // 2, 0], geo_d.p[a[3] // 2, 1]
            cv = O.cut_values_exact(og_d, om, [a[0], o[0]], [a[1], o[1]], [a[2], o[2]], [a[3], o[3]], 1)
            # (the track's own half-curvature, 5.7e-10 / cm at 1e7 GeV, adds at most c * gap)
            assert cv.v[0] == pytest.approx(math.asin(d0 / r_lo) - math.asin(d0 / r_up), rel=1e-7, abs=1e-9)
            n_md += 1
        for (la, a, a2), (lb, b, b2) in zip(pairs, pairs[1:]):
            ra, rb = math.hypot(a[0], a[1]), math.hypot(b[0], b[1])
            hs = [a, a2, b, b2]
            cv = O.cut_values_exact(og_d, om, [h[0] for h in hs], [h[1] for h in hs], [h[2] for h in hs],
                                    [h[3] for h in hs], 2)
            assert cv.v[1] == pytest.approx(d0 / (ra * rb), rel=1e-7, abs=2e-9)
            n_ls += 1
    assert n_md > 200 and n_ls > 150


def _efficiency(geo, og, om, keys, bins):
    """Fraction of muons with at least 10 hits that have a real T5 (more than
    75 % of its hits from the muon), per bin of transverse vertex radius; and
    the found flags of every muon."""
    tot = np.zeros(len(bins) - 1)
    fnd = np.zeros(len(bins) - 1)
    flags = []
    for key in keys:
        ev = E.make_event(geo, E.muon_cube_config(200), key)
        r = O.build_objects(og, om, ev.x, ev.y, ev.z, ev.sensor)
        real, tid = TR.t5_truth(r.md, r.t5_mds(), ev.truth)
        found = np.zeros(len(ev.tracks), bool)
        found[np.unique(tid[real])] = True
        flags.append(found)
        nh = np.bincount(ev.truth[ev.truth >= 0], minlength=len(ev.tracks))
        b = np.digitize(np.hypot(ev.tracks[:, 5], ev.tracks[:, 6]), bins) - 1
        for k in range(len(bins) - 1):
            m = (nh >= 10) & (b == k)
            tot[k] += m.sum()
            fnd[k] += (found & m).sum()
    return fnd / tot, tot, np.concatenate(flags)


def test_relaxed_cuts_keep_displaced_muons(geo_d, og_d, om):
    geo0 = G.make_geometry(True)
    og0 = O.Geom(geo0.to_blob())
    bins = np.array([0.0, 1.5, 2.5, 3.6])
    keys = [(9, 100 + e) for e in range(20)]
    e0, n0, f0 = _efficiency(geo0, og0, om, keys, bins)
    ed, nd, fd = _efficiency(geo_d, og_d, om, keys, bins)
    assert np.array_equal(n0, nd) and n0.min() > 500
    assert ed[2] >= e0[2] + 0.03             # displaced muons recovered
    assert e0[0] - e0[2] >= 0.03             # the default cuts lose them
    # looser thresholds: every muon the default set finds is still found
    # (not exact in general: the MD direction check of a segment uses its
    # curvature clamped at c_max, which moves with the threshold)
    assert not np.any(f0 & ~fd)
    assert np.all(ed >= e0)


def test_windows_hold_under_the_relaxed_cuts(geo_d, og_d, om):
    from tests.test_ls_windows import Windows, _check_event
    win = Windows(geo_d)
    evs = [E.make_event(geo_d, E.muon_cube_config(200), (9, 200 + e)) for e in range(4)]
    evs.append(E.make_event(geo_d, E.PU200, (1, 0)))
    n = 0
    for ev in evs:
        orc = O.build_objects(og_d, om, ev.x, ev.y, ev.z, ev.sensor)
        _check_event(win, geo_d, ev, orc)
        n += len(orc.ls)
    assert n > 50_000
