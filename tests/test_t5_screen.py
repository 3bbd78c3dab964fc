"""The FP32 chi2_rz screen of the quintuplet pre-cuts leaves every decision to
the FP64 fits.

The pre-cut kernel drops a T3 pair only when an FP32 evaluation of the r-z
chi2 exceeds twice the cut. This test models that evaluation in numpy
float32 (the same steps: weighted Taubin circle fit in the chord frame, arc
lengths at the fitted curvature, weighted line fit), models the FP64 fits the
same way in float64, pins the float64 model to the oracle's own circle and
line fits on a sample, and checks on every T3 pair of a PU200-like event that
the two precisions agree far inside the factor of two.
"""
import numpy as np
import pytest

from oracle import oracle as O
from paper_2403_13166_amd.synth import events as E, geometry as G, model as M


def _fits(x, y, z, endc, prm, dt):
    x = x.astype(dt); y = y.astype(dt); z = z.astype(dt)
    isg = np.where(endc, dt(1 / prm["sigma_r"]), dt(1 / prm["sigma_rphi"])).astype(dt)
    w = isg * isg
    w = w / w.sum(1, keepdims=True)
    xm = (w * x).sum(1, keepdims=True); ym = (w * y).sum(1, keepdims=True)
    cx = x[:, 4:5] - x[:, 0:1]; cy = y[:, 4:5] - y[:, 0:1]; cl = np.sqrt(cx * cx + cy * cy)
    ca = cx / cl; sa = cy / cl
    u0 = x - xm; v0 = y - ym
    u = ca * u0 + sa * v0; v = -sa * u0 + ca * v0
    Mxx = (w * u * u).sum(1); Myy = (w * v * v).sum(1); Mxy = (w * u * v).sum(1)
    Mz = Mxx + Myy
    zt = u * u + v * v - Mz[:, None]
    Mxz = (w * u * zt).sum(1); Myz = (w * v * zt).sum(1); varz = (w * zt * zt).sum(1)
    cov = Mxx * Myy - Mxy * Mxy
    c3 = 4 * Mz; c2 = -4 * Mz * Mz - varz
    c1 = varz * Mz + 4 * cov * Mz - Mxz * Mxz - Myz * Myz
    c0 = Mxz * (Mxz * Myy - Myz * Mxy) + Myz * (Myz * Mxx - Mxz * Mxy) - varz * cov
    eta = np.zeros_like(Mz); fprev = np.full_like(Mz, np.inf); act = np.ones(len(Mz), bool)
    tol = dt(1e-14 if dt == np.float64 else 1e-6)
    with np.errstate(all="ignore"):
        for _ in range(32 if dt == np.float64 else 16):
            f = c0 + eta * (c1 + eta * (c2 + eta * c3))
            act &= ~(np.abs(f) >= np.abs(fprev))
            fprev = np.where(act, f, fprev)
            nx = eta - f / (c1 + eta * (2 * c2 + eta * 3 * c3))
            neg = ~(nx >= 0)
            eta = np.where(act & neg, 0, eta); act &= ~neg
            conv = np.abs(nx - eta) <= tol * np.abs(nx)
            eta = np.where(act, nx, eta); act &= ~conv
    k1 = np.stack([varz - 4 * Mz * eta, Mxz, Myz], 1)
    k2 = np.stack([Mxz, Mxx - eta, Mxy], 1)
    k3 = np.stack([Myz, Mxy, Myy - eta], 1)
    best = np.zeros_like(k1); bn = np.full(len(Mz), -1.0, dt)
    for a, b in ((k2, k3), (k3, k1), (k1, k2)):
        vv = np.cross(a, b); nn = (vv * vv).sum(1)
        take = nn > bn
        best = np.where(take[:, None], vv, best); bn = np.where(take, nn, bn)
    A, B, C = best[:, 0], best[:, 1], best[:, 2]
    cf = np.abs(A) / np.sqrt(B * B + C * C + 4 * A * A * Mz)
    r = np.sqrt(x * x + y * y)
    xx = cf[:, None] * r
    with np.errstate(all="ignore"):
        s = np.where(xx < 1e-4, r * (1 + xx * xx / 6), np.arcsin(np.minimum(xx, 1)) / cf[:, None])
        kAE = np.abs((z[:, 4] - z[:, 0]) / (s[:, 4] - s[:, 0]))
        ike = dt(1 / prm["sigma_r"]) / np.maximum(kAE, dt(0.1))
        iv = np.where(endc, ike[:, None], dt(1 / prm["sigma_z"]))
        wz = iv * iv
        Wt = wz.sum(1); sm = (wz * s).sum(1) / Wt; zm = (wz * z).sum(1) / Wt
        Sss = (wz * (s - sm[:, None]) ** 2).sum(1); Ssz = (wz * (s - sm[:, None]) * (z - zm[:, None])).sum(1)
        t = Ssz / Sss; z0 = zm - t * sm
        d = z - z0[:, None] - t[:, None] * s
        chi2 = (d * d * wz).sum(1)
    bad = ~(s[:, 4] > s[:, 0]) | ~(Sss > 0)
    return np.where(bad, np.nan, chi2).astype(np.float64), cf.astype(np.float64), s.astype(np.float64)


@pytest.fixture(scope="module")
def pu200_pairs():
    geo = G.make_geometry(True)
    ev = E.make_event(geo, E.PU200, (1, 0))
    res = O.build_objects(O.Geom(geo.to_blob()), O.Model(M.make_model().to_blob()),
                          ev.x, ev.y, ev.z, ev.sensor, mode=0)
    t3m = res.t3_mds()
    order = np.argsort(t3m[:, 0], kind="stable")
    a_sorted = t3m[order, 0]
    lo = np.searchsorted(a_sorted, t3m[:, 2], "left"); hi = np.searchsorted(a_sorted, t3m[:, 2], "right")
    us = np.repeat(np.arange(len(t3m)), hi - lo)
    vs = order[np.concatenate([np.arange(a, b) for a, b in zip(lo, hi)])]
    ha = res.md[:, 0]
    ids = np.stack([t3m[us, 0], t3m[us, 1], t3m[us, 2], t3m[vs, 1], t3m[vs, 2]], 1)
    endc = (geo.kind[ev.sensor[ha] // 2] != 0)[ids]
    x = ev.x[ha][ids].astype(np.float64); y = ev.y[ha][ids].astype(np.float64); z = ev.z[ha][ids].astype(np.float64)
    return geo.params, x, y, z, endc, res


def test_float64_model_matches_oracle_fits(pu200_pairs):
    prm, x, y, z, endc, _ = pu200_pairs
    rng = np.random.default_rng(5)
    pick = rng.choice(len(x), 300, replace=False)
    c64, cf, s = _fits(x[pick], y[pick], z[pick], endc[pick], prm, np.float64)
    for j, i in enumerate(pick):
        sg = np.where(endc[i], prm["sigma_r"], prm["sigma_rphi"])
        circ = O.circle_fit(x[i], y[i], sg)
        assert abs(abs(circ[2]) - cf[j]) <= 1e-9 * max(cf[j], 1e-6)
        if not np.isfinite(c64[j]):
            continue
        kAE = abs((z[i][4] - z[i][0]) / (s[j][4] - s[j][0]))
        sz = np.where(endc[i], prm["sigma_r"] * max(kAE, 0.1), prm["sigma_z"])
        ref = O.line_fit(s[j], z[i], sz)[2]
        assert abs(ref - c64[j]) <= 1e-7 * max(ref, 1e-3)


def test_screen_never_decides(pu200_pairs):
    prm, x, y, z, endc, res = pu200_pairs
    thr = prm["chi2_rz_max"]
    c64, _, _ = _fits(x, y, z, endc, prm, np.float64)
    c32, _, _ = _fits(x, y, z, endc, prm, np.float32)
    # every T5 the oracle keeps passes the FP64 chi2 cut here too
    assert int(np.sum(c64 <= thr)) >= len(res.t5)
    # where either estimate is anywhere near the cut, they agree within 1 %
    near = (c64 <= 8 * thr) | (c32 <= 8 * thr)
    both = near & np.isfinite(c64) & np.isfinite(c32)
    assert both.sum() > 10_000
    assert np.max(np.abs(c32[both] / c64[both] - 1)) < 0.01
    # hence no candidate within the cut is dropped by the screen (2x the cut)
    assert not np.any((c64 <= thr) & (c32 > 2 * thr))
    # and the screen does remove most candidates
    assert np.mean(c32 > 2 * thr) > 0.5
