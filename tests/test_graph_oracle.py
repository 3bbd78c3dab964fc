"""Pins of the LST-graph oracle (oracle/graph.py) on the CPU.

* Node features on noise-free helices against closed forms of the helix: the
  MD bend alpha equals sgn asin(c m) (m = radius of the chord midpoint, sgn
  the sign of the track's bending) and the chord pseudorapidity equals
  asinh(cot(theta) / sqrt(1 - (c m)^2)), both to first order in the sensor
  gap; layer and endcap flag follow the module the generator placed the hit on.
* Edges: one per LS, from its outer to its inner MD.
* Components against hand-worked cases (tests/golden/graph_components_cases.json)
  and against a union-find written here on random graphs.
"""
import json
import math
import os

import numpy as np
import pytest

from oracle import graph as GR

GOLD = json.load(open(os.path.join(os.path.dirname(__file__), "golden", "graph_components_cases.json")))


def test_features_on_noise_free_helices(geo_full, model):
    from oracle import oracle as O
    from paper_2403_13166_amd.synth import events as E
    rng = E.event_rng(8, 1)
    tr = E.make_tracks(E.pileup_event_config(1.0), rng, 40)
    ev = E.make_event_from_tracks(geo_full, tr, 0, 0.0, rng)
    r = O.build_objects(O.Geom(geo_full.to_blob()), O.Model(model.to_blob()), ev.x, ev.y, ev.z, ev.sensor)
    X = GR.md_features(ev.x, ev.y, ev.z, ev.sensor, r.md, geo_full.kind, geo_full.layer)
    kb = geo_full.params["k_b"]
    assert len(X) > 100
    for i, (a, o) in enumerate(r.md.tolist()):
        q, pt, eta, phi0, zv = ev.tracks[ev.truth[a]]
        c = kb / (2 * pt)
        xa, ya, xo, yo = (float(v) for v in (ev.x[a], ev.y[a], ev.x[o], ev.y[o]))
        za, zo = float(ev.z[a]), float(ev.z[o])
        m = math.hypot(0.5 * (xa + xo), 0.5 * (ya + yo))
        chord = math.hypot(xo - xa, yo - ya)
        dr = math.hypot(xo, yo) - math.hypot(xa, ya)
        # FP32 rounding of the hit coordinates (half an ulp each, two hits)
        # bounds the deviation from the closed forms; the chord-versus-tangent
        # difference is far below it
        d = 2 * 2.0 ** -24 * max(abs(xa), abs(ya), abs(za), abs(xo), abs(yo), abs(zo))
        # sign of the bending: points move to smaller phi for q > 0 (A x O < 0)
        assert X[i, 3] / 10 == pytest.approx(-q * math.asin(c * m), abs=2 * d / chord + 1e-6)
        u = math.sinh(eta) / math.sqrt(1 - (c * m) ** 2)
        want = max(-5, min(5, math.asinh(u)))
        assert X[i, 4] == pytest.approx(want, abs=(d + abs(u) * d) / abs(dr) / math.sqrt(1 + u * u) + 1e-5)
        mod = int(ev.sensor[a]) // 2
        assert X[i, 5] == float(geo_full.kind[mod] != 0) and X[i, 6] * 11 == pytest.approx(geo_full.layer[mod])
        assert X[i, 0] * 100 == pytest.approx(math.hypot(xa, ya), rel=1e-12)


def test_edges_run_from_outer_to_inner_md():
    ls = np.array([[3, 7], [3, 9], [5, 7]])
    src, dst = GR.ls_edges(ls)
    assert src.tolist() == [7, 9, 7] and dst.tolist() == [3, 3, 5]


@pytest.mark.parametrize("case", GOLD["cases"], ids=lambda c: c["note"][:30])
def test_components_hand_cases(case):
    lab = GR.components(case["n_nodes"], case["src"], case["dst"], case["scores"], case["threshold"])
    assert lab.tolist() == case["labels"]


def _union_find(n, src, dst, keep):
    par = list(range(n))

    def find(v):
        while par[v] != v:
            v = par[v]
        return v
    for s, d, k in zip(src, dst, keep):
        if k:
            a, b = find(s), find(d)
            if a != b:
                par[max(a, b)] = min(a, b)
    return [find(v) for v in range(n)]


def test_components_against_union_find():
    rng = np.random.default_rng(4)
    for _ in range(50):
        n = int(rng.integers(1, 200))
        e = int(rng.integers(0, 400))
        src, dst = rng.integers(0, n, e), rng.integers(0, n, e)
        sc = rng.random(e)
        lab = GR.components(n, src, dst, sc, 0.4)
        assert lab.tolist() == _union_find(n, src.tolist(), dst.tolist(), (sc >= 0.4).tolist())


def test_track_candidates_by_size():
    tcs = GR.track_candidates([0, 0, 0, 3, 3, 5], 3)
    assert tcs == {0: [0, 1, 2]}
