"""The GPU-vs-oracle classifier (tests/compare.py) on real disagreements.

A result is made from the oracle's own objects and then perturbed, so that
every count the classifier reports is known in advance:
  * an object dropped whose deciding cut lies within the relative 1e-5 band
    of its threshold -> marginal; one dropped far from every threshold ->
    violation; every object built on a dropped one -> inherited;
  * a candidate the oracle rejects added, with every failing cut inside the
    band -> marginal; with a failing cut far outside it -> violation.
Near-threshold objects come from the analytic threshold case: with the
resolution terms off (n_sigma = 0), a noise-free track at pT = pT_min sits
exactly on the curvature thresholds (mini-doublet bend, line-segment
curvature), and only the FP32 rounding of its hit positions decides whether
the oracle keeps it. Such objects must be reported marginal, never violation.
"""
import math
from dataclasses import dataclass

import numpy as np
import pytest

from oracle import oracle as O
from paper_2403_13166_amd.synth import geometry as G, events as E
from tests import compare as CMP
from tests.helix import threshold_event


@dataclass
class KeyObjects:
    """Objects in the layout compare() reads: MD hit pairs, LS as MD index
    pairs, T3 / T5 as MD index tuples."""
    md_hits: np.ndarray
    ls_md: np.ndarray
    t3: np.ndarray
    t5: np.ndarray

    def t3_mds(self):
        return self.t3

    def t5_mds(self):
        return self.t5


def _rel(cv):
    with np.errstate(invalid="ignore", divide="ignore"):
        return np.abs(cv.v - cv.t) / np.abs(cv.t)


def _pick(cands, cvs, kept, want):
    """First candidate (in order) whose oracle cut values meet `want`."""
    for c, cv in zip(cands, cvs):
        if want(cv, c in kept):
            return c
    raise AssertionError("no candidate of the requested kind")


in_band_kept = lambda cv, kept: kept and bool(np.any(_rel(cv) <= CMP.MARGIN))
far_kept = lambda cv, kept: kept and bool(np.all(_rel(cv) > 1e-2))
in_band_rejected = lambda cv, kept: (not kept) and bool(np.all(_rel(cv)[~cv.passes()] <= CMP.MARGIN))
far_rejected = lambda cv, kept: (not kept) and bool(np.any(_rel(cv)[~cv.passes()] > 1e-2))


@pytest.mark.parametrize("seed", [0, 1])
def test_classifier_counts_marginal_violation_inherited(seed):
    geo = G.make_geometry(True, {"n_sigma": 0.0})
    og = O.Geom(geo.to_blob())
    ev = threshold_event(geo, seed)
    orc = O.build_objects(og, None, ev.x, ev.y, ev.z, ev.sensor)
    md = [tuple(r) for r in orc.md.tolist()]
    md_set = set(md)
    ls = [(md[a], md[b]) for a, b in orc.ls.tolist()]
    t3 = [tuple(md[k] for k in row) for row in orc.t3_mds().tolist()]
    t5 = [tuple(md[k] for k in row) for row in orc.t5_mds().tolist()]
    print("oracle counts", len(md), len(ls), len(t3), len(t5))
    assert len(md) > 800 and len(ls) > 200 and len(t3) > 50 and len(t5) > 5

    # mini-doublet candidates: every (anchor hit, other hit) of one module
    by_sensor = {}
    for i, sid in enumerate(ev.sensor.tolist()):
        by_sensor.setdefault(sid, []).append(i)
    md_cands = [(i, j) for sid, hs in sorted(by_sensor.items()) if sid % 2 == 0
                for i in hs for j in by_sensor.get(sid + 1, [])]
    md_cv = [O.cut_values(og, None, ev.x, ev.y, ev.z, ev.sensor, 1, list(c)) for c in md_cands]
    # the dropped MDs carry line segments, so their dependents are inherited
    has_ls = {k for pair in ls for k in pair}
    with_ls = [(c, cv) for c, cv in zip(md_cands, md_cv) if c in has_ls]
    drop_md_marg = _pick([c for c, _ in with_ls], [cv for _, cv in with_ls], md_set, in_band_kept)
    drop_md_far = _pick([c for c, _ in with_ls], [cv for _, cv in with_ls], md_set, far_kept)
    add_md_marg = _pick(md_cands, md_cv, md_set, in_band_rejected)
    add_md_far = _pick(md_cands, md_cv, md_set, far_rejected)

    # line-segment candidates on the kept MDs not touched above
    gone_md = {drop_md_marg, drop_md_far}
    ls_set = set(ls)
    off = geo.map_off.astype(np.int64)
    by_mod = {}
    for k in md:
        by_mod.setdefault(int(ev.sensor[k[0]]) // 2, []).append(k)
    ls_cands = []
    for a in md:
        if a in gone_md:
            continue
        ma = int(ev.sensor[a[0]]) // 2
        for mb in geo.map_tgt[off[ma]:off[ma + 1]].tolist():
            ls_cands += [(a, b) for b in by_mod.get(mb, []) if b not in gone_md]
    ls_cv = [O.cut_values(og, None, ev.x, ev.y, ev.z, ev.sensor, 2, [*a, *b]) for a, b in ls_cands]
    drop_ls_marg = _pick(ls_cands, ls_cv, ls_set, in_band_kept)
    drop_ls_far = _pick(ls_cands, ls_cv, ls_set, far_kept)
    add_ls_marg = _pick(ls_cands, ls_cv, ls_set, in_band_rejected)
    add_ls_far = _pick(ls_cands, ls_cv, ls_set, far_rejected)

    # the perturbed result, with everything built on a dropped object removed
    g_md = [k for k in md if k not in gone_md] + [add_md_marg, add_md_far]
    gone_ls = {l for l in ls if l[0] in gone_md or l[1] in gone_md} | {drop_ls_marg, drop_ls_far}
    g_ls = [l for l in ls if l not in gone_ls] + [add_ls_marg, add_ls_far]
    gone_t3 = {t for t in t3 if (t[0], t[1]) in gone_ls or (t[1], t[2]) in gone_ls}
    g_t3 = [t for t in t3 if t not in gone_t3]
    gone_t5 = {t for t in t5 if t[:3] in gone_t3 or t[2:] in gone_t3}
    g_t5 = [t for t in t5 if t not in gone_t5]
    assert gone_t3 and gone_t5

    idx = {k: i for i, k in enumerate(g_md)}
    fake = KeyObjects(np.array(g_md, np.int64), np.array([(idx[a], idx[b]) for a, b in g_ls], np.int64),
                      np.array([[idx[k] for k in t] for t in g_t3], np.int64).reshape(-1, 3),
                      np.array([[idx[k] for k in t] for t in g_t5], np.int64).reshape(-1, 5))
    reps = CMP.compare(og, None, ev, fake, orc)
    got = [(r.marginal, r.violation, r.inherited) for r in reps]
    n_ls_inh = len([l for l in ls if l[0] in gone_md or l[1] in gone_md])
    expect = [(2, 2, 0), (2, 2, n_ls_inh), (0, 0, len(gone_t3)), (0, 0, len(gone_t5))]
    assert got == expect, (got, expect)
    assert n_ls_inh > 0
    # the example list names the violations, with the side that kept them
    assert {e[1] for e in reps[0].examples} == {"gpu", "oracle"}


def test_classifier_on_identical_results_is_clean(geo_full):
    og = O.Geom(geo_full.to_blob())
    ev = E.make_event(geo_full, E.EventConfig("t", 200, 0.1, 1.0, 2.4, 5.0, 2000, True), (7, 0))
    orc = O.build_objects(og, None, ev.x, ev.y, ev.z, ev.sensor)
    t3 = orc.t3_mds(); t5 = orc.t5_mds()
    fake = KeyObjects(orc.md.astype(np.int64), orc.ls.astype(np.int64), t3, t5)
    for r in CMP.compare(og, None, ev, fake, orc):
        assert (r.marginal, r.violation, r.inherited, r.duplicates) == (0, 0, 0, 0)
        assert r.n_gpu == r.n_oracle
