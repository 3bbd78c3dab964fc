"""CPU tests of the T5-DNN training step (Sec. 2, Sec. 3; matching rule of Sec. 1).

* the truth rule: a T5 is real with more than 75 % of its 10 hits from one
  simulated track (noise hits belong to none);
* the cross-entropy gradient against central finite differences of the loss;
* training on FP64 oracle features of PU200-like events separates real from
  fake T5s, and at the working point that matches the pre-DNN (chi2_rphi cut)
  real-T5 efficiency it keeps fewer fake T5s than the cut (the paper's
  qualitative claim; its numbers come from CMS data and are not comparable).
"""
import numpy as np
import pytest

from oracle import oracle as O
from paper_2403_13166_amd import train as TR
from paper_2403_13166_amd.synth import events as E, geometry as G, model as M


def test_truth_rule_more_than_75_percent():
    md_hits = np.arange(10).reshape(5, 2)        # MD k = hits (2k, 2k + 1)
    t5 = np.array([[0, 1, 2, 3, 4]])
    cases = [([3] * 10, True, 3), ([3] * 8 + [5, 5], True, 3), ([3] * 7 + [5, 5, 5], False, -1),
             ([3] * 8 + [-1, -1], True, 3), ([-1] * 3 + [3] * 7, False, -1), ([-1] * 10, False, -1),
             ([1, 2] * 5, False, -1), ([9] * 9 + [2], True, 9)]
    for tr, real, tid in cases:
        r, t = TR.t5_truth(md_hits, t5, np.array(tr))
        assert bool(r[0]) == real and int(t[0]) == tid, (tr, r, t)
    # the hit order inside the T5 does not matter
    r, t = TR.t5_truth(md_hits, np.array([[4, 2, 0, 3, 1]]), np.array([5, 3, 3, 3, 3, 3, 3, 3, 3, 5]))
    assert r[0] and t[0] == 3


def test_bce_gradient_matches_finite_differences():
    rng = np.random.default_rng(1)
    P = TR.init_params((9, 9))
    for k in P:
        P[k] = P[k] + rng.normal(0, 0.1, P[k].shape)    # nonzero biases, mixed ReLU states
    xs = rng.normal(0, 1, (64, 42))
    y = (rng.random(64) < 0.5).astype(float)
    g = TR.bce_grad(P, xs, y)
    h = 1e-6
    for k in P:
        flat = P[k].reshape(-1)
        for idx in rng.choice(flat.size, min(6, flat.size), replace=False):
            old = flat[idx]
            flat[idx] = old + h
            lp = TR.bce_loss(TR.forward(P, xs)[4], y)
            flat[idx] = old - h
            lm = TR.bce_loss(TR.forward(P, xs)[4], y)
            flat[idx] = old
            num = (lp - lm) / (2 * h)
            assert abs(num - g[k].reshape(-1)[idx]) < 1e-6 * max(1.0, abs(num)), (k, idx, num)
    # the loss itself: binary cross entropy of the sigmoid
    z = TR.forward(P, xs)[4]
    p = 1 / (1 + np.exp(-z))
    assert abs(TR.bce_loss(z, y) + np.mean(y * np.log(p) + (1 - y) * np.log(1 - p))) < 1e-12


def test_working_point_keeps_the_target_fraction():
    s = np.linspace(0, 1, 1001)
    for eff in (0.1, 0.5, 0.753, 1.0):
        t = TR.working_point(s, eff)
        assert np.mean(s >= t) >= eff and np.mean(s > t) < eff


def test_training_beats_the_circle_fit_cut_at_matched_efficiency():
    geo = G.make_geometry(True)
    og, om = O.Geom(geo.to_blob()), O.Model(M.make_model().to_blob())
    X, y, c2 = [], [], []
    for e in range(3):
        ev = E.make_event(geo, E.PU200, (5, 500 + e))
        r = O.build_objects(og, om, ev.x, ev.y, ev.z, ev.sensor, mode=0)
        real, _ = TR.t5_truth(r.md, r.t5_mds(), ev.truth)
        X.append(r.feat); y.append(real); c2.append(r.chi2_rphi)
    X, y, c2 = np.concatenate(X), np.concatenate(y), np.concatenate(c2)
    assert len(y) > 50_000 and 0.3 < y.mean() < 0.9
    res = TR.fit(X, y, epochs=6)
    assert res.history[-1][2] < res.history[0][2] and res.history[-1][2] < 0.3
    te = res.test_index
    p = TR.predict(res.model, X[te])
    # ranking quality: probability that a real T5 outscores a fake one
    pr, pf = p[y[te]], p[~y[te]]
    auc = np.mean(pr[:, None] > pf[None, :2000])
    assert auc > 0.9, auc
    cmp = TR.compare_selections(p, c2[te], y[te], np.arange(len(te)), np.arange(len(te)),
                                geo.params["chi2_rphi_max"])
    assert abs(cmp["dnn"]["real_t5_efficiency"] - cmp["pre_dnn"]["real_t5_efficiency"]) < 1e-3
    assert cmp["dnn"]["fakes_kept"] < 0.5 * cmp["pre_dnn"]["fakes_kept"], cmp
    # the trained blob scores like its FP64 forward in the oracle's MLP
    om2 = O.Model(res.model.to_blob())
    assert np.max(np.abs(O.mlp(om2, X[te[:2000]].astype(np.float32)) - TR.predict(res.model, X[te[:2000]].astype(np.float32)))) < 1e-9
