"""Pins of the track-candidate selection oracle (oracle/tc.py) on the CPU.

* Object helix parameters on noise-free helices equal the generated track's
  parameters (a closed form independent of the selection code): a wrong sign,
  angle convention or arc length shows here.
* Match chi2: zero at equal parameters, k^2 for a k-sigma shift of each
  parameter alone (sigma from the seed and object widths in quadrature), and
  phi0 differences taken across the +-pi seam.
* Mutual best matching and duplicate removal against hand-worked cases
  (tests/golden/tc_selection_cases.json).
* Whole selection: on noise-free tracks with exact seeds every track with a
  T5 ends as one pT5; on a noisy event with fake seeds, the structural
  invariants of the reading hold (every seed and T5 in exactly one TC before
  duplicate removal, the pT5 / pT3 pairs are mutual best matches by brute
  force, no two kept TCs are duplicates, every removed TC has a better
  duplicate).
"""
import json
import math
import os

import numpy as np
import pytest

from oracle import tc as TC

GOLD = json.load(open(os.path.join(os.path.dirname(__file__), "golden", "tc_selection_cases.json")))


@pytest.fixture(scope="module")
def clean(geo_full, model):
    from oracle import oracle as O
    from paper_2403_13166_amd.synth import events as E
    rng = E.event_rng(9, 1)
    tr = E.make_tracks(E.pileup_event_config(1.0), rng, 20)
    ev = E.make_event_from_tracks(geo_full, tr, 0, 0.0, rng)
    r = O.build_objects(O.Geom(geo_full.to_blob()), O.Model(model.to_blob()), ev.x, ev.y, ev.z, ev.sensor)
    return ev, r


def test_object_params_equal_the_generated_helix(geo_full, clean):
    from paper_2403_13166_amd.synth import seeds as S
    ev, r = clean
    truth = S.true_params(geo_full, ev.tracks)
    for mds in (r.t5_mds(), r.t3_mds()):
        assert len(mds) > 20
        P, v = TC.object_params(ev.x, ev.y, ev.z, r.md, mds)
        assert v.all()
        tid = ev.truth[r.md[mds[:, 0], 0]]
        assert np.all(ev.truth[r.md[mds[:, -1], 0]] == tid)
        d = P - truth[tid]
        d[:, 1] = (d[:, 1] + math.pi) % (2 * math.pi) - math.pi
        # FP32 hit coordinates (~1e-5 relative near 100 cm) bound the deviations
        assert np.all(np.abs(d[:, 0]) <= 1e-5 * np.abs(truth[tid][:, 0]) + 1e-9)
        assert np.all(np.abs(d[:, 1]) <= 1e-6)
        assert np.all(np.abs(d[:, 2]) <= 1e-5 * (1 + np.abs(truth[tid][:, 2])))
        assert np.all(np.abs(d[:, 3]) <= 1e-3)


def test_chi2_shifts_and_seam():
    opt = TC.TcOptions()
    P = np.array([[3e-3, 3.1, 0.5, 1.0], [-2e-3, -1.0, -2.0, -4.0]])
    v = np.ones(2, bool)
    f = lambda v: float(np.float32(v))        # the options are FP32 numbers
    sig_o = lambda p: np.array([f(opt.kappa_rel) * abs(p[0]) + f(opt.kappa_abs), f(opt.phi0), f(opt.cot), f(opt.z0)])
    for j in range(2):
        s_seed = np.array([1e-4, 1e-3, 2e-3, 0.05])
        seed = np.concatenate([P[j], s_seed])[None, :]
        assert TC.chi2_matrix(seed, P, v, opt)[0, j] == pytest.approx(0.0, abs=1e-20)
        for i in range(4):
            for k in (0.5, 1.0, 3.0):
                sh = seed.copy()
                w = math.sqrt(s_seed[i] ** 2 + sig_o(P[j])[i] ** 2)
                sh[0, i] += k * w
                if i == 1:       # across the seam: +pi and -pi are the same direction
                    sh[0, 1] = (sh[0, 1] + math.pi) % (2 * math.pi) - math.pi
                assert TC.chi2_matrix(sh, P, v, opt)[0, j] == pytest.approx(k * k, rel=1e-9)
    # an object without parameters never matches
    assert np.isinf(TC.chi2_matrix(np.zeros((1, 8)) + 1, P, np.array([False, True]), opt)[0, 0])


@pytest.mark.parametrize("case", GOLD["mutual_best"], ids=lambda c: c["note"][:30])
def test_mutual_best_hand_cases(case):
    C = np.array([[np.inf if v is None else v for v in row] for row in case["chi2"]])
    got = TC.mutual_best(C, case["chi2_max"], np.ones(C.shape[0], bool), np.ones(C.shape[1], bool))
    assert sorted(map(list, got)) == sorted(case["pairs"])


def test_duplicate_removal_hand_case():
    g = GOLD["duplicates"]
    t5 = np.array(g["t5_mds"])
    n_md = int(t5.max()) + 1
    md_hits = np.stack([np.arange(n_md), np.arange(n_md)], axis=1)
    x = np.linspace(20, 30, n_md).astype(np.float32)
    y = np.zeros(n_md, np.float32)
    z = np.zeros(n_md, np.float32)
    res = TC.select_event(x, y, z, md_hits, np.zeros((0, 3), int), t5, np.zeros((len(t5), 2), int),
                          np.array(g["quality"]), np.zeros((0, 8), np.float32))
    assert [o for k, _, o in res.before] == list(range(len(t5)))
    assert sorted(o for k, _, o in res.tcs) == g["kept"]


def test_exact_seeds_give_one_pt5_per_track(geo_full, clean):
    from paper_2403_13166_amd.synth import events as E, seeds as S
    ev, r = clean
    sd = S.make_seeds(geo_full, ev, E.event_rng(9, 2), eff=1.0, fake_frac=0.0)
    sd.params[:, :4] = S.true_params(geo_full, ev.tracks)[sd.track].astype(np.float32)
    t5m = r.t5_mds()
    res = TC.select_event(ev.x, ev.y, ev.z, r.md, r.t3_mds(), t5m, r.t5, TC.t5_quality(r.score, r.chi2_rphi),
                          sd.params)
    with_t5 = set(ev.truth[r.md[t5m[:, 0], 0]].tolist())
    pt5 = [(p, o) for k, p, o in res.tcs if k == TC.K_PT5]
    assert len(pt5) == len(with_t5) > 10
    # each pT5 joins a seed with a T5 of its own track; nothing else of those tracks is kept
    assert all(sd.track[p] == ev.truth[r.md[t5m[o, 0], 0]] for p, o in pt5)
    assert not any(k == TC.K_T5 and ev.truth[r.md[t5m[o, 0], 0]] in with_t5 for k, _, o in res.tcs)


def test_selection_invariants_on_a_noisy_event(geo_full, model):
    from oracle import oracle as O
    from paper_2403_13166_amd.synth import events as E, seeds as S
    ev = E.make_event(geo_full, E.pileup_event_config(8.0), (9, 3, 0))
    r = O.build_objects(O.Geom(geo_full.to_blob()), O.Model(model.to_blob()), ev.x, ev.y, ev.z, ev.sensor)
    sd = S.make_seeds(geo_full, ev, E.event_rng(9, 4), eff=0.9, fake_frac=0.1)
    t5m, t3m = r.t5_mds(), r.t3_mds()
    opt = TC.TcOptions()
    res = TC.select_event(ev.x, ev.y, ev.z, r.md, t3m, t5m, r.t5, TC.t5_quality(r.score, r.chi2_rphi),
                          sd.params, opt)
    b = res.before
    assert sorted(p for k, p, _ in b if k != TC.K_T5) == list(range(sd.n))
    assert sorted(o for k, _, o in b if k in (TC.K_PT5, TC.K_T5)) == list(range(len(t5m)))
    # brute force: pT5 pairs are mutual best matches
    P5, v5 = TC.object_params(ev.x, ev.y, ev.z, r.md, t5m)
    C5 = TC.chi2_matrix(sd.params, P5, v5, opt).astype(np.float32)
    C5[C5 > opt.chi2_max] = np.inf
    for k, p, o in b:
        if k == TC.K_PT5:
            assert C5[p, o] == C5[p].min() and np.argmin(C5[p]) == o and np.argmin(C5[:, o]) == p
    used_t3 = {int(t) for k, _, o in b if k == TC.K_PT5 for t in r.t5[o]}
    assert not any(k == TC.K_PT3 and o in used_t3 for k, _, o in b)
    # duplicates: none among the kept, a better one for every removed TC
    sets = {tc: set((t5m[tc[2]] if tc[0] < 2 else t3m[tc[2]]).tolist()) for tc in b if tc[0] != TC.K_PLS}
    dup = lambda a, c: len(sets[a] & sets[c]) > min(len(sets[a]), len(sets[c])) / 2
    kept = [tc for tc in res.tcs if tc[0] != TC.K_PLS]
    for i, a in enumerate(kept):
        for c in kept[i + 1:]:
            assert not dup(a, c)
    removed = set(b) - set(res.tcs)
    assert removed and all(tc[0] != TC.K_PLS for tc in removed)
    qual = TC.t5_quality(r.score, r.chi2_rphi)
    key = lambda tc: (tc[0], res.chi2[tc] if tc[0] == TC.K_PT3 else qual[tc[2]], tc[2])
    for a in removed:
        assert any(c != a and dup(a, c) and key(c) < key(a) for c in sets)
    # the reading is useful: most seeded tracks with a T5 end as pT5, most fakes as pLS
    t5_tracks = set(ev.truth[r.md[t5m[:, 0], 0]].tolist())
    seeded = [p for p in range(sd.n) if sd.track[p] in t5_tracks]
    in_pt5 = {p for k, p, _ in res.tcs if k == TC.K_PT5}
    assert len(in_pt5 & set(seeded)) >= 0.8 * len(seeded)
    fakes = [p for p in range(sd.n) if sd.track[p] < 0]
    pls = {p for k, p, _ in res.tcs if k == TC.K_PLS}
    assert len(pls & set(fakes)) >= 0.8 * len(fakes)
