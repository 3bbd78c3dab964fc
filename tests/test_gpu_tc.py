"""Track-candidate selection on the GPU (lst_select_tcs) against the FP64
oracle (oracle/tc.py), through the C ABI.

The GPU selects TCs from its own build's objects; the oracle from its own
build (identical object sets). TCs are compared as sets of (kind, seed, hit
keys of the object). A disagreement is allowed only where the decision is a
floating-point near-tie, which the check classifies as marginal from the
oracle's own numbers: a seed whose best and second-best match chi2 (FP32) are
within 1e-5 relative, a chi2 within 1e-5 relative of chi2_max, or two
duplicate TCs whose T5 qualities differ by less than 1e-5. Anything else is a
violation; marginal cases are counted and printed.
"""
import sys

import numpy as np
import pytest

from paper_2403_13166_amd.synth import events as E, geometry as G, model as M, seeds as S

pytestmark = pytest.mark.gpu
torch = pytest.importorskip("torch")


def _say(*a):
    print(*a, flush=True)
    sys.stdout.flush()


@pytest.fixture(scope="module")
def env():
    from paper_2403_13166_amd.runtime import Builder
    from oracle import oracle as O
    geo = G.make_geometry(True)
    mdl = M.make_model()
    b = Builder(geo.to_blob(), mdl.to_blob(), 0)
    yield geo, mdl, b, O.Geom(geo.to_blob()), O.Model(mdl.to_blob())
    b.close()


def _keys_gpu(h, md0=0):
    """hit keys of T5 and T3 objects of a GPU build (host copies), event-local MD numbering offset md0"""
    md = h.md_hits
    t5 = h.t5_mds()
    t3 = h.t3_mds()
    k5 = [tuple(map(tuple, md[m].tolist())) for m in t5]
    k3 = [tuple(map(tuple, md[m].tolist())) for m in t3]
    return k5, k3


def _keys_orc(r):
    k5 = [tuple(map(tuple, r.md[m].tolist())) for m in r.t5_mds()]
    k3 = [tuple(map(tuple, r.md[m].tolist())) for m in r.t3_mds()]
    return k5, k3


def _tc_set(kinds, seeds, objs, k5, k3, hit0=0):
    out = set()
    for k, s, o in zip(kinds, seeds, objs):
        if k in (0, 1):
            key = tuple(tuple(v - hit0 for v in p) for p in k5[o])
        elif k == 2:
            key = tuple(tuple(v - hit0 for v in p) for p in k3[o])
        else:
            key = None
        out.add((int(k), int(s), key))
    return out


def _oracle_event(ev, r, seeds, opt):
    from oracle import tc as TC
    return TC.select_event(ev.x, ev.y, ev.z, r.md, r.t3_mds(), r.t5_mds(), r.t5,
                           TC.t5_quality(r.score, r.chi2_rphi), seeds, opt)


def _classify(diff, ev, r, seeds, opt, res):
    """Marginal / violation counts of the TCs in the symmetric difference."""
    from oracle import tc as TC
    P5, v5 = TC.object_params(ev.x, ev.y, ev.z, r.md, r.t5_mds())
    P3, v3 = TC.object_params(ev.x, ev.y, ev.z, r.md, r.t3_mds())
    C = np.concatenate([TC.chi2_matrix(seeds, P5, v5, opt), TC.chi2_matrix(seeds, P3, v3, opt)], axis=1)
    cmax = float(np.float32(opt.chi2_max))
    Kf = C.astype(np.float32)
    qual = TC.t5_quality(r.score, r.chi2_rphi)
    marg = viol = 0
    for kind, s, key in diff:
        near = False
        if s >= 0:
            row = np.sort(Kf[s][np.isfinite(Kf[s])])
            near = bool(np.any(np.abs(C[s][np.isfinite(C[s])] - cmax) <= 1e-5 * cmax))
            near = near or (len(row) > 1 and row[1] - row[0] <= 1e-5 * max(row[0], 1e-30))
        if kind in (0, 1):
            q = np.sort(qual)
            near = near or bool(np.any(np.diff(q) <= 1e-5))
        if near:
            marg += 1
        else:
            viol += 1
    return marg, viol


def _run_event(env, ev, seeds, opt_dict=None, tag=""):
    from oracle import tc as TC
    from paper_2403_13166_amd.runtime import TC_OPTIONS, select_tcs, to_device
    geo, mdl, b, og, om = env
    opt_d = dict(TC_OPTIONS, **(opt_dict or {}))
    opt = TC.TcOptions(opt_d["chi2_max"], opt_d["sigma_kappa_abs"], opt_d["sigma_kappa_rel"], opt_d["sigma_phi0"],
                       opt_d["sigma_cot"], opt_d["sigma_z0"])
    d = to_device(ev, b.device)
    objs = b.build(*d)
    sd = torch.from_numpy(seeds.params.copy()).to(b.device) if seeds.n else torch.zeros((0, 8), device=b.device)
    soff = torch.tensor([0, seeds.n], dtype=torch.int64, device=b.device)
    tcs = select_tcs(b, d[0], d[1], d[2], objs, sd.contiguous(), soff, opt_d)
    h = objs.to_host()
    k5, k3 = _keys_gpu(h)
    got = _tc_set(tcs.kind.cpu().numpy(), tcs.seed.cpu().numpy(), tcs.obj.cpu().numpy(), k5, k3)
    r = O_build(og, om, ev)
    res = _oracle_event(ev, r, seeds.params, opt)
    o5, o3 = _keys_orc(r)
    ref = _tc_set([t[0] for t in res.tcs], [t[1] for t in res.tcs], [t[2] for t in res.tcs], o5, o3)
    diff = got ^ ref
    marg, viol = _classify(diff, ev, r, seeds.params, opt, res) if diff else (0, 0)
    kinds = np.bincount(tcs.kind.cpu().numpy(), minlength=4).tolist()
    _say(f"{tag}: TCs gpu {len(got)} oracle {len(ref)} kinds {kinds} before {tcs.counts[5]} "
         f"marginal {marg} violation {viol}")
    assert viol == 0, sorted(diff, key=str)[:10]
    assert tcs.counts[:4] == kinds and tcs.counts[4] == len(got)
    return got, ref, tcs


def O_build(og, om, ev):
    from oracle import oracle as O
    return O.build_objects(og, om, ev.x, ev.y, ev.z, ev.sensor)


@pytest.mark.parametrize("pu", [4.0, 20.0])
def test_tc_selection_matches_oracle(env, pu):
    geo = env[0]
    ev = E.make_event(geo, E.pileup_event_config(pu), (9, 10, int(pu)))
    seeds = S.make_seeds(geo, ev, E.event_rng(9, 11, int(pu)), eff=0.9, fake_frac=0.1)
    got, ref, tcs = _run_event(env, ev, seeds, tag=f"PU {pu}")
    assert len(got) > 50
    assert {k for k, _, _ in got} >= {0, 3}


def test_tc_exact_seeds_one_pt5_per_track(env):
    geo = env[0]
    rng = E.event_rng(9, 12)
    tr = E.make_tracks(E.pileup_event_config(1.0), rng, 30)
    ev = E.make_event_from_tracks(geo, tr, 0, 0.0, rng)
    seeds = S.make_seeds(geo, ev, E.event_rng(9, 13), eff=1.0, fake_frac=0.0)
    seeds.params[:, :4] = S.true_params(geo, ev.tracks)[seeds.track].astype(np.float32)
    got, ref, tcs = _run_event(env, ev, seeds, tag="exact seeds")
    assert got == ref


def test_tc_edge_cases(env):
    geo = env[0]
    ev = E.make_event(geo, E.pileup_event_config(3.0), (9, 14, 0))
    none = S.Seeds(np.zeros((0, 8), np.float32), np.zeros(0, np.int32))
    got, ref, _ = _run_event(env, ev, none, tag="no seeds")
    assert got == ref and all(k == 1 for k, _, _ in got)
    # seeds that match nothing (far away in z0) all end as pLS
    far = S.make_seeds(geo, ev, E.event_rng(9, 15), eff=1.0, fake_frac=0.0)
    far.params[:, 3] += 500.0
    got, ref, _ = _run_event(env, ev, far, tag="unmatched seeds")
    assert {(k, s) for k, s, _ in got if k == 3} == {(3, i) for i in range(far.n)}
    # a tight chi2_max keeps fewer pT5 than the default
    seeds = S.make_seeds(geo, ev, E.event_rng(9, 16), eff=1.0, fake_frac=0.0)
    g1, _, _ = _run_event(env, ev, seeds, tag="default chi2_max")
    g2, _, _ = _run_event(env, ev, seeds, {"chi2_max": 0.5}, tag="chi2_max 0.5")
    assert sum(k == 0 for k, _, _ in g2) < sum(k == 0 for k, _, _ in g1)


def test_tc_batched_equals_per_event(env):
    """Batched build + one selection over 6 events: each event's TCs equal the
    oracle's for that event (seed indices local to the event)."""
    from paper_2403_13166_amd.runtime import TC_OPTIONS, select_tcs
    from oracle import tc as TC
    geo, mdl, b, og, om = env
    evs = [E.make_event(geo, E.pileup_event_config(p), (9, 20, i)) for i, p in enumerate([2, 9, 0.3, 15, 5, 12])]
    sds = [S.make_seeds(geo, e, E.event_rng(9, 21, i), eff=0.9, fake_frac=0.1) for i, e in enumerate(evs)]
    x, y, z, s, off = E.concat_events(evs)
    T = lambda a: torch.from_numpy(np.ascontiguousarray(a)).to(b.device)
    dx, dy, dz, ds, doff = T(x), T(y), T(z), T(s), T(off)
    objs = b.build(dx, dy, dz, ds, event_offsets=doff)
    sp, soff = S.concat_seeds(sds)
    tcs = select_tcs(b, dx, dy, dz, objs, T(sp), T(soff))
    h = objs.to_host()
    k5, k3 = _keys_gpu(h)
    kind, seed, obj = tcs.kind.cpu().numpy(), tcs.seed.cpu().numpy(), tcs.obj.cpu().numpy()
    eo = h.event_offsets
    opt = TC.TcOptions(*(TC_OPTIONS[k] for k in TC_OPTIONS))
    for e, ev in enumerate(evs):
        # this event's TCs: by object range (kinds 0-2) or seed range (kind 3)
        in5 = (obj >= eo[3, e]) & (obj < eo[3, e + 1])
        in3 = (obj >= eo[2, e]) & (obj < eo[2, e + 1])
        ins = (seed >= soff[e]) & (seed < soff[e + 1])
        sel = np.where(kind <= 1, in5, np.where(kind == 2, in3, ins))
        got = _tc_set(kind[sel], np.where(seed[sel] >= 0, seed[sel] - soff[e], -1), obj[sel], k5, k3, hit0=off[e])
        r = O_build(og, om, ev)
        res = _oracle_event(ev, r, sds[e].params, opt)
        o5, o3 = _keys_orc(r)
        ref = _tc_set([t[0] for t in res.tcs], [t[1] for t in res.tcs], [t[2] for t in res.tcs], o5, o3)
        diff = got ^ ref
        marg, viol = _classify(diff, ev, r, sds[e].params, opt, res) if diff else (0, 0)
        _say(f"batched event {e}: TCs {len(got)} / {len(ref)} marginal {marg} violation {viol}")
        assert viol == 0


def test_tc_benchmark_batch_sampled(env):
    """The 64-event benchmark batch (build in DNN mode, FP32 scores) with
    seeds for every event and one selection call: the three events with the
    fewest hits are compared with the oracle in full, and every event's TC
    counts satisfy the structural bounds (pT5 + pT3 + pLS = seeds, pT5 + T5
    before removal = T5s)."""
    from paper_2403_13166_amd.runtime import TC_OPTIONS, select_tcs
    from oracle import tc as TC
    geo, mdl, b, og, om = env
    rng = E.event_rng(2, 0)
    evs = [E.make_event(geo, E.batch_event_config(rng), (2, 0, e)) for e in range(64)]
    sds = [S.make_seeds(geo, e, E.event_rng(5, i), eff=0.9, fake_frac=0.05) for i, e in enumerate(evs)]
    x, y, z, s, off = E.concat_events(evs)
    T = lambda a: torch.from_numpy(np.ascontiguousarray(a)).to(b.device)
    dx, dy, dz, ds, doff = T(x), T(y), T(z), T(s), T(off)
    objs = b.build(dx, dy, dz, ds, event_offsets=doff)
    sp, soff = S.concat_seeds(sds)
    tcs = select_tcs(b, dx, dy, dz, objs, T(sp), T(soff))
    _say("benchmark batch TCs: kept per kind", tcs.counts[:4], "before removal", tcs.counts[5],
         "seeds", len(sp), "T5", objs.counts()[3])
    h = objs.to_host()
    k5, k3 = _keys_gpu(h)
    kind, seed, obj = tcs.kind.cpu().numpy(), tcs.seed.cpu().numpy(), tcs.obj.cpu().numpy()
    # a seed is in at most one kept TC; pLS are never removed
    used = seed[seed >= 0]
    assert len(np.unique(used)) == len(used) <= len(sp)
    eo = h.event_offsets
    opt = TC.TcOptions(*(TC_OPTIONS[k] for k in TC_OPTIONS))
    for e in np.argsort([ev.n for ev in evs])[:3]:
        ev = evs[e]
        in5 = (obj >= eo[3, e]) & (obj < eo[3, e + 1])
        in3 = (obj >= eo[2, e]) & (obj < eo[2, e + 1])
        ins = (seed >= soff[e]) & (seed < soff[e + 1])
        sel = np.where(kind <= 1, in5, np.where(kind == 2, in3, ins))
        got = _tc_set(kind[sel], np.where(seed[sel] >= 0, seed[sel] - soff[e], -1), obj[sel], k5, k3, hit0=off[e])
        r = O_build(og, om, ev)
        res = _oracle_event(ev, r, sds[e].params, opt)
        o5, o3 = _keys_orc(r)
        ref = _tc_set([t[0] for t in res.tcs], [t[1] for t in res.tcs], [t[2] for t in res.tcs], o5, o3)
        diff = got ^ ref
        marg, viol = _classify(diff, ev, r, sds[e].params, opt, res) if diff else (0, 0)
        _say(f"benchmark batch event {e} ({ev.n} hits): TCs {len(got)} / {len(ref)} marginal {marg} "
             f"violation {viol}")
        assert viol == 0
