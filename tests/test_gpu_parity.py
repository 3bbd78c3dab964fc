"""GPU parity: the HIP library (through the C ABI) against the FP64 oracle.

Object sets must agree with zero violations (only marginal / inherited
differences, see tests/compare.py); T5 scores within 1e-5 absolute on the
FP32 path and 2e-2 on the BF16-MFMA path; chi2 values within FP32 rounding.
"""
import math
import sys

import numpy as np
import pytest

from oracle import oracle as O
from paper_2403_13166_amd.synth import geometry as G, events as E, model as M
from tests import compare as CMP

pytestmark = pytest.mark.gpu

torch = pytest.importorskip("torch")


def _say(*a):
    print(*a, flush=True)
    sys.stdout.flush()


@pytest.fixture(scope="module")
def geo_b():
    return G.make_geometry(False)


@pytest.fixture(scope="module")
def geo_f():
    return G.make_geometry(True)


@pytest.fixture(scope="module")
def mdl():
    return M.make_model()


@pytest.fixture(scope="module")
def builder_f(geo_f, mdl):
    from paper_2403_13166_amd.runtime import Builder
    b = Builder(geo_f.to_blob(), mdl.to_blob(), 0)
    yield b
    b.close()


@pytest.fixture(scope="module")
def builder_b(geo_b, mdl):
    from paper_2403_13166_amd.runtime import Builder
    b = Builder(geo_b.to_blob(), mdl.to_blob(), 0)
    yield b
    b.close()


def run_gpu(builder, ev, **kw):
    from paper_2403_13166_amd.runtime import to_device
    x, y, z, s = to_device(ev, builder.device)
    out = builder.build(x, y, z, s, **kw)
    torch.cuda.synchronize()
    return out.to_host()


def check_parity(geo, mdl, ev, gh, mode=0, score_tol=1e-5, label=""):
    og, om = O.Geom(geo.to_blob()), O.Model(mdl.to_blob())
    orc = O.build_objects(og, om, ev.x, ev.y, ev.z, ev.sensor, mode=mode)
    reps = CMP.compare(og, om, ev, gh, orc, mode)
    for st, r in zip(("MD", "LS", "T3", "T5"), reps):
        _say(f"{label} {st}: gpu {r.n_gpu} oracle {r.n_oracle} marginal {r.marginal} "
             f"inherited {r.inherited} violation {r.violation} dup {r.duplicates} {r.examples[:2]}")
        assert r.violation == 0, (st, r.examples)
        assert r.duplicates == 0, st
    err = CMP.score_errors(gh, orc)
    _say(f"{label} score/chi2 errors: {err}")
    if mode == 0:
        assert err["score"][0] <= score_tol
    else:
        assert np.all(np.isnan(gh.t5_score))
    assert err["chi2_rz_rel"][0] < 1e-4 and err["chi2_rphi_rel"][0] < 1e-4
    return reps, orc


def test_small_barrel_event_parity(builder_b, geo_b, mdl):
    for e in range(3):
        ev = E.make_event(geo_b, E.SMALL_BARREL, (0, e))
        _say(f"small barrel event {e}: {ev.n} hits")
        gh = run_gpu(builder_b, ev, with_features=True)
        reps, orc = check_parity(geo_b, mdl, ev, gh, label=f"C0[{e}]")
        assert reps[3].n_gpu > 100
        worst = CMP.feature_errors(gh, orc, PHI_COLS)
        assert np.max(worst) < 1e-5, np.argmax(worst)


# feature columns that are angles (anchor phi and the T5 direction): compared modulo 2 pi
PHI_COLS = [1, 7, 13, 19, 25, 36]


def test_pu200_event_parity_f32(builder_f, geo_f, mdl):
    """Object sets, scores, chi2 and every one of the 42 features of every
    common T5 (barrel and endcap anchors) against the oracle."""
    ev = E.make_event(geo_f, E.PU200, (1, 0))
    _say(f"PU200 event: {ev.n} hits")
    gh = run_gpu(builder_f, ev, with_features=True)
    reps, orc = check_parity(geo_f, mdl, ev, gh, label="C1 f32")
    assert reps[0].n_gpu > 30000 and reps[3].n_gpu > 10000
    worst = CMP.feature_errors(gh, orc, PHI_COLS)
    _say("C1 worst feature error per column", np.array2string(worst, precision=2))
    assert np.max(worst) < 1e-5, int(np.argmax(worst))
    # endcap anchors are among the compared rows
    assert np.any(gh.t5_feat[:, 5] == 1.0) and np.any(gh.t5_feat[:, 29] == 1.0)


def test_pu200_event_parity_bf16_scores(builder_f, geo_f, mdl):
    ev = E.make_event(geo_f, E.PU200, (1, 1))
    gh = run_gpu(builder_f, ev, precision=1)
    check_parity(geo_f, mdl, ev, gh, score_tol=2e-2, label="C1 bf16")


def test_pu200_pre_dnn_mode(builder_f, geo_f, mdl):
    ev = E.make_event(geo_f, E.PU200, (1, 2))
    gh = run_gpu(builder_f, ev, mode=1)
    reps, orc = check_parity(geo_f, mdl, ev, gh, mode=1, label="C1 pre-DNN")
    assert reps[3].n_gpu < len(O.build_objects(O.Geom(geo_f.to_blob()), O.Model(mdl.to_blob()),
                                               ev.x, ev.y, ev.z, ev.sensor, mode=0).t5)


def test_score_min_cut(builder_f, geo_f, mdl):
    ev = E.make_event(geo_f, E.PU200, (1, 3))
    gh = run_gpu(builder_f, ev, score_min=0.6)
    og, om = O.Geom(geo_f.to_blob()), O.Model(mdl.to_blob())
    orc = O.build_objects(og, om, ev.x, ev.y, ev.z, ev.sensor, mode=0, score_min=0.6)
    reps = CMP.compare(og, om, ev, gh, orc, 0, 0.6)
    for r in reps:
        assert r.violation == 0, r.examples
    assert np.all(gh.t5_score >= 0.6)


def test_deterministic_outputs(builder_f, geo_f):
    ev = E.make_event(geo_f, E.PU200, (1, 4))
    a = run_gpu(builder_f, ev)
    b = run_gpu(builder_f, ev)
    for f in ("md_hits", "ls_md", "t3_ls", "t5_t3", "t5_score", "t5_chi2_rz"):
        assert np.array_equal(getattr(a, f), getattr(b, f), equal_nan=True), f


def test_batched_equals_single_and_oracle(builder_f, geo_f, mdl):
    from paper_2403_13166_amd.runtime import Builder
    rng = E.event_rng(2, 99)
    evs = [E.make_event(geo_f, E.batch_event_config(rng), (2, 99, i)) for i in range(4)]
    evs.append(E.make_event(geo_f, E.EventConfig("tiny", 3, 0.1, 1.0, 1.0, 0.0, 20, True), (2, 99, 9)))
    # a one-hit event mid-batch: a run of every module without MDs in the
    # (event, module) offsets
    one = evs[1]
    evs.insert(2, E.Event(one.x[:1].copy(), one.y[:1].copy(), one.z[:1].copy(), one.sensor[:1].copy(),
                          one.truth[:1].copy(), one.tracks))
    x, y, z, s, off = E.concat_events(evs)
    dev = builder_f.device
    T = lambda a: torch.from_numpy(a).to(dev)
    out = builder_f.build(T(x), T(y), T(z), T(s), event_offsets=T(off))
    torch.cuda.synchronize()
    bh = out.to_host()
    eo = bh.event_offsets
    for i, ev in enumerate(evs):
        sh = run_gpu(builder_f, ev)
        md = bh.md_hits[eo[0, i]:eo[0, i + 1]] - off[i]
        assert np.array_equal(md, sh.md_hits), i
        ls = bh.ls_md[eo[1, i]:eo[1, i + 1]] - eo[0, i]
        assert np.array_equal(ls, sh.ls_md), i
        t3 = bh.t3_ls[eo[2, i]:eo[2, i + 1]] - eo[1, i]
        assert np.array_equal(t3, sh.t3_ls), i
        t5 = bh.t5_t3[eo[3, i]:eo[3, i + 1]] - eo[2, i]
        assert np.array_equal(t5, sh.t5_t3), i
        assert np.array_equal(bh.t5_score[eo[3, i]:eo[3, i + 1]], sh.t5_score), i
    # sampled events of the batch against the oracle
    for i in (0, len(evs) - 1):
        sh = run_gpu(builder_f, evs[i])
        check_parity(geo_f, mdl, evs[i], sh, label=f"batch[{i}]")


def test_standalone_scoring(builder_f, mdl):
    X = M.make_scoring_inputs(200_000, seed=(3, 0))
    om = O.Model(M.make_model(standardise=False).to_blob())
    from paper_2403_13166_amd.runtime import Builder
    geo = G.make_geometry(False)
    b = Builder(geo.to_blob(), M.make_model(standardise=False).to_blob(), 0)
    try:
        ref = O.mlp(om, X[:20000])
        Xd = torch.from_numpy(X).to(b.device)
        s32 = b.score(Xd, precision=0).cpu().numpy()
        s16 = b.score(Xd, precision=1).cpu().numpy()
        sb = b.score(Xd.to(torch.bfloat16), precision=1).cpu().numpy()
        e32 = np.max(np.abs(s32[:20000] - ref))
        e16 = np.max(np.abs(s16[:20000] - ref))
        _say(f"scoring: f32 max err {e32:.2e}, bf16-mfma max err {e16:.2e}, mean {np.mean(np.abs(s16[:20000]-ref)):.2e}")
        assert e32 <= 1e-5
        assert e16 <= 2e-2
        # bf16 inputs: same as rounding the inputs first
        Xr = torch.from_numpy(X[:20000]).to(torch.bfloat16).float().numpy()
        assert np.max(np.abs(sb[:20000] - O.mlp(om, Xr))) <= 2e-2
        assert np.all(np.isfinite(s16)) and s16.shape == (200_000,)
        # ragged tails: n not a multiple of 64 / 256
        for n in (1, 63, 65, 257, 1000):
            t = b.score(Xd[:n].contiguous(), precision=1).cpu().numpy()
            assert np.array_equal(t, s16[:n])
    finally:
        b.close()


def test_edge_cases(builder_f, geo_f):
    from paper_2403_13166_amd import binding as B
    dev = builder_f.device
    T = lambda a: torch.from_numpy(np.ascontiguousarray(a)).to(dev)
    # empty event
    e = np.zeros(0, np.float32)
    out = builder_f.build(T(e), T(e), T(e), T(np.zeros(0, np.int32)))
    assert out.counts() == (0, 0, 0, 0)
    # a single hit; hits all on one sensor
    ev = E.make_event(geo_f, E.PU200, (1, 5))
    one = builder_f.build(T(ev.x[:1]), T(ev.y[:1]), T(ev.z[:1]), T(ev.sensor[:1]))
    assert one.counts() == (0, 0, 0, 0)
    s0 = np.full(50, ev.sensor[0], np.int32)
    out = builder_f.build(T(ev.x[:50]), T(ev.y[:50]), T(ev.z[:50]), T(s0))
    assert out.counts()[0] == 0
    # invalid sensor id -> LST_E_INVAL
    bad = ev.sensor[:100].copy()
    bad[7] = 2 * geo_f.n_modules + 5
    with pytest.raises(B.LstError) as ex:
        builder_f.build(T(ev.x[:100]), T(ev.y[:100]), T(ev.z[:100]), T(bad))
    assert ex.value.status == B.LST_E_INVAL
    # too small capacities -> grown and retried transparently, same result
    from paper_2403_13166_amd.runtime import Builder, Caps
    ref = run_gpu(builder_f, ev)
    small = Caps(hits=ev.n, events=1, md=1000, ls=1000, t3=1000, t5=1000, cand=100_000)
    x, y, z, s = (T(a) for a in (ev.x, ev.y, ev.z, ev.sensor))
    h = B.LstHits(x.data_ptr(), y.data_ptr(), z.data_ptr(), s.data_ptr(), ev.n)
    builder_f.caps = None
    builder_f.reserve(small)
    st = B.lst_build_objects(builder_f.ctx, h, B.LstOptions(0, 0, float("nan"), 0), small.c(),
                             builder_f._objects_struct(False), builder_f._ws_ptr(), builder_f.ws_bytes,
                             torch.cuda.current_stream(dev).cuda_stream, check=False)
    assert st == B.LST_E_CAPACITY
    out = builder_f.build(x, y, z, s, caps=small).to_host()
    assert np.array_equal(out.t5_t3, ref.t5_t3) and np.array_equal(out.md_hits, ref.md_hits)


@pytest.mark.parametrize("stage", ["ls", "t3", "t5"])
def test_capacity_overflow_of_one_stage(geo_f, mdl, stage):
    """One capacity too small, the others ample: the call reports
    LST_E_CAPACITY with that stage's full required count, and the growing
    builder then returns the reference objects."""
    from paper_2403_13166_amd import binding as B
    from paper_2403_13166_amd.runtime import Builder, Caps
    ev = E.make_event(geo_f, E.PU200, (1, 8))
    b = Builder(geo_f.to_blob(), mdl.to_blob(), 0)
    ref = run_gpu(b, ev)
    n = {"ls": len(ref.ls_md), "t3": len(ref.t3_ls), "t5": len(ref.t5_t3)}
    full = Caps(hits=ev.n, events=1, md=2 * len(ref.md_hits), ls=2 * n["ls"], t3=2 * n["t3"], t5=2 * n["t5"],
                cand=40_000_000)
    small = Caps(**{**full.__dict__, stage: 1000})
    dev = b.device
    T = lambda a: torch.from_numpy(np.ascontiguousarray(a)).to(dev)
    x, y, z, s = (T(a) for a in (ev.x, ev.y, ev.z, ev.sensor))
    h = B.LstHits(x.data_ptr(), y.data_ptr(), z.data_ptr(), s.data_ptr(), ev.n)
    b.caps = None
    b.reserve(small)
    st = B.lst_build_objects(b.ctx, h, B.LstOptions(0, 0, float("nan"), 0), small.c(), b._objects_struct(False),
                             b._ws_ptr(), b.ws_bytes, torch.cuda.current_stream(dev).cuda_stream, check=False)
    assert st == B.LST_E_CAPACITY
    c = b.device_counts()
    got = {"ls": c[1], "t3": c[2], "t5": c[3]}[stage]
    _say(f"{stage} capacity 1000: reported {got}, required {n[stage]}")
    assert got == n[stage]                    # the full count, although only 1000 were stored
    out = b.build(x, y, z, s, caps=small).to_host()
    for k in ("md_hits", "ls_md", "t3_ls", "t5_t3", "t5_score"):
        assert np.array_equal(getattr(out, k), getattr(ref, k)), k
    b.close()


def test_mds_without_segments(builder_f, geo_f, mdl):
    """Hits on one barrel layer only: MDs but no LS, so the T3 stage runs on
    an empty list (its CSR by MD must be all zero) and nothing follows."""
    ev = E.make_event(geo_f, E.PU200, (1, 9))
    m = ev.sensor // 2
    keep = (geo_f.kind[m] == 0) & (geo_f.layer[m] == 3)
    one = E.Event(ev.x[keep], ev.y[keep], ev.z[keep], ev.sensor[keep], ev.truth[keep], ev.tracks)
    gh = run_gpu(builder_f, one)
    assert len(gh.md_hits) > 100 and len(gh.ls_md) == 0 and len(gh.t3_ls) == 0 and len(gh.t5_t3) == 0
    check_parity(geo_f, mdl, one, gh, label="one layer")


def test_dense_sensor_range_parity(builder_f, geo_f, mdl):
    """A PU200-like event plus 40k noise hits on the first sensor-id range:
    that range holds ~53k hits, more than one fine-binning block gathers
    through LDS, so its hits take the direct-store path."""
    ev = E.make_event(geo_f, E.PU200, (1, 7))
    rng = np.random.default_rng(11)
    x, y, z, s = E._noise_hits(geo_f, 1_500_000, rng)
    keep = s < 999
    dense = E.Event(np.concatenate([ev.x, x[keep].astype(np.float32)]),
                    np.concatenate([ev.y, y[keep].astype(np.float32)]),
                    np.concatenate([ev.z, z[keep].astype(np.float32)]),
                    np.concatenate([ev.sensor, s[keep].astype(np.int32)]),
                    np.concatenate([ev.truth, np.full(int(keep.sum()), -1, np.int32)]), ev.tracks)
    assert np.sum(dense.sensor < 999) > 40_000
    _say(f"dense range event: {dense.n} hits, {int(np.sum(dense.sensor < 999))} in sensors 0..998")
    gh = run_gpu(builder_f, dense)
    check_parity(geo_f, mdl, dense, gh, label="dense range")


def test_tunings_change_nothing_but_speed(builder_f, geo_f):
    from paper_2403_13166_amd import binding as B
    ev = E.make_event(geo_f, E.PU200, (1, 1))
    ref = run_gpu(builder_f, ev, precision=B.LST_PREC_BF16)
    default = B.lst_get_tuning(builder_f.ctx)
    variants = [
        # t3_masks 1 and 2 send most T3 wavefronts to the kernel for those
        # with more candidates than the kept pass masks
        {"bin_split": 1, "tile_per": [2, 2, 1, 1, 1], "eval_blocks": 256, "t3_masks": 1},
        {"bin_split": 32, "tile_per": [8, 8, 4, 4, 2], "eval_blocks": 8192, "t3_masks": 8},
        {"bin_split": 8, "tile_per": [2, 8, 4, 1, 2], "eval_blocks": 1024, "t3_masks": 2},
    ]
    try:
        for t in variants:
            _say("tuning", t)
            B.lst_set_tuning(builder_f.ctx, t)
            assert B.lst_get_tuning(builder_f.ctx) == t
            got = run_gpu(builder_f, ev, precision=B.LST_PREC_BF16)
            for k in ("md_hits", "ls_md", "t3_ls", "t5_t3", "t5_score", "t5_chi2_rphi", "t5_chi2_rz"):
                assert np.array_equal(getattr(got, k), getattr(ref, k)), (t, k)
        for bad in ({"bin_split": 0, "tile_per": [4, 4, 2, 2, 1], "eval_blocks": 4096},
                    {"bin_split": 4, "tile_per": [1, 4, 2, 2, 1], "eval_blocks": 4096},
                    {"bin_split": 4, "tile_per": [4, 4, 2, 2, 4], "eval_blocks": 4096},
                    {"bin_split": 4, "tile_per": [4, 3, 2, 2, 1], "eval_blocks": 4096},
                    {"bin_split": 4, "tile_per": [4, 4, 2, 2, 1], "eval_blocks": 100},
                    {"bin_split": 4, "tile_per": [4, 4, 2, 2, 1], "eval_blocks": 4096, "t3_masks": 0},
                    {"bin_split": 4, "tile_per": [4, 4, 2, 2, 1], "eval_blocks": 4096, "t3_masks": 9}):
            before = B.lst_get_tuning(builder_f.ctx)
            with pytest.raises(B.LstError) as ei:
                B.lst_set_tuning(builder_f.ctx, bad)
            assert ei.value.status == B.LST_E_INVAL
            assert B.lst_get_tuning(builder_f.ctx) == before
    finally:
        B.lst_set_tuning(builder_f.ctx, None)
    assert B.lst_get_tuning(builder_f.ctx) == default


def test_autotune_keeps_results(geo_f, mdl):
    from paper_2403_13166_amd import binding as B
    from paper_2403_13166_amd.autotune import autotune
    from paper_2403_13166_amd.runtime import Builder
    rng = E.event_rng(2, 5)
    evs = [E.make_event(geo_f, E.batch_event_config(rng), (2, 5, i)) for i in range(3)]
    x, y, z, s, off = E.concat_events(evs)
    b = Builder(geo_f.to_blob(), mdl.to_blob(), 0)
    T = lambda a: torch.from_numpy(a).to(b.device)
    dx, dy, dz, ds, doff = T(x), T(y), T(z), T(s), T(off)
    ref = b.build(dx, dy, dz, ds, event_offsets=doff).to_host()
    run = lambda: b.launch(dx, dy, dz, ds, event_offsets=doff)
    best, table = autotune(b, run, torch.cuda.synchronize, reps=1, log=_say)
    from paper_2403_13166_amd.autotune import KNOBS
    assert len(table) == len(KNOBS)
    B.lst_set_tuning(b.ctx, best)
    got = b.build(dx, dy, dz, ds, event_offsets=doff).to_host()
    for k in ("md_hits", "ls_md", "t3_ls", "t5_t3", "t5_score"):
        assert np.array_equal(getattr(got, k), getattr(ref, k)), k
    b.close()


def test_benchmark_batch_parity(geo_f, mdl):
    """The 64-event batch of the benchmark (same seeds, tuned launch shapes,
    replayed from a captured HIP graph): the replay equals the eager build bit
    for bit, and every one of its 64 events agrees with the oracle."""
    from paper_2403_13166_amd import binding as B
    from paper_2403_13166_amd.runtime import Builder, Caps
    rng = E.event_rng(2, 0)
    evs = [E.make_event(geo_f, E.batch_event_config(rng), (2, 0, e)) for e in range(64)]
    x, y, z, s, off = E.concat_events(evs)
    b = Builder(geo_f.to_blob(), mdl.to_blob(), 0)
    T = lambda a: torch.from_numpy(np.ascontiguousarray(a)).to(b.device)
    dx, dy, dz, ds, doff = T(x), T(y), T(z), T(s), T(off)
    eager = b.build(dx, dy, dz, ds, event_offsets=doff, precision=B.LST_PREC_BF16).to_host()
    _say("batch counts", [len(eager.md_hits), len(eager.ls_md), len(eager.t3_ls), len(eager.t5_t3)])
    B.lst_set_tuning(b.ctx, {"bin_split": 4, "tile_per": [2, 8, 2, 2, 1], "eval_blocks": 8192})
    stream = torch.cuda.Stream(device=b.device)
    with torch.cuda.stream(stream):
        b.launch(dx, dy, dz, ds, event_offsets=doff, precision=B.LST_PREC_BF16)
        stream.synchronize()
        g = torch.cuda.CUDAGraph()
        with torch.cuda.graph(g, stream=stream, capture_error_mode="relaxed"):
            b.launch(dx, dy, dz, ds, event_offsets=doff, precision=B.LST_PREC_BF16)
        for _ in range(3):
            g.replay()
            stream.synchronize()
            rep = b.view().to_host()
            for k in ("md_hits", "ls_md", "t3_ls", "t5_t3", "t5_score", "t5_chi2_rphi", "t5_chi2_rz",
                      "event_offsets"):
                assert np.array_equal(getattr(rep, k), getattr(eager, k)), k
    b.close()
    # every event of the batch against the oracle (oracle builds on host threads)
    from concurrent.futures import ThreadPoolExecutor
    from paper_2403_13166_amd.runtime import HostObjects
    og, om = O.Geom(geo_f.to_blob()), O.Model(mdl.to_blob())
    with ThreadPoolExecutor(8) as pool:
        orcs = list(pool.map(lambda ev: O.build_objects(og, om, ev.x, ev.y, ev.z, ev.sensor), evs))
    eo = eager.event_offsets
    tot = np.zeros((4, 3), np.int64)
    worst = 0.0
    for i in range(64):
        md = eager.md_hits[eo[0, i]:eo[0, i + 1]] - off[i]
        ls = eager.ls_md[eo[1, i]:eo[1, i + 1]] - eo[0, i]
        t3 = eager.t3_ls[eo[2, i]:eo[2, i + 1]] - eo[1, i]
        t5 = eager.t5_t3[eo[3, i]:eo[3, i + 1]] - eo[2, i]
        sl = slice(eo[3, i], eo[3, i + 1])
        gh = HostObjects(md, ls, t3, t5, eager.t5_score[sl], eager.t5_chi2_rphi[sl], eager.t5_chi2_rz[sl], None)
        reps = CMP.compare(og, om, evs[i], gh, orcs[i])
        for k, r in enumerate(reps):
            assert r.violation == 0 and r.duplicates == 0, (i, k, r.examples)
            tot[k] += (r.n_gpu, r.marginal, r.inherited)
        err = CMP.score_errors(gh, orcs[i])
        assert err["score"][0] <= 2e-2, (i, err)
        worst = max(worst, err["score"][0])
    _say("bench batch, all 64 events vs oracle: (objects, marginal, inherited) per stage MD/LS/T3/T5",
         tot.tolist(), f"max BF16 score error {worst:.2e}")


def test_threshold_edge_marginal_cases_counted(mdl):
    """The analytic threshold case on the GPU: with the resolution terms off
    (n_sigma = 0), noise-free tracks at pT = pT_min and z_v = +-Z sit on the
    curvature, bend and z-window thresholds, so the FP32 kernels and the FP64
    oracle decide some of them differently. Every such disagreement must be
    classified marginal (or inherited), never a violation, and there are
    some to classify."""
    from paper_2403_13166_amd.runtime import Builder
    from tests.helix import threshold_event
    geo = G.make_geometry(True, {"n_sigma": 0.0})
    ev = threshold_event(geo, 3, n_min=3000, n_high=300, n_noise=4000)
    _say(f"threshold-edge event: {ev.n} hits")
    b = Builder(geo.to_blob(), mdl.to_blob(), 0)
    try:
        gh = run_gpu(b, ev)
    finally:
        b.close()
    reps, _ = check_parity(geo, mdl, ev, gh, label="threshold edge")
    assert sum(r.marginal for r in reps) > 0
