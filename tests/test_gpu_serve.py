"""Serving on the GPU: every event's objects are the same when it is built
alone and when it is served inside a mixed, overlapping stream of batches.

Indices are compared exactly (event-local numbering); scores and chi2 values
to 1e-6 absolute (each object's arithmetic does not depend on its batch, so
they are expected to be bit-identical)."""
import sys

import numpy as np
import pytest

from paper_2403_13166_amd.synth import events as E, geometry as G, model as M

pytestmark = pytest.mark.gpu
torch = pytest.importorskip("torch")

KEYS_INT = ("md_hits", "ls_md", "t3_ls", "t5_t3")
KEYS_F = ("t5_score", "t5_chi2_rphi", "t5_chi2_rz")


def _say(*a):
    print(*a, flush=True)
    sys.stdout.flush()


@pytest.fixture(scope="module")
def setup():
    geo = G.make_geometry(True)
    mdl = M.make_model()
    rng = E.event_rng(4, 77)
    pus = rng.uniform(10, 60, size=7)
    pool = [E.make_event(geo, E.pileup_event_config(float(p)), (4, 77, i)) for i, p in enumerate(pus)]
    return geo, mdl, pool


def _alone(geo, mdl, pool, precision):
    from paper_2403_13166_amd.runtime import Builder, to_device
    b = Builder(geo.to_blob(), mdl.to_blob(), 0)
    out = []
    for ev in pool:
        o = b.build(*to_device(ev, b.device), precision=precision).to_host()
        out.append({k: getattr(o, k) for k in KEYS_INT + KEYS_F})
    torch.cuda.synchronize()
    b.close()
    return out


def _check(res, ref, tag):
    for k in KEYS_INT:
        assert np.array_equal(res[k], ref[k]), (tag, k, res[k].shape, ref[k].shape)
    for k in KEYS_F:
        assert res[k].shape == ref[k].shape, (tag, k)
        if res[k].size:
            d = np.abs(res[k] - ref[k])
            assert np.nanmax(np.where(np.isnan(ref[k]) & np.isnan(res[k]), 0, d)) <= 1e-6, (tag, k)


@pytest.mark.parametrize("use_graph", [True, False])
def test_served_equals_alone(setup, use_graph):
    from paper_2403_13166_amd.serve import Admission, GpuExecutor, Request, pinned_event, run_loop, slot_caps
    geo, mdl, pool = setup
    prec = 1
    ref = _alone(geo, mdl, pool, prec)
    hits = [e.n for e in pool]
    cap = sum(sorted(hits)[-3:])
    _say("serve: graph", use_graph, "hits", hits, "slot hits cap", cap)
    ex = GpuExecutor(geo.to_blob(), mdl.to_blob(), 2, slot_caps(cap, 3), mode=0, precision=prec,
                     use_graph=use_graph, keep_results=True)
    pins = [pinned_event(e) for e in pool]
    # a burst, then stragglers that arrive while the first batches run, then a repeat of event 0
    arr = [0, 0, 0, 0, 0.002, 0.004, 0.004, 0.03]
    idx = [0, 1, 2, 3, 4, 5, 6, 0]
    reqs = [Request(i, a, pool[j].n, pins[j]) for i, (a, j) in enumerate(zip(arr, idx))]
    done, st = run_loop(reqs, ex, Admission(cap, 3))
    _say("serve stats", st)
    assert st["events"] == len(reqs)
    assert st["max_inflight"] == 2 and st["max_batch"] >= 2
    for i, j in enumerate(idx):
        _check(ex.results[i], ref[j], f"request {i} (event {j})")
    ex.close()


def test_heterogeneous_slots_equal_alone(setup):
    from paper_2403_13166_amd.serve import GpuExecutor, Request, pinned_event, run_loop, slot_caps
    geo, mdl, pool = setup
    ref = _alone(geo, mdl, pool, 1)
    big = sum(sorted(e.n for e in pool)[-4:])
    caps = [slot_caps(max(e.n for e in pool), 1), slot_caps(big, 4)]
    ex = GpuExecutor(geo.to_blob(), mdl.to_blob(), 2, caps, precision=1, use_graph=True, keep_results=True)
    pins = [pinned_event(e) for e in pool]
    arr = [0, 0, 0, 0, 0, 0.003, 0.02]
    reqs = [Request(i, a, pool[i].n, pins[i]) for i, a in enumerate(arr)]
    done, st = run_loop(reqs, ex)
    _say("heterogeneous slots", st, sorted({d.slot for d in done}))
    assert st["events"] == len(reqs) and {d.slot for d in done} == {0, 1}
    for i in range(len(reqs)):
        _check(ex.results[i], ref[i], f"request {i}")
    ex.close()


def test_served_capacity_overflow_recovers(setup):
    from paper_2403_13166_amd.runtime import Caps
    from paper_2403_13166_amd.serve import Admission, GpuExecutor, Request, pinned_event, run_loop
    geo, mdl, pool = setup
    ref = _alone(geo, mdl, pool[:3], 1)
    hits = sum(e.n for e in pool[:3])
    small = Caps(hits=hits, events=3, md=2048, ls=2048, t3=2048, t5=2048, cand=1 << 16)
    _say("serve overflow: caps", small)
    ex = GpuExecutor(geo.to_blob(), mdl.to_blob(), 1, small, precision=1, use_graph=True, keep_results=True)
    pins = [pinned_event(e) for e in pool[:3]]
    reqs = [Request(i, 0.0, pool[i].n, pins[i]) for i in range(3)]
    done, st = run_loop(reqs, ex, Admission(hits, 3))
    assert st["events"] == 3
    assert ex.slots[0].caps.md > 2048
    for i in range(3):
        _check(ex.results[i], ref[i], f"overflow request {i}")
    # the slot keeps working (graph re-captured at the grown capacities)
    reqs2 = [Request(10 + i, 0.0, pool[i].n, pins[i]) for i in range(3)]
    run_loop(reqs2, ex, Admission(hits, 3))
    for i in range(3):
        _check(ex.results[10 + i], ref[i], f"after overflow request {i}")
    ex.close()


@pytest.mark.parametrize("stage", [3, 6])
def test_injected_failure_is_isolated(setup, stage):
    """A request whose build fails (failure injection before the LS stage, or
    before the scoring) fails alone: its batch mates are rebuilt one by one
    and equal their builds alone, and the slots keep serving."""
    from paper_2403_13166_amd.serve import Admission, GpuExecutor, Request, pinned_event, run_loop, slot_caps
    geo, mdl, pool = setup
    ref = _alone(geo, mdl, pool, 1)
    cap = sum(e.n for e in pool)
    _say("serve with injected failure before stage", stage)
    ex = GpuExecutor(geo.to_blob(), mdl.to_blob(), 2, slot_caps(cap, 4), precision=1, use_graph=True,
                     keep_results=True)
    ex.inject = {2: stage}
    pins = [pinned_event(e) for e in pool]
    reqs = [Request(i, 0.0 if i < 4 else 0.003, pool[i].n, pins[i]) for i in range(len(pool))]
    done, st = run_loop(reqs, ex, Admission(cap, 4))
    _say("stats", {k: v for k, v in st.items() if k != "failed"}, "failed", st["failed"])
    assert [f["idx"] for f in st["failed"]] == [2]
    assert f"stage {stage}" in st["failed"][0]["error"]
    assert sorted(d.idx for d in done) == [i for i in range(len(pool)) if i != 2]
    for i in range(len(pool)):
        if i != 2:
            _check(ex.results[i], ref[i], f"request {i} next to a failed one")
    # the slots still serve, the failed event included once injection is off
    ex.inject = {}
    reqs2 = [Request(100 + i, 0.0, pool[i].n, pins[i]) for i in range(4)]
    done2, st2 = run_loop(reqs2, ex, Admission(cap, 4))
    assert st2["failed"] == [] and st2["events"] == 4
    for i in range(4):
        _check(ex.results[100 + i], ref[i], f"after the failure, request {i}")
    ex.close()


def test_served_equals_alone_at_serving_occupancy():
    """The serving workload's occupancy (PU ~ U[50, 200]: 30 tracks and 500
    noise hits per unit) on the benchmark's slot shapes, a single-event slot
    and two 48-event slots of 4.8M hits: a burst fills a large batch while
    later arrivals go to the other slots, overlapping on the device. Every
    served event equals the event built alone."""
    from paper_2403_13166_amd.serve import GpuExecutor, Request, make_pool, pinned_event, run_loop, slot_caps
    geo, pool = make_pool(56, seed=5)
    mdl = M.make_model()
    ref = _alone(geo, mdl, pool, 1)
    caps = [slot_caps(250_000, 1), slot_caps(4_800_000, 48), slot_caps(4_800_000, 48)]
    ex = GpuExecutor(geo.to_blob(), mdl.to_blob(), 3, caps, precision=1, use_graph=True, keep_results=True)
    pins = [pinned_event(e) for e in pool]
    arr = [0.0] * 44 + [0.0005 * k for k in range(1, 13)]
    reqs = [Request(i, a, pool[i].n, pins[i]) for i, a in enumerate(arr)]
    done, st = run_loop(reqs, ex)
    _say("serving occupancy", st, "hits", [e.n for e in pool[:8]], "...", "slots used", sorted({d.slot for d in done}))
    assert st["events"] == len(reqs)
    assert st["max_batch"] >= 30 and st["max_inflight"] >= 2
    for i in range(len(reqs)):
        _check(ex.results[i], ref[i], f"request {i}")
    ex.close()
