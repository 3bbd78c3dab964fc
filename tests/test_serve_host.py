"""Host logic of the serving loop, on the CPU: admission by footprint,
continuous batching over slots, and latency accounting, driven by a simulated
executor on a virtual clock."""
from collections import deque

import numpy as np
import pytest

from paper_2403_13166_amd.serve import Admission, Request, poisson_arrivals, run_loop


class Clock:
    def __init__(self):
        self.t = 0.0

    def __call__(self):
        return self.t

    def sleep(self, dt):
        self.t += max(dt, 1e-6)


class SimExecutor:
    """A batch takes fixed + per_hit * hits seconds; slots run concurrently."""

    def __init__(self, clock, n_slots, fixed=1e-3, per_hit=1e-8):
        self.clock, self.n_slots, self.fixed, self.per_hit = clock, n_slots, fixed, per_hit
        self.launched = []          # (slot, [idx...], t)
        self.busy = set()
        self.finished = []

    def launch(self, slot, batch):
        assert slot not in self.busy, "a slot was reused while busy"
        self.busy.add(slot)
        hits = sum(r.n_hits for r in batch)
        self.launched.append((slot, [r.idx for r in batch], self.clock()))
        return {"slot": slot, "end": self.clock() + self.fixed + self.per_hit * hits, "batch": batch}

    def poll(self, h):
        return self.clock() >= h["end"]

    def finish(self, h):
        self.busy.discard(h["slot"])
        self.finished.extend(r.idx for r in h["batch"])


def _reqs(arrivals, hits):
    return [Request(i, float(a), int(n)) for i, (a, n) in enumerate(zip(arrivals, hits))]


def test_admission_fifo_and_footprint():
    q = deque(_reqs([0] * 6, [40, 30, 50, 10, 10, 100]))
    adm = Admission(hits_cap=100, events_cap=4)
    b1 = adm.take(q)
    assert [r.idx for r in b1] == [0, 1]            # 40 + 30 fit, + 50 would not
    b2 = adm.take(q)
    assert [r.idx for r in b2] == [2, 3, 4]         # 50 + 10 + 10; 100 more would not
    b3 = adm.take(q)
    assert [r.idx for r in b3] == [5]
    assert not q


def test_admission_oversized_event_goes_alone():
    q = deque(_reqs([0, 0], [500, 10]))
    adm = Admission(hits_cap=100, events_cap=8)
    assert [r.idx for r in adm.take(q)] == [0]
    assert [r.idx for r in adm.take(q)] == [1]


def test_admission_events_cap():
    q = deque(_reqs([0] * 10, [1] * 10))
    assert len(Admission(1000, 3).take(q)) == 3


def test_every_request_served_once_in_fifo_order():
    clk = Clock()
    rng = np.random.default_rng(0)
    arr = poisson_arrivals(300.0, 400, rng)
    hits = rng.integers(30_000, 120_000, size=400)
    ex = SimExecutor(clk, n_slots=3, fixed=2e-3, per_hit=2e-8)
    done, st = run_loop(_reqs(arr, hits), ex, Admission(600_000, 16), clock=clk, sleep=clk.sleep)
    assert sorted(d.idx for d in done) == list(range(400))
    admitted = [i for _, ids, _ in ex.launched for i in ids]
    assert admitted == list(range(400))             # admission preserves arrival order
    for d in done:
        assert d.arrival <= d.admitted <= d.finished
    for slot, ids, _ in ex.launched:
        assert sum(hits[i] for i in ids) <= 600_000 or len(ids) == 1
    assert st["events"] == 400


def test_light_load_runs_one_event_per_batch_with_service_latency():
    clk = Clock()
    arr = np.arange(50) * 0.1                       # 10 ev/s, service 3 ms
    ex = SimExecutor(clk, n_slots=2, fixed=3e-3, per_hit=0.0)
    done, st = run_loop(_reqs(arr, [100] * 50), ex, Admission(10_000, 16), clock=clk, sleep=clk.sleep)
    assert st["max_batch"] == 1
    lat = np.array([d.latency for d in done])
    assert np.all(lat >= 3e-3) and np.all(lat < 3e-3 + 1e-3)


def test_heavy_load_batches_grow_and_slots_overlap():
    clk = Clock()
    arr = np.zeros(200)                             # a burst: all queued at once
    ex = SimExecutor(clk, n_slots=3, fixed=5e-3, per_hit=1e-8)
    done, st = run_loop(_reqs(arr, [50_000] * 200), ex, Admission(800_000, 16), clock=clk, sleep=clk.sleep)
    assert st["max_batch"] == 16 and st["max_inflight"] == 3
    # 200 events = 13 batches on 3 slots = 5 rounds of one full batch time
    t_batch = 5e-3 + 16 * 50_000 * 1e-8
    assert st["span_s"] <= 5 * t_batch + 1e-3
    # against one event per launch on one slot: ~16x more throughput
    assert st["events_per_s"] > 10 / (5e-3 + 50_000 * 1e-8)


def test_latency_percentiles_match_definition():
    clk = Clock()
    rng = np.random.default_rng(1)
    arr = poisson_arrivals(100.0, 300, rng)
    ex = SimExecutor(clk, n_slots=2)
    done, st = run_loop(_reqs(arr, rng.integers(1000, 5000, 300)), ex, Admission(50_000, 8),
                        clock=clk, sleep=clk.sleep)
    lat = np.sort([d.latency for d in done])
    assert st["p50_ms"] == pytest.approx(np.percentile(lat, 50) * 1e3)
    assert st["p99_ms"] == pytest.approx(np.percentile(lat, 99) * 1e3)
    assert st["p99_ms"] >= st["p50_ms"]


def test_poisson_arrival_rate():
    arr = poisson_arrivals(200.0, 20000, np.random.default_rng(2))
    assert np.all(np.diff(arr) > 0)
    assert 20000 / arr[-1] == pytest.approx(200.0, rel=0.03)


def test_choose_slot_prefers_smallest_fitting():
    from paper_2403_13166_amd.serve import choose_slot
    lim = {0: (250_000, 1), 1: (4_000_000, 48), 2: (4_000_000, 48), 3: (1_000_000, 8)}.get
    assert choose_slot([0, 1, 2, 3], 1, lim) == 0
    assert choose_slot([1, 2, 3], 1, lim) == 3
    assert choose_slot([0, 1, 2, 3], 5, lim) == 3
    assert choose_slot([0, 1, 2, 3], 30, lim) == 1
    assert choose_slot([0, 3], 30, lim) == 3          # none fits: the largest free one
    assert choose_slot([0], 30, lim, busy=[1, 2]) is None   # backlog: wait for a large slot
    assert choose_slot([0], 1, lim, busy=[1, 2]) == 0


class SizedExecutor(SimExecutor):
    """Slots of different sizes; a batch costs fixed + per-event-slot padding."""

    def __init__(self, clock, limits, fixed=2e-4, per_slot=2e-5, per_hit=1e-8):
        super().__init__(clock, len(limits), fixed, per_hit)
        self.limits, self.per_slot = limits, per_slot

    def slot_limits(self, slot):
        return self.limits[slot]

    def launch(self, slot, batch):
        h = super().launch(slot, batch)
        h["end"] += self.per_slot * self.limits[slot][1]
        return h


def test_heterogeneous_slots_light_and_heavy_load():
    limits = [(250_000, 1), (4_000_000, 48), (4_000_000, 48)]
    clk = Clock()
    arr = np.arange(100) * 0.01                     # 100 ev/s: the small slot takes them all
    ex = SizedExecutor(clk, limits)
    done, st = run_loop(_reqs(arr, [100_000] * 100), ex, clock=clk, sleep=clk.sleep)
    assert sorted(d.idx for d in done) == list(range(100))
    assert {d.slot for d in done} == {0} and st["max_batch"] == 1
    clk = Clock()
    ex = SizedExecutor(clk, limits)
    done, st = run_loop(_reqs(np.zeros(300), [100_000] * 300), ex, clock=clk, sleep=clk.sleep)
    assert sorted(d.idx for d in done) == list(range(300))
    assert st["max_batch"] == 40                    # 4M hits / 100k per event
    # the backlog went to the large slots, not one event at a time to the small one
    assert sum(len(ids) for slot, ids, _ in ex.launched if slot == 0) <= 2
    for slot, ids, _ in ex.launched:
        assert len(ids) <= limits[slot][1] and len(ids) * 100_000 <= limits[slot][0] or len(ids) == 1


class FailingExecutor(SimExecutor):
    """Batches holding a request of `bad_launch` raise at launch; those
    holding one of `bad_poll` raise when polled after their service time
    (the device failed mid-build). Counts the resets of freed slots."""

    def __init__(self, clock, n_slots, bad_launch=(), bad_poll=(), **kw):
        super().__init__(clock, n_slots, **kw)
        self.bad_launch, self.bad_poll = set(bad_launch), set(bad_poll)
        self.resets = []

    def launch(self, slot, batch):
        if self.bad_launch & {r.idx for r in batch}:
            raise RuntimeError("injected launch failure")
        return super().launch(slot, batch)

    def poll(self, h):
        ready = super().poll(h)
        if ready and self.bad_poll & {r.idx for r in h["batch"]}:
            raise RuntimeError("injected device failure")
        return ready

    def reset(self, slot):
        self.busy.discard(slot)
        self.resets.append(slot)


@pytest.mark.parametrize("where", ["launch", "poll"])
def test_failed_request_is_isolated_and_its_slot_freed(where):
    clk = Clock()
    rng = np.random.default_rng(3)
    n = 120
    arr = np.concatenate([np.zeros(40), 0.05 + poisson_arrivals(400.0, n - 40, rng)])
    bad = {7, 61}
    kw = {"bad_launch": bad} if where == "launch" else {"bad_poll": bad}
    ex = FailingExecutor(clk, n_slots=2, fixed=2e-3, per_hit=1e-8, **kw)
    done, st = run_loop(_reqs(arr, [20_000] * n), ex, Admission(200_000, 8), clock=clk, sleep=clk.sleep)
    # every other request is served exactly once; the bad ones fail alone
    assert sorted(d.idx for d in done) == sorted(set(range(n)) - bad)
    assert sorted(f["idx"] for f in st["failed"]) == sorted(bad)
    assert all("injected" in f["error"] for f in st["failed"])
    # a bad request's batch mates were retried, each in a batch of its own
    # (request 7 arrives in the initial burst, so its first batch is shared)
    if where == "poll":
        for b in bad:
            first = next(ids for _, ids, _ in ex.launched if b in ids)
            assert len(first) > 1 or b != 7
            for m in set(first) - {b}:
                assert [ids for _, ids, _ in ex.launched if m in ids][-1] == [m]
            assert [ids for _, ids, _ in ex.launched if b in ids][-1] == [b]
    # every slot was freed after each failure and is idle at the end
    assert not ex.busy
    assert len(ex.resets) >= len(bad)
    assert st["events"] == n - len(bad)


def test_stream_goes_on_after_every_request_fails():
    clk = Clock()
    ex = FailingExecutor(clk, n_slots=2, bad_launch=set(range(10)))
    done, st = run_loop(_reqs(np.zeros(10), [1000] * 10), ex, Admission(100_000, 4), clock=clk, sleep=clk.sleep)
    assert done == [] and sorted(f["idx"] for f in st["failed"]) == list(range(10))
