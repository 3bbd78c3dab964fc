"""Serving loop: events of uneven occupancy arrive over time and are built with
continuous batching on one GPU.

Structure (the paper processes events concurrently on several streams,
Sec. 3; this loop is the serving form of that):

  * A *slot* is one device context with its own stream, device-resident input
    buffers, object buffers, workspace and pinned host buffers, sized once for
    `hits_cap` hits and `events_cap` events. The slot count follows from an
    HBM budget: every slot's bytes are known before the first request.
  * Admission is FIFO by footprint: when a slot is free, queued events are
    taken in arrival order while their hits fit the slot (an event larger
    than a slot is admitted alone and the slot grows).
  * A batch on a slot is: asynchronous H2D copies of the events' hits into the
    slot, one batched build (a replay of the slot's captured HIP graph when
    enabled), D2H of the counts and per-event offsets, then D2H of the
    objects. Slots run on separate streams, so batches admitted while others
    are on the GPU overlap with them on the device.
  * A request is finished when its objects are in host memory; latency is
    finish - arrival.
  * A batch whose launch, completion or read-back raises is isolated: its
    slot is freed at once and, if it held several requests, each is run
    again alone ahead of the queue; a request that fails alone is reported
    failed and the stream goes on.

The scheduler (`run_loop`) is host logic that talks to an executor through
launch / poll / finish, so it is tested on the CPU with a simulated executor
and clock; `GpuExecutor` is the device implementation.
"""
from __future__ import annotations

import ctypes
import time
from collections import deque
from dataclasses import asdict, dataclass

import numpy as np


@dataclass
class Request:
    idx: int
    arrival: float        # seconds from the start of the stream
    n_hits: int
    payload: object = None


@dataclass
class Done:
    idx: int
    arrival: float
    admitted: float
    finished: float
    batch: int
    slot: int

    @property
    def latency(self) -> float:
        return self.finished - self.arrival


@dataclass
class Failed:
    idx: int
    arrival: float
    failed: float
    error: str


class Admission:
    """FIFO admission of queued requests into one slot by hit footprint."""

    def __init__(self, hits_cap: int, events_cap: int):
        if hits_cap <= 0 or events_cap <= 0:
            raise ValueError("slot capacities must be positive")
        self.hits_cap = int(hits_cap)
        self.events_cap = int(events_cap)

    def take(self, queue: deque) -> list:
        batch, hits = [], 0
        while queue and len(batch) < self.events_cap:
            r = queue[0]
            if batch and hits + r.n_hits > self.hits_cap:
                break
            batch.append(queue.popleft())
            hits += r.n_hits
        return batch


def choose_slot(free: list, n_queued: int, limits, busy=()):
    """Slot for the next batch among the free ones: the smallest slot (by
    events) that takes every queued request; if none does, the largest free
    slot, unless a larger slot is busy, in which case None (wait for it).
    Small slots serve light load with little padding; large ones absorb
    bursts, and a backlog is not fed one event at a time to a small slot."""
    fit = [s for s in free if limits(s)[1] >= n_queued]
    if fit:
        return min(fit, key=lambda s: (limits(s)[1], limits(s)[0], s))
    best = max(free, key=lambda s: (limits(s)[1], limits(s)[0], -s))
    if any(limits(b)[1] > limits(best)[1] for b in busy):
        return None
    return best


def run_loop(requests, executor, admission: Admission | None = None, clock=time.perf_counter, sleep=time.sleep,
             idle_poll: float = 50e-6):
    """Serve `requests` (sorted by arrival) on executor.n_slots slots. With
    `admission` every slot admits by those limits; without, each slot by its
    own (executor.slot_limits) and choose_slot picks the slot.
    Returns (done list in finishing order, stats dict); stats["failed"] lists
    the requests that failed alone (Failed records as dicts)."""
    reqs = sorted(requests, key=lambda r: (r.arrival, r.idx))
    nxt = 0
    queue = deque()
    solo = deque()                        # requests of failed batches, each to run alone
    free = list(range(executor.n_slots))[::-1]
    inflight = {}                         # slot -> (handle, batch, admitted, batch id)
    done, batches, failed = [], [], []
    n_batch = 0
    max_inflight = 0
    t0 = clock()

    def batch_failed(slot, batch, err):
        reset = getattr(executor, "reset", None)
        if reset is not None:
            reset(slot)
        free.append(slot)
        if len(batch) > 1:
            solo.extend(batch)
        else:
            failed.append(Failed(batch[0].idx, batch[0].arrival, clock() - t0, repr(err)))

    while nxt < len(reqs) or queue or solo or inflight:
        now = clock() - t0
        while nxt < len(reqs) and reqs[nxt].arrival <= now:
            queue.append(reqs[nxt])
            nxt += 1
        progressed = False
        for slot in list(inflight):
            h, batch, t_adm, bid = inflight[slot]
            try:
                ready = executor.poll(h)
                if ready:
                    t_fin = clock() - t0
                    executor.finish(h)
            except Exception as err:          # noqa: BLE001 - isolate any failure of the batch
                del inflight[slot]
                batch_failed(slot, batch, err)
                progressed = True
                continue
            if ready:
                for r in batch:
                    done.append(Done(r.idx, r.arrival, t_adm, t_fin, bid, slot))
                del inflight[slot]
                free.append(slot)
                progressed = True
        while free and (queue or solo):
            if solo:
                slot = free.pop() if admission is not None else choose_slot(free, 1, executor.slot_limits)
                if admission is None:
                    free.remove(slot)
                batch = [solo.popleft()]
            elif admission is not None:
                slot = free.pop()
                batch = admission.take(queue)
            else:
                slot = choose_slot(free, len(queue), executor.slot_limits, list(inflight))
                if slot is None:
                    break
                free.remove(slot)
                batch = Admission(*executor.slot_limits(slot)).take(queue)
            t_adm = clock() - t0
            progressed = True
            try:
                h = executor.launch(slot, batch)
            except Exception as err:          # noqa: BLE001
                batch_failed(slot, batch, err)
                continue
            inflight[slot] = (h, batch, t_adm, n_batch)
            batches.append(len(batch))
            n_batch += 1
            max_inflight = max(max_inflight, len(inflight))
        if not progressed:
            wait = idle_poll
            if not inflight and not queue and nxt < len(reqs):
                wait = max(0.0, min(reqs[nxt].arrival - now, 1e-3))
            sleep(wait)
    span = (max(d.finished for d in done) - min(d.arrival for d in done)) if done else 0.0
    lat = np.array([d.latency for d in done]) if done else np.zeros(1)
    stats = {"events": len(done), "batches": n_batch, "span_s": span,
             "events_per_s": len(done) / span if span > 0 else float("nan"),
             "p50_ms": float(np.percentile(lat, 50) * 1e3), "p99_ms": float(np.percentile(lat, 99) * 1e3),
             "mean_batch": float(np.mean(batches)) if batches else 0.0,
             "max_batch": int(max(batches)) if batches else 0, "max_inflight": max_inflight,
             "failed": [asdict(f) for f in failed]}
    return done, stats


def poisson_arrivals(rate: float, n: int, rng: np.random.Generator) -> np.ndarray:
    """Arrival times (s) of a Poisson stream of `rate` events/s."""
    return np.cumsum(rng.exponential(1.0 / rate, size=n))


# ------------------------------------------------------------------ device side

_HIP = None


def _hip():
    """The HIP runtime this process already uses (the one torch loaded), for
    2-D asynchronous copies: one call places an event's four hit arrays."""
    global _HIP
    if _HIP is None:
        path = "libamdhip64.so.7"
        with open("/proc/self/maps") as fh:
            for line in fh:
                if "libamdhip64" in line:
                    path = line.split()[-1]
                    break
        L = ctypes.CDLL(path)
        L.hipMemcpy2DAsync.argtypes = [ctypes.c_void_p, ctypes.c_size_t, ctypes.c_void_p, ctypes.c_size_t,
                                       ctypes.c_size_t, ctypes.c_size_t, ctypes.c_int, ctypes.c_void_p]
        L.hipMemcpy2DAsync.restype = ctypes.c_int
        _HIP = L
    return _HIP


_HIP_H2D = 1

class _Slot:
    def __init__(self, geometry_blob, model_blob, caps, mode, precision, device, use_graph):
        import torch
        from .runtime import Builder
        self.torch = torch
        self.dev = torch.device("cuda", device)
        self.b = Builder(geometry_blob, model_blob, device)
        self.mode, self.precision, self.use_graph = mode, precision, use_graph
        self.stream = torch.cuda.Stream(device=self.dev)
        self._alloc(caps)

    def _alloc(self, caps):
        """Device inputs, object buffers and workspace, and host buffers, for `caps`."""
        torch = self.torch
        self.caps = caps
        self.b.caps = None
        self.b.reserve(caps)
        # hit arrays of the batch as the rows of one [4, hits] buffer (x, y, z,
        # sensor bits), so one 2-D copy places an event's four arrays
        self.dhits = torch.zeros((4, caps.hits), dtype=torch.float32, device=self.dev)
        self.dx, self.dy, self.dz = self.dhits[0], self.dhits[1], self.dhits[2]
        self.ds = self.dhits[3].view(torch.int32)
        self.doff = torch.zeros(caps.events + 1, dtype=torch.int64, device=self.dev)
        self.h_off = torch.zeros(caps.events + 1, dtype=torch.int64, pin_memory=True)
        self.h_counts = torch.zeros(8, dtype=torch.int64, pin_memory=True)
        self.h_evobj = torch.zeros((4, caps.events + 1), dtype=torch.int64, pin_memory=True)
        self._alloc_host_objects(caps)
        self.graph = None
        torch.cuda.synchronize(self.dev)      # the fills above ran on another stream

    def _alloc_host_objects(self, caps):
        torch = self.torch
        pin = dict(pin_memory=True)
        self.h_obj = {
            "md_hits": torch.zeros((caps.md, 2), dtype=torch.int32, **pin),
            "ls_md": torch.zeros((caps.ls, 2), dtype=torch.int32, **pin),
            "t3_ls": torch.zeros((caps.t3, 2), dtype=torch.int32, **pin),
            "t5_t3": torch.zeros((caps.t5, 2), dtype=torch.int32, **pin),
            "t5_score": torch.zeros(caps.t5, dtype=torch.float32, **pin),
            "t5_chi2_rphi": torch.zeros(caps.t5, dtype=torch.float32, **pin),
            "t5_chi2_rz": torch.zeros(caps.t5, dtype=torch.float32, **pin),
        }

    def nbytes(self) -> int:
        """Device bytes held by this slot (inputs, outputs, workspace)."""
        buf = self.b._buf
        dev = sum(t.numel() * t.element_size() for t in buf.values() if t is not None)
        dev += sum(t.numel() * t.element_size() for t in (self.dhits, self.doff))
        return int(dev)

    def _launch_build(self):
        # every batch runs with events_cap events: unused events are empty
        self.b.launch(self.dx, self.dy, self.dz, self.ds, event_offsets=self.doff, mode=self.mode,
                      precision=self.precision)

    def _capture(self):
        torch = self.torch
        with torch.cuda.stream(self.stream):
            self._launch_build()          # warm-up outside capture
            self.stream.synchronize()
            g = torch.cuda.CUDAGraph()
            with torch.cuda.graph(g, stream=self.stream, capture_error_mode="relaxed"):
                self._launch_build()
        self.stream.synchronize()
        self.graph = g

    def launch(self, batch, fail_stage: int = 0):
        """Enqueue the batch; with fail_stage > 0 the build is run eagerly with
        failure injection before that stage and raises."""
        torch = self.torch
        hits = sum(r.n_hits for r in batch)
        if hits > self.caps.hits or len(batch) > self.caps.events:
            from .runtime import Caps
            need = Caps.for_hits(max(hits, self.caps.hits), max(len(batch), self.caps.events))
            self.stream.synchronize()
            self._alloc(need)
        if self.use_graph and self.graph is None:
            self._capture()
        off = 0
        ho = self.h_off.numpy()
        ho[0] = 0
        hip = _hip()
        base = self.dhits.data_ptr()
        pitch = self.caps.hits * 4
        sp = self.stream.cuda_stream
        with torch.cuda.stream(self.stream):
            for i, r in enumerate(batch):
                n = r.n_hits
                if n:
                    err = hip.hipMemcpy2DAsync(base + 4 * off, pitch, r.payload.data_ptr(), 4 * n, 4 * n, 4,
                                               _HIP_H2D, sp)
                    if err != 0:
                        raise RuntimeError(f"hipMemcpy2DAsync failed ({err})")
                off += n
                ho[i + 1] = off
            ho[len(batch) + 1:] = off
            self.doff.copy_(self.h_off, non_blocking=True)
            if fail_stage:
                from . import binding as B
                B.lst_set_fail_stage(self.b.ctx, fail_stage)
                try:
                    self._launch_build()
                finally:
                    B.lst_set_fail_stage(self.b.ctx, 0)
            elif self.graph is not None:
                self.graph.replay()
            else:
                self._launch_build()
            buf = self.b._buf
            self.h_counts.copy_(buf["counts"], non_blocking=True)
            ne = self.caps.events + 1
            self.h_evobj.view(-1).copy_(buf["ev_obj"].view(-1)[:4 * ne], non_blocking=True)
            ev = torch.cuda.Event()
            ev.record(self.stream)
        return {"state": 0, "ev": ev, "batch": batch}

    def _overflowed(self, c) -> bool:
        k = self.caps
        return bool(c[4]) or c[0] > k.md or c[1] > k.ls or c[2] > k.t3 or c[3] > k.t5 or c[5] > k.cand

    def _recover(self):
        """The batch exceeded a capacity: rebuild it eagerly with growing
        capacities (the builder re-allocates its buffers, so the slot's graph
        is dropped and re-captured at the next launch), then size the host
        buffers to match."""
        torch = self.torch
        with torch.cuda.stream(self.stream):
            self.b.build(self.dx, self.dy, self.dz, self.ds, event_offsets=self.doff, mode=self.mode,
                         precision=self.precision, caps=self.caps)
        self.stream.synchronize()
        self.graph = None
        if self.b.caps != self.caps:
            self.caps = self.b.caps
            self._alloc_host_objects(self.caps)
        buf = self.b._buf
        self.h_counts.copy_(buf["counts"])
        ne = self.caps.events + 1
        self.h_evobj.view(-1).copy_(buf["ev_obj"].view(-1)[:4 * ne])

    def reset(self):
        """After a failed batch: wait for the slot's stream to drain."""
        self.stream.synchronize()

    def poll(self, h) -> bool:
        torch = self.torch
        if h["state"] == 0:
            if not h["ev"].query():
                return False
            c = self.h_counts.tolist()
            if self._overflowed(c):
                self._recover()
                c = self.h_counts.tolist()
            h["counts"] = c
            buf = self.b._buf
            n = {"md_hits": c[0], "ls_md": c[1], "t3_ls": c[2], "t5_t3": c[3], "t5_score": c[3],
                 "t5_chi2_rphi": c[3], "t5_chi2_rz": c[3]}
            with torch.cuda.stream(self.stream):
                for k, m in n.items():
                    if m:
                        self.h_obj[k][:m].copy_(buf[k][:m], non_blocking=True)
                ev = torch.cuda.Event()
                ev.record(self.stream)
            h["ev"] = ev
            h["state"] = 1
            return False
        return h["ev"].query()

    def results(self, h) -> list:
        """Per-request objects with event-local indices (host numpy copies)."""
        ho = self.h_off.numpy()
        eo = self.h_evobj.numpy()
        o = {k: v.numpy() for k, v in self.h_obj.items()}
        out = []
        for i, r in enumerate(h["batch"]):
            md = slice(eo[0, i], eo[0, i + 1])
            ls = slice(eo[1, i], eo[1, i + 1])
            t3 = slice(eo[2, i], eo[2, i + 1])
            t5 = slice(eo[3, i], eo[3, i + 1])
            out.append({
                "md_hits": o["md_hits"][md] - ho[i], "ls_md": o["ls_md"][ls] - eo[0, i],
                "t3_ls": o["t3_ls"][t3] - eo[1, i], "t5_t3": o["t5_t3"][t5] - eo[2, i],
                "t5_score": o["t5_score"][t5].copy(), "t5_chi2_rphi": o["t5_chi2_rphi"][t5].copy(),
                "t5_chi2_rz": o["t5_chi2_rz"][t5].copy()})
        return out


class GpuExecutor:
    """Slots on one GPU; `keep_results` stores every request's objects
    (event-local indices) in `self.results[idx]`. `inject` maps request ids
    to a pipeline stage (1..6): a batch holding such a request is built with
    the library's failure injection before that stage, so it fails."""

    def __init__(self, geometry_blob: bytes, model_blob: bytes, n_slots: int, caps, mode: int = 0,
                 precision: int = 1, device: int = 0, use_graph: bool = True, keep_results: bool = False):
        """caps: one Caps for every slot, or a list of n_slots Caps (slots of different sizes)."""
        per = list(caps) if isinstance(caps, (list, tuple)) else [caps] * n_slots
        if len(per) != n_slots:
            raise ValueError("one Caps per slot")
        self.slots = [_Slot(geometry_blob, model_blob, c, mode, precision, device, use_graph) for c in per]
        self.n_slots = n_slots
        self.keep_results = keep_results
        self.results = {}
        self.inject = {}

    def slot_bytes(self) -> int:
        return max(s.nbytes() for s in self.slots)

    def total_bytes(self) -> int:
        return sum(s.nbytes() for s in self.slots)

    def slot_limits(self, slot: int):
        """(hits, events) one batch on `slot` may hold."""
        c = self.slots[slot].caps
        return c.hits, c.events

    def warm(self, request):
        """Run one request on every slot (capture the graphs, page memory in)."""
        for slot in range(self.n_slots):
            h = self.launch(slot, [request])
            while not self.poll(h):
                pass
            self.finish(h)

    def launch(self, slot: int, batch):
        stage = max((self.inject.get(r.idx, 0) for r in batch), default=0)
        h = self.slots[slot].launch(batch, stage)
        h["slot"] = slot
        return h

    def reset(self, slot: int):
        self.slots[slot].reset()

    def poll(self, h) -> bool:
        return self.slots[h["slot"]].poll(h)

    def finish(self, h):
        if self.keep_results:
            for r, res in zip(h["batch"], self.slots[h["slot"]].results(h)):
                self.results[r.idx] = res

    def close(self):
        for s in self.slots:
            s.b.close()


def slot_caps(hits_cap: int, events_cap: int):
    from .runtime import Caps
    return Caps.for_hits(hits_cap, events_cap)


def pinned_event(ev):
    """An event's hits in pinned host memory as one [4, n] float32 block (x, y,
    z, sensor ids as bits): the source of one asynchronous 2-D copy."""
    import torch
    t = torch.empty((4, ev.n), dtype=torch.float32, pin_memory=True)
    a = t.numpy()
    a[0], a[1], a[2] = ev.x, ev.y, ev.z
    a[3] = np.ascontiguousarray(ev.sensor, dtype=np.int32).view(np.float32)
    return t


def make_pool(n: int, seed: int = 0):
    """Serving workload: n events, pile-up PU ~ U[50, 200] (30 tracks and 500
    noise hits per unit), full geometry."""
    from .synth import events as E, geometry as G
    geo = G.make_geometry(True)
    rng = E.event_rng(4, seed)
    pus = rng.uniform(50, 200, size=n)
    return geo, [E.make_event(geo, E.pileup_event_config(float(pu)), (4, seed, i)) for i, pu in enumerate(pus)]


def serve_stream(geo, pool, rate: float, n_events: int, slots, budget_bytes: int, mode: int = 0,
                 precision: int = 1, seed: int = 0, use_graph: bool = True, executor=None):
    """One Poisson stream over events drawn cyclically from `pool`. `slots` is a
    list of (hits_cap, events_cap), one per slot. Returns stats."""
    from .synth import model as M
    own = executor is None
    if own:
        executor = GpuExecutor(geo.to_blob(), M.make_model().to_blob(), len(slots),
                               [slot_caps(h, e) for h, e in slots], mode, precision, use_graph=use_graph)
    used = executor.total_bytes()
    if used > budget_bytes:
        raise ValueError(f"{executor.n_slots} slots need {used} B, over the HBM budget {budget_bytes} B")
    pins = [pinned_event(e) for e in pool]
    rng = np.random.default_rng([4, int(rate), seed])
    arr = poisson_arrivals(rate, n_events, rng)
    reqs = [Request(i, float(arr[i]), pool[i % len(pool)].n, pins[i % len(pool)]) for i in range(n_events)]
    executor.warm(Request(-1, 0.0, pool[0].n, pins[0]))
    done, stats = run_loop(reqs, executor)
    stats.update({"rate": rate, "slots": [list(executor.slot_limits(s)) for s in range(executor.n_slots)],
                  "slot_bytes": [s.nbytes() for s in executor.slots], "budget_bytes": budget_bytes})
    if own:
        executor.close()
    return stats


def main():
    import argparse
    import json
    ap = argparse.ArgumentParser(description="Poisson-stream serving of PU-varying events")
    ap.add_argument("--rates", default="50,100,200,300,500")
    ap.add_argument("--events", type=int, default=2000)
    ap.add_argument("--pool", type=int, default=48)
    ap.add_argument("--slots", default="250000x1,4800000x48,4800000x48,4800000x48",
                    help="comma-separated HITSxEVENTS capacities, one per slot")
    ap.add_argument("--budget-gib", type=float, default=64.0)
    ap.add_argument("--plain", action="store_true", help="also serve each stream one event at a time")
    a = ap.parse_args()
    geo, pool = make_pool(a.pool)
    budget = int(a.budget_gib * (1 << 30))
    slots = [tuple(int(v) for v in c.split("x")) for c in a.slots.split(",")]
    for rate in [float(r) for r in a.rates.split(",")]:
        s = serve_stream(geo, pool, rate, a.events, slots, budget)
        s["path"] = "served"
        print(json.dumps(s), flush=True)
        if a.plain:
            p = serve_stream(geo, pool, rate, a.events, [(max(e.n for e in pool), 1)], budget, use_graph=False)
            p["path"] = "plain"
            print(json.dumps(p), flush=True)


if __name__ == "__main__":
    main()
