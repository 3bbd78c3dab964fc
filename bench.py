#!/usr/bin/env python3
"""Throughput benchmark of LST object building on one MI355X.

A step is one pass of the whole hot path (hit binning, mini-doublets, line
segments, triplets, quintuplets with FP64 fits, T5-DNN scoring) over one batch
of 64 synthetic PU200-like events (per event 1500-6000 helical tracks and
25k-100k noise hits, ~105k hits on average), inputs already resident in HBM,
launched as one captured HIP graph. Prints one JSON line.

Also measured (reported beside the headline, never as `value`):
  * the plain path: one event per build call with a host synchronisation
    after each event (events/s, p50/p99 latency);
  * per-stage kernel durations from HIP events recorded on the launch stream
    inside the timed region, and the roofline of the dominant kernel;
  * per-stage windows of the eval kernels and of the whole stages (scans,
    copies and CSR fills included), with compulsory bytes per stage;
  * the plain and served paths on the same Poisson arrivals (PCIe included);
  * event-level concurrency: 1, 2, 4 and 8 builders, each replaying the
    graph of the build of its own copy of the batch on its own HIP stream
    (events/s per stream count);
  * the FP64 oracle on a bounded sample of the same events, on one thread and
    on one thread per usable host core (host CPU model stated).
"""
from __future__ import annotations

import argparse
import json
import os
import sys
import time

import numpy as np

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

METRIC = "events/s at PU200-like occupancy (served+batched vs plain); p99 latency"
HBM_PEAK_GBS = 8000.0

# HBM bytes per launch of the dominant kernel from two rocprofv3 --pmc passes
# (FETCH_SIZE, WRITE_SIZE, each scaled by the counts of a plain 512 MiB
# elementwise kernel), kept with the hash of the kernel sources they were
# taken on: a changed kernel reports null until it is measured again.
MEASURED_TRAFFIC = {
    "ls stage": {"bytes": 151.71e6, "source_sha1": "c53f11c26a87ce2e3c024529e49605c0cd37ce14"},
}
KERNEL_SOURCES = ("paper_2403_13166_amd/csrc/lst_pipeline.hip", "paper_2403_13166_amd/csrc/lst_device.h",
                  "paper_2403_13166_amd/csrc/lst_internal.h")


def measured_traffic(kernel: str):
    import hashlib
    rec = MEASURED_TRAFFIC.get(kernel)
    if rec is None:
        return None
    h = hashlib.sha1()
    for f in KERNEL_SOURCES:
        with open(os.path.join(ROOT, f), "rb") as fh:
            h.update(fh.read())
    return rec["bytes"] if h.hexdigest() == rec["source_sha1"] else None


def parse():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=20)
    ap.add_argument("--warmup", type=int, default=3)
    ap.add_argument("--events", type=int, default=64)
    ap.add_argument("--batch-seed", type=int, default=0)
    ap.add_argument("--precision", choices=("bf16", "f32"), default="bf16")
    ap.add_argument("--mode", choices=("dnn", "pre_dnn"), default="dnn")
    ap.add_argument("--no-graph", action="store_true")
    ap.add_argument("--no-autotune", action="store_true")
    ap.add_argument("--tuning", default=None,
                    help='fixed launch shapes as JSON {"bin_split", "tile_per": [5], "eval_blocks", "t3_masks"} (no autotuning)')
    ap.add_argument("--plain-events", type=int, default=64)
    ap.add_argument("--cpu-seconds", type=float, default=15.0)
    ap.add_argument("--skip-cpu-baseline", action="store_true")
    ap.add_argument("--serve-events", type=int, default=5000,
                    help="events per served stream (0: skip the serving measurement)")
    ap.add_argument("--serve-rates", default="500,100000",
                    help="Poisson arrival rates (events/s) of the served streams; the largest saturates the GPU")
    ap.add_argument("--skip-extras", action="store_true",
                    help="skip the standalone scoring, edge-classifier and pre-DNN measurements")
    ap.add_argument("--streams", default="1,2,4,8",
                    help="stream counts of the event-level concurrency scan, one batch and builder per stream "
                         "(empty: skip)")
    ap.add_argument("--copy-calibration-mb", type=int, default=0,
                    help="run one device copy of this size after the timed region (HBM counter scale)")
    return ap.parse_args()


def make_batch(n_events: int, batch_seed: int):
    from paper_2403_13166_amd.synth import events as E, geometry as G
    geo = G.make_geometry(True)
    rng = E.event_rng(2, batch_seed)
    evs = [E.make_event(geo, E.batch_event_config(rng), (2, batch_seed, e)) for e in range(n_events)]
    return geo, evs


def sized_builder(geo_blob, model_blob, d, mode, prec):
    """A builder whose capacities fit the batch d = (x, y, z, sensor, event
    offsets) on the device with 10 % headroom: one eager build (which grows
    and retries as needed), then buffers reserved for its counts. Returns the
    builder and the device counts of that build."""
    import torch
    from paper_2403_13166_amd.runtime import Builder, Caps
    b = Builder(geo_blob, model_blob, 0)
    first = b.build(*d[:4], event_offsets=d[4], mode=mode, precision=prec)
    counts = list(first.counts())
    torch.cuda.synchronize()
    c0 = b.device_counts()
    caps = Caps(hits=int(d[0].shape[0]), events=int(d[4].shape[0]) - 1, md=int(counts[0] * 1.1) + 1024,
                ls=int(counts[1] * 1.1) + 1024, t3=int(counts[2] * 1.1) + 1024, t5=int(counts[3] * 1.1) + 1024,
                cand=int(c0[5] * 1.1) + 4096)
    b.caps = None
    b.reserve(caps)
    return b, c0


def measure_streams(a, geo, host_batch, tuned, mode, prec):
    """Event-level concurrency, the analogue of the paper's throughput at 1,
    2, 4 and 8 CUDA streams (Sec. 3): k builders, each with its own context,
    workspace, HIP stream, device copy of the benchmark batch and captured
    graph of its build, all replaying together; events/s over rounds in which
    every stream replays its graph once. Every builder's counts after the
    timed rounds must equal those of its eager sizing build."""
    import torch
    from paper_2403_13166_amd import binding as B
    from paper_2403_13166_amd.synth import model as M
    ks = sorted({int(k) for k in a.streams.split(",") if k.strip()})
    if not ks:
        return None
    dev = torch.device("cuda", 0)
    T = lambda arr: torch.from_numpy(np.ascontiguousarray(arr)).to(dev)
    gblob, mblob = geo.to_blob(), M.make_model().to_blob()
    # (builder, stream, graph, counts, inputs): the inputs stay referenced
    # here while the graph that reads them exists
    units = []
    for i in range(ks[-1]):
        d = tuple(T(v) for v in host_batch)
        b, c0 = sized_builder(gblob, mblob, d, mode, prec)
        B.lst_set_tuning(b.ctx, tuned)
        st = torch.cuda.Stream(device=dev)
        g = torch.cuda.CUDAGraph()
        with torch.cuda.stream(st):
            b.launch(*d[:4], event_offsets=d[4], mode=mode, precision=prec)
            st.synchronize()
            with torch.cuda.graph(g, stream=st, capture_error_mode="relaxed"):
                b.launch(*d[:4], event_offsets=d[4], mode=mode, precision=prec)
            st.synchronize()
        units.append((b, st, g, c0, d))
        print(f"streams: builder {i} sized and captured ({b.ws_bytes / 2**30:.2f} GiB workspace)",
              file=sys.stderr, flush=True)
    rounds = max(a.steps, 20)
    rows = []
    for k in ks:
        def go(n):
            for _ in range(n):
                for b, st, g, _, _ in units[:k]:
                    with torch.cuda.stream(st):
                        g.replay()
        go(2)
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        go(rounds)
        torch.cuda.synchronize()
        wall = time.perf_counter() - t0
        rows.append({"streams": k, "events_per_s": k * a.events * rounds / wall, "ms_per_round": wall / rounds * 1e3})
        print(f"streams {k}: {rows[-1]['events_per_s']:.1f} events/s, {rows[-1]['ms_per_round']:.3f} ms per round",
              file=sys.stderr, flush=True)
    for b, st, g, c0, _ in units:
        chk = b.device_counts()
        assert chk[:4] == c0[:4] and chk[4] == 0, (chk, c0)
    out = {"builders": len(units), "events_per_batch": a.events, "rounds": rounds,
           "batch": "each builder replays its own device copy of the benchmark batch",
           "workspace_bytes_per_builder": units[0][0].ws_bytes, "rows": rows}
    torch.cuda.synchronize()
    builders = [u[0] for u in units]
    units.clear()                   # graphs and their inputs first, then the contexts
    for b in builders:
        b.close()
    return out


def stage_bytes(c, n_hits, n_ev, n_mod, n_sens):
    """Compulsory (algorithmic) HBM bytes of each stage per launch: every
    input record read once and every output record written once, at the
    record sizes of the object layouts (hits 16 B; an MD 32 B: two hit
    indices, anchor position, chord; an LS 12 B: two MD indices and its
    curvature; a T3 12 B; a T5 20 B: two T3 indices, two chi2, score), plus
    the CSR offsets (8 B per entry) a stage reads or writes. The same bytes
    are used for a stage's eval kernel and for the whole stage."""
    md, ls, t3, t5 = c[:4]
    em = n_ev * n_mod
    # features come from the T5's T3 pair, its MDs and the fit outputs, and
    # stay on chip (LDS) until the score is written
    score = (8 + 32 + 4) * t5 + 16 * t3 + 16 * md
    return {
        "bin": 16 * n_hits + 16 * n_hits + 8 * n_ev * n_sens,
        "md": 16 * n_hits + 32 * md,
        "ls": 32 * md + 12 * ls + 8 * em,
        "t3": 12 * ls + 32 * md + 8 * md + 12 * t3,
        "t5": 12 * t3 + 32 * md + 20 * t5,
        "score": score,
    }


def implementation_bytes(c):
    """Bytes the build moves beyond the compulsory ones: the LS stage's
    (A, B, rank) records (16 B, written by the eval kernel and read by the
    placement kernel) and its per-MD segment counts (4 B written, read by the
    scan); the T3 stage's candidate range of every inner LS (8 B written by
    the count kernel, read by the write kernel) and first T3 position of
    every inner LS (8 B written, read by the CSR kernel)."""
    md, ls = c[0], c[1]
    return {"ls_records": 2 * 16 * ls, "ls_counts": 2 * 4 * md, "t3_ranges": 2 * 8 * ls,
            "t3_positions": 2 * 8 * ls}


def _time_ms(fn, stream, reps=10):
    import torch
    e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
    fn()
    stream.synchronize()
    ts = []
    for _ in range(reps):
        e0.record(stream)
        fn()
        e1.record(stream)
        stream.synchronize()
        ts.append(e0.elapsed_time(e1))
    return float(np.median(ts))


def measure_extras(b, dx, dy, dz, ds, doff, stream, prec, geo, evs):
    """Track-candidate selection on the batch's objects with synthetic pixel
    seeds, standalone T5-DNN scoring of 1M feature rows (BF16 MFMA and FP32),
    the edge classifier on a 200k-node / 1M-edge LST-like graph, and the T5
    stage of the same batch in pre-DNN mode (circle-fit chi2 cut, no DNN)."""
    import torch
    from paper_2403_13166_amd import binding as B
    from paper_2403_13166_amd.runtime import EdgeClassifier, select_tcs
    from paper_2403_13166_amd.synth import events as E, gnn as SG, model as M, seeds as S
    dev = dx.device
    out = {}
    with torch.cuda.stream(stream):
        # TC selection (Table 1 steps 5-8 + duplicate removal) on this batch
        b.launch(dx, dy, dz, ds, event_offsets=doff, mode=B.LST_MODE_DNN, precision=prec)
        stream.synchronize()
        objs = b.view()
        sds = [S.make_seeds(geo, e, E.event_rng(5, i), eff=0.9, fake_frac=0.05) for i, e in enumerate(evs)]
        sp, soff = S.concat_seeds(sds)
        tsp, tsoff = torch.from_numpy(sp).to(dev), torch.from_numpy(soff).to(dev)
        res = {}
        ms = _time_ms(lambda: res.__setitem__("t", select_tcs(b, dx, dy, dz, objs, tsp, tsoff)), stream)
        c = res["t"].counts
        # the MD/LS graph of Sec. 4 on the same objects: graph building alone,
        # then graph + edge classifier + components (TCs of >= 3 MDs)
        from paper_2403_13166_amd.runtime import graph_tcs
        gclf = EdgeClassifier(SG.make_gnn_model().to_blob(), dev.index or 0)
        n_md, n_ls = objs.counts()[:2]
        gf = torch.empty((n_md, 7), dtype=torch.float32, device=dev)
        gs = torch.empty(n_ls, dtype=torch.int32, device=dev)
        gd = torch.empty(n_ls, dtype=torch.int32, device=dev)
        gob = B.LstObjects(objs.md_hits.data_ptr(), objs.ls_md.data_ptr(), None, None, None, None, None, None,
                           None, n_md, n_ls, 0, 0)
        ghits = B.LstHits(dx.data_ptr(), dy.data_ptr(), dz.data_ptr(), ds.data_ptr(), int(dx.shape[0]))
        ms_g = _time_ms(lambda: B.lst_md_graph(b.ctx, ghits, gob, gf.data_ptr(), gs.data_ptr(), gd.data_ptr(),
                                               stream.cuda_stream), stream)
        gres = {}
        ms_p = _time_ms(lambda: gres.__setitem__("r", graph_tcs(b, gclf, dx, dy, dz, ds, objs)), stream)
        out["md_ls_graph"] = {"graph_build_ms": ms_g, "graph_classify_components_ms": ms_p, "nodes": int(n_md),
                              "edges": int(n_ls), "tcs_min3": int(gres["r"].n_tc),
                              "note": "untrained classifier weights: the TC count shows the pipeline, not a physics figure"}
        gclf.close()
        out["tc_selection"] = {"ms": ms, "seeds": int(len(sp)), "t5": int(objs.counts()[3]),
                               "t3": int(objs.counts()[2]), "kept": {k: int(v) for k, v in zip(B.TC_KINDS, c[:4])},
                               "before_duplicate_removal": int(c[5]),
                               "events_per_s": len(evs) / (ms * 1e-3)}
        X = torch.from_numpy(M.make_scoring_inputs(1_000_000)).to(dev)
        for name, p_ in (("bf16_mfma", B.LST_PREC_BF16), ("f32_valu", B.LST_PREC_F32)):
            ms = _time_ms(lambda: b.score(X, precision=p_), stream)
            out[f"score_1M_{name}"] = {"ms": ms, "gb_per_s": (168 + 4) * 1e6 / (ms * 1e-3) / 1e9,
                                       "rows_per_s": 1e6 / (ms * 1e-3)}
        g = SG.make_graph()
        clf = EdgeClassifier(SG.make_gnn_model().to_blob(), dev.index or 0)
        gx, gs, gd = (torch.from_numpy(v).to(dev) for v in (g.x, g.src, g.dst))
        sc = torch.empty(g.n_edges, dtype=torch.float32, device=dev)
        ms = _time_ms(lambda: clf.score(gx, gs, gd, out=sc, asynchronous=True), stream)
        macs = g.n_nodes * (7 * 64 + 64 * 64 + 128 * 64 + 64 * 64) + g.n_edges * (
            128 * 64 + 2 * (192 * 64 + 64 * 64) + 64 * 32 + 32)
        out["edge_classifier_200k_1M"] = {"ms": ms, "tflop_per_s": 2 * macs / (ms * 1e-3) / 1e12,
                                          "edges_per_s": g.n_edges / (ms * 1e-3)}
        clf.close()
        # T5 stage in both modes on the batch (paper Table 2 analogue)
        t5 = {}
        B.lst_set_timing(b.ctx, True)
        for mname, mode in (("dnn", B.LST_MODE_DNN), ("pre_dnn", B.LST_MODE_PRE_DNN)):
            vals = []
            for _ in range(5):
                b.launch(dx, dy, dz, ds, event_offsets=doff, mode=mode, precision=prec)
                stream.synchronize()
                st_ = B.lst_stage_times(b.ctx)
                vals.append((st_["t5"], st_["score"], st_["build"]))
            v = np.median(np.array(vals), axis=0)
            t5[mname] = {"t5_ms": float(v[0]), "dnn_ms": float(v[1]), "build_ms": float(v[2])}
        B.lst_set_timing(b.ctx, False)
        out["t5_stage_by_mode"] = t5
        out["displaced"] = measure_displaced(b, dx, dy, dz, ds, doff, stream, prec, geo)
    return out


CUBE_BINS = (0.0, 1.0, 2.0, 2.5, 3.0, 3.6)


def measure_displaced(b, dx, dy, dz, ds, doff, stream, prec, geo):
    """Displaced workload (Sec. 3, muon-cube sample): 64 events of 200 muons
    from vertices uniform in a 5 cm cube, built with the default and the
    relaxed cut sets; track efficiency (muons with at least 10 hits that have
    a T5 with more than 75 % of its hits from them) per bin of transverse
    vertex radius, and the batch time. Also the time of the benchmark batch
    under the relaxed cuts (their cost on PU200-like occupancy)."""
    import torch
    from paper_2403_13166_amd import binding as B, train as TR
    from paper_2403_13166_amd.runtime import Builder
    from paper_2403_13166_amd.synth import events as E, geometry as G, model as M
    dev = dx.device
    gd = G.make_geometry(True, G.DISPLACED_PARAMS)
    cube = [E.make_event(geo, E.muon_cube_config(200), (9, 5000 + e)) for e in range(64)]
    x, y, z, s, off = E.concat_events(cube)
    T = lambda a: torch.from_numpy(np.ascontiguousarray(a)).to(dev)
    cx, cy, cz, cs, coff = T(x), T(y), T(z), T(s), T(off)
    truth = np.concatenate([np.where(e.truth >= 0, e.truth + 1000 * i, -1) for i, e in enumerate(cube)])
    rv = np.concatenate([np.hypot(e.tracks[:, 5], e.tracks[:, 6]) for e in cube])
    nh = np.concatenate([np.bincount(e.truth[e.truth >= 0], minlength=len(e.tracks)) for e in cube])
    ids = np.concatenate([np.arange(len(e.tracks)) + 1000 * i for i, e in enumerate(cube)])
    bins = np.digitize(rv, CUBE_BINS) - 1
    res = {"events": len(cube), "muons_per_event": 200, "hits": int(len(x)), "r_vertex_bins_cm": list(CUBE_BINS),
           "muons_per_bin": [int(np.count_nonzero((nh >= 10) & (bins == k))) for k in range(len(CUBE_BINS) - 1)],
           "relaxed_params": dict(G.DISPLACED_PARAMS)}
    bd = Builder(gd.to_blob(), M.make_model().to_blob(), dev.index or 0)
    with torch.cuda.stream(stream):
        for name, bb in (("default_cuts", b), ("relaxed_cuts", bd)):
            h = bb.build(cx, cy, cz, cs, event_offsets=coff, precision=prec).to_host()
            real, tid = TR.t5_truth(h.md_hits, h.t5_mds(), truth)
            found = np.isin(ids, np.unique(tid[real]))
            eff = [float(np.mean(found[(nh >= 10) & (bins == k)])) for k in range(len(CUBE_BINS) - 1)]
            ms = _time_ms(lambda: bb.launch(cx, cy, cz, cs, event_offsets=coff, precision=prec), stream, reps=5)
            res[name] = {"efficiency_by_r_vertex": eff, "t5": int(len(h.t5_t3)), "batch_ms": ms,
                         "events_per_s": len(cube) / (ms * 1e-3)}
        bd.build(dx, dy, dz, ds, event_offsets=doff, precision=prec)
        ms = _time_ms(lambda: bd.launch(dx, dy, dz, ds, event_offsets=doff, precision=prec), stream, reps=5)
        res["benchmark_batch_relaxed_cuts"] = {"batch_ms": ms, "counts": [int(v) for v in bd.device_counts()[:4]]}
    bd.close()
    return res


def measure_end_to_end(b, step, dev_hits, host_hits, counts, stream, reps):
    """The batch with its PCIe transfers: hits copied host -> device from
    pinned memory, the same build, then every object array and the T5
    scores and chi2 values copied back to pinned host memory, one batch at a
    time with a host sync per batch (no overlap between batches)."""
    import torch
    pinned = [torch.from_numpy(np.ascontiguousarray(h)).pin_memory() for h in host_hits]
    n_md, n_ls, n_t3, n_t5 = counts[:4]
    buf = b._buf
    srcs = [buf["md_hits"][:n_md], buf["ls_md"][:n_ls], buf["t3_ls"][:n_t3], buf["t5_t3"][:n_t5],
            buf["t5_score"][:n_t5], buf["t5_chi2_rphi"][:n_t5], buf["t5_chi2_rz"][:n_t5], buf["counts"]]
    outs = [torch.empty(t.shape, dtype=t.dtype, pin_memory=True) for t in srcs]
    h2d = sum(t.numel() * t.element_size() for t in pinned)
    d2h = sum(t.numel() * t.element_size() for t in srcs)
    ts = []
    with torch.cuda.stream(stream):
        for i in range(reps + 1):
            t0 = time.perf_counter()
            for d, h in zip(dev_hits, pinned):
                d.copy_(h, non_blocking=True)
            step()
            for h, d in zip(outs, srcs):
                h.copy_(d, non_blocking=True)
            stream.synchronize()
            if i:
                ts.append((time.perf_counter() - t0) * 1e3)
    got = outs[-1].tolist()[:4]
    assert got == list(counts[:4]), (got, counts[:4])
    ms = float(np.median(ts))
    return {"ms_per_batch": ms, "h2d_bytes": h2d, "d2h_bytes": d2h,
            "pcie_gb_per_s": (h2d + d2h) / (ms * 1e-3) / 1e9, "batches": reps}


def host_cpu():
    """Model name and logical CPU count of this host, and the CPUs this
    process may run on (its share of the host when the host is shared)."""
    model = "unknown"
    try:
        with open("/proc/cpuinfo") as f:
            for line in f:
                if line.startswith("model name"):
                    model = line.split(":", 1)[1].strip()
                    break
    except OSError:
        pass
    try:
        usable = len(os.sched_getaffinity(0))
    except AttributeError:
        usable = os.cpu_count() or 1
    return {"model": model, "nproc": os.cpu_count(), "usable": usable}


def cpu_baseline(geo, evs, seconds):
    """The FP64 oracle on the batch's events, in order and cycling, for a
    bounded time: once on one thread, once on one thread per usable core
    (events distributed over threads; the oracle call releases the GIL)."""
    from concurrent.futures import ThreadPoolExecutor
    from oracle import oracle as O
    from paper_2403_13166_amd.synth import model as M
    og = O.Geom(geo.to_blob())
    om = O.Model(M.make_model().to_blob())
    build = lambda ev: O.build_objects(og, om, ev.x, ev.y, ev.z, ev.sensor, mode=0)
    cpu = host_cpu()
    # at most 16 threads: the CPU share of one GPU
    nthr = max(1, min(cpu["usable"], 16))

    def leg(threads, budget):
        t0 = time.perf_counter()
        n = 0
        with ThreadPoolExecutor(threads) as pool:
            while n < 3 * len(evs) and time.perf_counter() - t0 <= budget:
                chunk = [evs[(n + k) % len(evs)] for k in range(threads)]
                list(pool.map(build, chunk))
                n += threads
        return n, time.perf_counter() - t0

    n1, dt1 = leg(1, seconds / 2)
    nn, dtn = leg(nthr, seconds / 2)
    return {"value": nn / dtn, "unit": "events/s", "cores": nthr, "kind": "oracle",
            "sample": f"{nn} builds of the {len(evs)} batch events taken in order (cycling), FP64 C oracle, "
                      f"{nthr} threads over events, {dtn:.1f} s; single thread: {n1} builds in {dt1:.1f} s",
            "single_thread_events_per_s": n1 / dt1, "host_cpu": cpu["model"], "nproc": cpu["nproc"],
            "usable_cpus": cpu["usable"]}


def main():
    a = parse()
    if a.gpus != 1:
        print(f"bench.py runs on one GPU: the library has no multi-GPU path (events shard by event "
              f"with no collectives); got --gpus {a.gpus}", file=sys.stderr)
        sys.exit(2)
    import torch
    from paper_2403_13166_amd import binding as B
    from paper_2403_13166_amd.runtime import Builder, Caps
    from paper_2403_13166_amd.synth import events as E, model as M

    prec = B.LST_PREC_BF16 if a.precision == "bf16" else B.LST_PREC_F32
    mode = B.LST_MODE_DNN if a.mode == "dnn" else B.LST_MODE_PRE_DNN
    t_gen = time.perf_counter()
    geo, evs = make_batch(a.events, a.batch_seed)
    x, y, z, s, off = E.concat_events(evs)
    t_gen = time.perf_counter() - t_gen
    dev = torch.device("cuda", 0)
    T = lambda arr: torch.from_numpy(np.ascontiguousarray(arr)).to(dev)
    dx, dy, dz, ds, doff = T(x), T(y), T(z), T(s), T(off)
    b, c0 = sized_builder(geo.to_blob(), M.make_model().to_blob(), (dx, dy, dz, ds, doff), mode, prec)
    B.lst_set_timing(b.ctx, True)

    stream = torch.cuda.Stream(device=dev)
    run = lambda: b.launch(dx, dy, dz, ds, event_offsets=doff, mode=mode, precision=prec)
    graph = None
    tuned, tune_table = B.lst_get_tuning(b.ctx), []
    with torch.cuda.stream(stream):
        for _ in range(max(1, a.warmup)):
            run()
        stream.synchronize()
        if a.tuning:
            B.lst_set_tuning(b.ctx, json.loads(a.tuning))
            tuned = B.lst_get_tuning(b.ctx)
        elif not a.no_autotune:
            # untimed: pick launch shapes for this workload on this GPU
            from paper_2403_13166_amd.autotune import autotune
            tuned, tune_table = autotune(b, run, stream.synchronize, reps=5,
                                         log=lambda m: print(m, file=sys.stderr, flush=True))
        if not a.no_graph:
            graph = torch.cuda.CUDAGraph()
            with torch.cuda.graph(graph, stream=stream, capture_error_mode="relaxed"):
                run()
            stream.synchronize()
            for _ in range(a.warmup):
                graph.replay()
            stream.synchronize()
        step = graph.replay if graph is not None else run
        # verify the replayed build against the eager sizing build
        step()
        stream.synchronize()
        chk = b.device_counts()
        assert chk[:4] == c0[:4] and chk[4] == 0, (chk, c0)

        # ---------------- timed region: K steps, one sync + stage-time read each
        stage_ms = {k: [] for k in B.STAGE_WINDOWS}
        step_ms = []
        timing_src = "graph" if graph is not None else "eager"
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        for _ in range(a.steps):
            ts = time.perf_counter()
            step()
            stream.synchronize()
            step_ms.append((time.perf_counter() - ts) * 1e3)
            if timing_src != "unavailable":
                try:
                    for k, v in B.lst_stage_times(b.ctx).items():
                        stage_ms[k].append(v)
                except B.LstError:
                    timing_src = "unavailable"
        torch.cuda.synchronize()
        t1 = time.perf_counter()
        if timing_src == "unavailable":
            # event records inside the graph gave no durations: time the same
            # build launched eagerly on the same stream instead
            timing_src = "eager-after-graph"
            stage_ms = {k: [] for k in B.STAGE_WINDOWS}
            for _ in range(a.steps):
                run()
                stream.synchronize()
                for k, v in B.lst_stage_times(b.ctx).items():
                    stage_ms[k].append(v)
    B.lst_set_timing(b.ctx, False)
    wall = t1 - t0
    value = a.events * a.steps / wall
    final = b.device_counts()

    # ---------------- plain per-event path (one build call + sync per event)
    plain_lat = [float("nan")]
    plain_rate = float("nan")
    n_plain = min(a.plain_events, a.events)
    if n_plain > 0:
        plain_lat = []
        pb = Builder(geo.to_blob(), M.make_model().to_blob(), 0)
        pcaps = Caps.for_hits(max(e.n for e in evs[:n_plain]))
        pb.reserve(pcaps)
        devs = [tuple(T(arr) for arr in (e.x, e.y, e.z, e.sensor)) for e in evs[:n_plain]]
        for ev in devs[:2]:
            pb.build(*ev, mode=mode, precision=prec)
        torch.cuda.synchronize()
        tp0 = time.perf_counter()
        for ev in devs:
            ts = time.perf_counter()
            pb.build(*ev, mode=mode, precision=prec)
            plain_lat.append((time.perf_counter() - ts) * 1e3)
        plain_rate = n_plain / (time.perf_counter() - tp0)
        pb.close()

    # ---------------- other rows of the path, each timed with HIP events on its stream
    extras = None
    if not a.skip_extras:
        e2e = measure_end_to_end(b, step, (dx, dy, dz, ds), (x, y, z, s), final, stream, 10)
        e2e["events_per_s"] = a.events / (e2e["ms_per_batch"] * 1e-3)
        extras = measure_extras(b, dx, dy, dz, ds, doff, stream, prec, geo, evs)
        extras["batched_with_pcie"] = e2e

    # ---------------- event-level concurrency: one builder, batch and graph per HIP stream
    streams = measure_streams(a, geo, (x, y, z, s, off), tuned, mode, prec) if a.streams.strip() else None

    # ---------------- served path: Poisson streams of PU-varying events with
    # continuous batching over HBM-budgeted slots (latency = arrival -> objects on host)
    served = None
    if a.serve_events > 0:
        from paper_2403_13166_amd import serve as S
        sgeo, pool = S.make_pool(32)
        slots = [(250_000, 1), (4_800_000, 48), (4_800_000, 48), (4_800_000, 48)]
        served = {"pool": "32 events, PU ~ U[50, 200], 30 tracks + 500 noise hits per unit PU",
                  "slots": slots, "budget_gib": 64, "streams": []}
        keys = ("rate", "events", "events_per_s", "p50_ms", "p99_ms", "mean_batch", "max_batch", "max_inflight")
        for rate in [float(r) for r in a.serve_rates.split(",")]:
            st = S.serve_stream(sgeo, pool, rate, a.serve_events, slots, 64 << 30, mode=mode, precision=prec)
            row = {k: st[k] for k in keys}
            # the plain path on the same arrivals: one single-event slot, one
            # eager build per event (PCIe included on both paths)
            pl = S.serve_stream(sgeo, pool, rate, a.serve_events, [(max(e.n for e in pool), 1)], 64 << 30,
                                mode=mode, precision=prec, use_graph=False)
            row["plain"] = {k: pl[k] for k in ("events_per_s", "p50_ms", "p99_ms")}
            served["streams"].append(row)
            print(f"stream at {rate:.0f} ev/s: served {st['events_per_s']:.1f} ev/s, p50 {st['p50_ms']:.2f} ms, "
                  f"p99 {st['p99_ms']:.2f} ms; plain {pl['events_per_s']:.1f} ev/s, p50 {pl['p50_ms']:.2f} ms, "
                  f"p99 {pl['p99_ms']:.2f} ms", file=sys.stderr, flush=True)

    if a.copy_calibration_mb > 0:
        # one plain elementwise kernel that reads and writes exactly this many
        # bytes: the scale of the HBM byte counters
        src = torch.ones((a.copy_calibration_mb << 20) // 4, dtype=torch.float32, device=dev)
        dst = torch.empty_like(src)
        torch.neg(src, out=dst)
        torch.cuda.synchronize()

    # ---------------- roofline of the dominant kernel
    avg = {k: float(np.mean(v)) for k, v in stage_ms.items()}
    kern = {k: avg[k] for k in ("md", "ls", "t3", "t5", "score")}
    dom = max(kern, key=kern.get)
    sb = stage_bytes(final, len(x), a.events, geo.n_modules, geo.n_sensors)
    achieved = sb[dom] / (avg[dom] * 1e-3) / 1e9
    roofline = {"bound": "hbm", "kernel": f"{dom} stage eval kernel", "achieved": achieved, "peak": HBM_PEAK_GBS,
                "unit": "GB/s", "frac": achieved / HBM_PEAK_GBS, "traffic": measured_traffic(f"{dom} stage"),
                "algorithmic_bytes_per_launch": sb[dom], "avg_launch_ms": avg[dom]}
    stage_gbs = {k: sb[k] / (avg[k] * 1e-3) / 1e9 for k in kern}
    # whole stages: count scan, eval, tile scan, copy, CSR fill (LS: eval, count scan, placement)
    whole = {"bin": avg["bin"], "md": avg["md_all"], "ls": avg["ls_all"], "t3": avg["t3_all"], "t5": avg["t5"],
             "score": avg["score"]}
    stage_whole = {k: {"ms": v, "gb_per_s": sb[k] / (v * 1e-3) / 1e9,
                       "frac_hbm": sb[k] / (v * 1e-3) / 1e9 / HBM_PEAK_GBS} for k, v in whole.items()}

    cpu = None
    if not a.skip_cpu_baseline:
        cpu = cpu_baseline(geo, evs, a.cpu_seconds)

    per_ev = [round(final[i] / a.events, 1) for i in range(4)]
    out = {
        "metric": METRIC, "value": value, "unit": "events/s", "n_gpus": 1, "steps": a.steps,
        "warmup": a.warmup, "ms_per_step": wall / a.steps * 1e3, "higher_is_better": True,
        "scaling": "weak", "vs_baseline": None, "dtype": "f32", "data": "synthetic",
        "config": {"workload": f"{a.events} PU200-like events per batch (tracks U[1500,6000], noise U[25k,100k], "
                               f"pT 0.8-50 GeV, |eta|<2.4, barrel+endcap doublet modules), one HIP-graph launch",
                   "events_per_step": a.events, "hits_per_step": int(len(x)),
                   "mode": a.mode, "dnn_precision": a.precision, "graph": graph is not None},
        "roofline": roofline,
        "cpu_baseline": cpu,
        "plain": {"events_per_s": plain_rate, "events": n_plain, "p50_ms": float(np.percentile(plain_lat, 50)),
                  "p99_ms": float(np.percentile(plain_lat, 99))},
        "batch_latency_ms": {"p50": float(np.percentile(step_ms, 50)), "p99": float(np.percentile(step_ms, 99))},
        "speedup_batched_vs_plain": value / plain_rate,
        "stage_ms": avg, "stage_gbs": stage_gbs, "stage_whole": stage_whole,
        "algorithmic_bytes": sb, "implementation_bytes": implementation_bytes(final),
        "objects_per_event": {"md": per_ev[0], "ls": per_ev[1], "t3": per_ev[2], "t5": per_ev[3]},
        "max_candidates_per_stage": int(final[5]), "t5_pre_candidates": int(final[6]),
        "served": served, "streams": streams, "extras": extras,
        "input_generation_s": t_gen, "stage_timing": timing_src,
        "tuning": tuned, "autotune": tune_table,
    }
    print(json.dumps(out), flush=True)
    b.close()


if __name__ == "__main__":
    main()
