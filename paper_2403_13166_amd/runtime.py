"""Python runtime over the C ABI: device buffers (PyTorch-ROCm tensors),
capacity management and the object-set view of the results.

PyTorch provides device memory and the stream; every step of object building
runs in the HIP library (binding.py fails loudly when it is not built).
"""
from __future__ import annotations

import math
from dataclasses import dataclass

import numpy as np
import torch

from . import binding as B


@dataclass
class Caps:
    hits: int
    events: int
    md: int
    ls: int
    t3: int
    t5: int
    cand: int

    @staticmethod
    def for_hits(n_hits: int, n_events: int = 1) -> "Caps":
        """Generous defaults from the hit count (PU200-like events give ~0.22 MD,
        0.36 LS, 0.62 T3, 0.18 T5 per hit and tens of candidates per hit)."""
        n = max(int(n_hits), 1)
        e = max(int(n_events), 1)
        return Caps(hits=n, events=e, md=n // 2 + 4096 * e, ls=n + 8192 * e, t3=2 * n + 8192 * e,
                    t5=n + 8192 * e, cand=12 * n + (1 << 20))

    def grown(self, counts) -> "Caps":
        """Capacities that hold the required counts of a failed call, with headroom.
        A stage that overflowed fed only part of its objects to the later
        stages, whose reported counts are then underestimates: those are
        scaled by the truncation ratio (bounded), and later calls grow again
        if that was not enough."""
        caps = [self.md, self.ls, self.t3, self.t5]
        out, factor = [], 1.0
        for cur, need in zip(caps, counts[:4]):
            need_eff = need * factor
            out.append(max(cur, int(math.ceil(need_eff * 1.25)) + 1024))
            if need > cur:
                factor = min(8.0, factor * need / max(cur, 1))
        cand = max(self.cand, int(math.ceil(counts[5] * min(factor, 4.0) * 1.25)) + 4096)
        return Caps(self.hits, self.events, *out, cand)

    def c(self) -> B.LstCaps:
        return B.LstCaps(self.hits, self.events, self.md, self.ls, self.t3, self.t5, self.cand)


@dataclass
class Objects:
    """Device tensors of one build (sliced to the produced counts)."""
    md_hits: torch.Tensor     # [n_md, 2] int32
    ls_md: torch.Tensor       # [n_ls, 2]
    t3_ls: torch.Tensor       # [n_t3, 2]
    t5_t3: torch.Tensor       # [n_t5, 2]
    t5_score: torch.Tensor    # [n_t5] f32
    t5_chi2_rphi: torch.Tensor
    t5_chi2_rz: torch.Tensor
    t5_feat: torch.Tensor | None
    event_offsets: torch.Tensor | None = None   # [4, n_events + 1] int64 (batched)

    def counts(self):
        return (self.md_hits.shape[0], self.ls_md.shape[0], self.t3_ls.shape[0], self.t5_t3.shape[0])

    def to_host(self) -> "HostObjects":
        f = lambda t: None if t is None else t.detach().cpu().numpy()
        return HostObjects(f(self.md_hits), f(self.ls_md), f(self.t3_ls), f(self.t5_t3), f(self.t5_score),
                           f(self.t5_chi2_rphi), f(self.t5_chi2_rz), f(self.t5_feat), f(self.event_offsets))


@dataclass
class HostObjects:
    md_hits: np.ndarray
    ls_md: np.ndarray
    t3_ls: np.ndarray
    t5_t3: np.ndarray
    t5_score: np.ndarray
    t5_chi2_rphi: np.ndarray
    t5_chi2_rz: np.ndarray
    t5_feat: np.ndarray | None
    event_offsets: np.ndarray | None = None

    def t3_mds(self) -> np.ndarray:
        if not len(self.t3_ls):
            return np.zeros((0, 3), np.int64)
        a = self.ls_md[self.t3_ls[:, 0]]
        b = self.ls_md[self.t3_ls[:, 1]]
        return np.stack([a[:, 0], a[:, 1], b[:, 1]], axis=1)

    def t5_mds(self) -> np.ndarray:
        if not len(self.t5_t3):
            return np.zeros((0, 5), np.int64)
        t3 = self.t3_mds()
        u = t3[self.t5_t3[:, 0]]
        v = t3[self.t5_t3[:, 1]]
        return np.concatenate([u, v[:, 1:]], axis=1)


def _ptr(t: torch.Tensor | None) -> int | None:
    return None if t is None else t.data_ptr()


class Builder:
    """One device context with loaded geometry and model, plus reusable buffers."""

    def __init__(self, geometry_blob: bytes, model_blob: bytes, device: int = 0):
        if not torch.cuda.is_available():
            raise RuntimeError("the LST builder needs a ROCm GPU (torch.cuda is not available)")
        self.device = torch.device("cuda", device)
        torch.cuda.set_device(self.device)
        self.ctx = B.lst_create(device)
        B.lst_load_geometry(self.ctx, geometry_blob)
        B.lst_load_model(self.ctx, model_blob)
        self.caps: Caps | None = None
        self._buf = None

    def close(self):
        if getattr(self, "ctx", None):
            B.lst_destroy(self.ctx)
            self.ctx = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass

    # -------------------------------------------------------------- buffers
    def reserve(self, caps: Caps, with_features: bool = False):
        """(Re)allocate outputs and workspace for `caps` (no-op if already large enough)."""
        if (self.caps is not None and self._buf is not None and all(
                getattr(self.caps, k) >= getattr(caps, k) for k in caps.__dataclass_fields__)
                and (self._buf["t5_feat"] is not None or not with_features)):
            return
        dev = self.device
        i32 = dict(dtype=torch.int32, device=dev)
        f32 = dict(dtype=torch.float32, device=dev)
        ws_bytes = B.lst_workspace_size(self.ctx, caps.c())
        self._buf = dict(
            md_hits=torch.empty((caps.md, 2), **i32), ls_md=torch.empty((caps.ls, 2), **i32),
            t3_ls=torch.empty((caps.t3, 2), **i32), t5_t3=torch.empty((caps.t5, 2), **i32),
            t5_score=torch.empty(caps.t5, **f32), t5_chi2_rphi=torch.empty(caps.t5, **f32),
            t5_chi2_rz=torch.empty(caps.t5, **f32),
            t5_feat=torch.empty((caps.t5, B.N_FEATURES), **f32) if with_features else None,
            counts=torch.zeros(B.LST_COUNTS_LEN, dtype=torch.int64, device=dev),
            ev_obj=torch.zeros((4, caps.events + 1), dtype=torch.int64, device=dev),
            ws=torch.empty(ws_bytes + 256, dtype=torch.uint8, device=dev),
        )
        self.ws_bytes = ws_bytes
        self.caps = caps

    def _ws_ptr(self) -> int:
        p = self._buf["ws"].data_ptr()
        return (p + 255) & ~255

    def _objects_struct(self, with_features: bool) -> B.LstObjects:
        b = self._buf
        return B.LstObjects(_ptr(b["md_hits"]), _ptr(b["ls_md"]), _ptr(b["t3_ls"]), _ptr(b["t5_t3"]),
                            _ptr(b["t5_score"]), _ptr(b["t5_chi2_rphi"]), _ptr(b["t5_chi2_rz"]),
                            _ptr(b["t5_feat"]) if with_features else None, _ptr(b["counts"]), 0, 0, 0, 0)

    def _slice(self, n, with_features, ev=None) -> Objects:
        b = self._buf
        return Objects(b["md_hits"][:n[0]], b["ls_md"][:n[1]], b["t3_ls"][:n[2]], b["t5_t3"][:n[3]],
                       b["t5_score"][:n[3]], b["t5_chi2_rphi"][:n[3]], b["t5_chi2_rz"][:n[3]],
                       b["t5_feat"][:n[3]] if with_features else None, ev)

    # ---------------------------------------------------------------- build
    def build(self, x, y, z, sensor, mode: int = B.LST_MODE_DNN, precision: int = B.LST_PREC_F32,
              score_min: float = float("nan"), with_features: bool = False, caps: Caps | None = None,
              event_offsets: torch.Tensor | None = None, max_retries: int = 6) -> Objects:
        """Build the objects of one event (or of a batch when event_offsets, a
        device int64 tensor of n_events + 1 hit offsets, is given). Grows the
        capacities and retries when the library reports LST_E_CAPACITY."""
        n = int(x.shape[0])
        n_ev = 1 if event_offsets is None else int(event_offsets.shape[0]) - 1
        caps = caps or self.caps or Caps.for_hits(n, n_ev)
        if caps.hits < n or caps.events < n_ev:
            caps = Caps.for_hits(n, n_ev)
        stream = torch.cuda.current_stream(self.device).cuda_stream
        hits = B.LstHits(_ptr(x), _ptr(y), _ptr(z), _ptr(sensor), n)
        opts = B.LstOptions(int(mode), int(precision), float(score_min), 0)
        for _ in range(max_retries + 1):
            self.reserve(caps, with_features)
            out = self._objects_struct(with_features)
            if event_offsets is None:
                st = B.lst_build_objects(self.ctx, hits, opts, self.caps.c(), out, self._ws_ptr(),
                                         self.ws_bytes, stream, check=False)
            else:
                st = B.lst_build_objects_batched(self.ctx, hits, _ptr(event_offsets), n_ev, opts,
                                                 self.caps.c(), out, _ptr(self._buf["ev_obj"]),
                                                 self._ws_ptr(), self.ws_bytes, stream, check=False)
            if st == B.LST_E_CAPACITY:
                caps = self.caps.grown(self._buf["counts"].cpu().tolist())
                continue
            B._check(self.ctx, st, "build")
            ev = None if event_offsets is None else \
                self._buf["ev_obj"].view(-1)[:4 * (n_ev + 1)].view(4, n_ev + 1)
            return self._slice((out.n_md, out.n_ls, out.n_t3, out.n_t5), with_features, ev)
        raise B.LstError(B.LST_E_CAPACITY, "capacity still exceeded after retries")

    def launch(self, x, y, z, sensor, event_offsets: torch.Tensor | None = None, mode: int = B.LST_MODE_DNN,
               precision: int = B.LST_PREC_F32, score_min: float = float("nan"),
               with_features: bool = False) -> None:
        """Enqueue one build on the current stream with the reserved capacities,
        without synchronising (LST_ASYNC): safe to capture into a HIP graph.
        Read the outcome afterwards with device_counts() / view()."""
        n = int(x.shape[0])
        n_ev = 1 if event_offsets is None else int(event_offsets.shape[0]) - 1
        if self.caps is None or self.caps.hits < n or self.caps.events < n_ev:
            raise ValueError("reserve() capacities for this input first")
        stream = torch.cuda.current_stream(self.device).cuda_stream
        hits = B.LstHits(_ptr(x), _ptr(y), _ptr(z), _ptr(sensor), n)
        opts = B.LstOptions(int(mode), int(precision), float(score_min), B.LST_ASYNC)
        out = self._objects_struct(with_features)
        if event_offsets is None:
            B.lst_build_objects(self.ctx, hits, opts, self.caps.c(), out, self._ws_ptr(), self.ws_bytes, stream)
        else:
            B.lst_build_objects_batched(self.ctx, hits, _ptr(event_offsets), n_ev, opts, self.caps.c(), out,
                                        _ptr(self._buf["ev_obj"]), self._ws_ptr(), self.ws_bytes, stream)
        self._last_n_ev = n_ev

    def device_counts(self) -> list:
        """Counts of the last launched build (synchronises): md, ls, t3, t5, err, max_cand."""
        return self._buf["counts"].cpu().tolist()

    def view(self, with_features: bool = False) -> Objects:
        """Objects of the last launched build (after device_counts() shows no overflow)."""
        c = self.device_counts()
        if c[B.LST_COUNT_ERR] or c[0] > self.caps.md or c[1] > self.caps.ls or c[2] > self.caps.t3 \
                or c[3] > self.caps.t5:
            raise B.LstError(B.LST_E_CAPACITY, f"last build overflowed or failed: counts {c}")
        n_ev = getattr(self, "_last_n_ev", 1)
        ev = self._buf["ev_obj"].view(-1)[:4 * (n_ev + 1)].view(4, n_ev + 1)
        return self._slice(c[:4], with_features, ev)

    def score(self, X: torch.Tensor, precision: int = B.LST_PREC_BF16) -> torch.Tensor:
        """T5-DNN scores of feature rows X [n, 42] (f32 or bf16, device)."""
        if X.dim() != 2 or X.shape[1] != B.N_FEATURES or not X.is_contiguous():
            raise ValueError("X must be a contiguous [n, 42] tensor")
        dt = {torch.float32: B.LST_DTYPE_F32, torch.bfloat16: B.LST_DTYPE_BF16}[X.dtype]
        out = torch.empty(X.shape[0], dtype=torch.float32, device=X.device)
        B.lst_score(self.ctx, X.data_ptr(), dt, X.shape[0], out.data_ptr(), precision,
                    torch.cuda.current_stream(X.device).cuda_stream)
        return out


class EdgeClassifier:
    """Edge scores of an LST object graph (own device context; see lst_gnn_score)."""

    def __init__(self, gnn_blob: bytes, device: int = 0):
        if not torch.cuda.is_available():
            raise RuntimeError("the edge classifier needs a ROCm GPU (torch.cuda is not available)")
        self.device = torch.device("cuda", device)
        torch.cuda.set_device(self.device)
        self.ctx = B.lst_create(device)
        B.lst_load_gnn(self.ctx, gnn_blob)
        self._ws = None
        self._ws_bytes = 0

    def close(self):
        if getattr(self, "ctx", None):
            B.lst_destroy(self.ctx)
            self.ctx = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass

    def reserve(self, n_nodes: int, n_edges: int):
        need = B.lst_gnn_workspace_size(self.ctx, n_nodes, n_edges)
        if self._ws is None or need > self._ws_bytes:
            self._ws = torch.empty(need + 256, dtype=torch.uint8, device=self.device)
            self._ws_bytes = need

    def score(self, x: torch.Tensor, src: torch.Tensor, dst: torch.Tensor, out: torch.Tensor | None = None,
              asynchronous: bool = False) -> torch.Tensor:
        """x [N, 7] f32, src/dst [E] int32 with dst sorted; returns scores [E] f32."""
        if x.dim() != 2 or x.shape[1] != 7 or x.dtype != torch.float32 or not x.is_contiguous():
            raise ValueError("x must be a contiguous [N, 7] float32 tensor")
        for t in (src, dst):
            if t.dtype != torch.int32 or not t.is_contiguous() or t.shape != src.shape:
                raise ValueError("src and dst must be contiguous int32 tensors of one length")
        n, e = int(x.shape[0]), int(src.shape[0])
        self.reserve(n, e)
        if out is None:
            out = torch.empty(e, dtype=torch.float32, device=x.device)
        ws = (self._ws.data_ptr() + 255) & ~255
        B.lst_gnn_score(self.ctx, x.data_ptr(), n, src.data_ptr(), dst.data_ptr(), e, out.data_ptr(), ws,
                        self._ws_bytes, B.LST_ASYNC if asynchronous else 0,
                        torch.cuda.current_stream(x.device).cuda_stream)
        return out


def to_device(ev, device) -> tuple:
    """Event arrays (numpy) -> device tensors (x, y, z, sensor)."""
    d = torch.device(device)
    return tuple(torch.from_numpy(np.ascontiguousarray(a)).to(d) for a in (ev.x, ev.y, ev.z, ev.sensor))


# default options of track-candidate selection (object widths match the
# resolution of the first-to-last anchor helix estimate)
TC_OPTIONS = dict(chi2_max=20.0, sigma_kappa_abs=5e-6, sigma_kappa_rel=0.05, sigma_phi0=2e-3, sigma_cot=5e-3,
                  sigma_z0=0.3)


@dataclass
class Tcs:
    kind: torch.Tensor        # [n] int32: 0 pT5, 1 T5, 2 pT3, 3 pLS
    seed: torch.Tensor        # [n] int32 seed index or -1
    obj: torch.Tensor         # [n] int32 T5 / T3 index or -1
    counts: list              # kept per kind (4), kept, before duplicate removal


def select_tcs(builder: Builder, x, y, z, objects: Objects, seeds: torch.Tensor, seed_offsets: torch.Tensor,
               options: dict | None = None) -> Tcs:
    """Track candidates of a completed build (lst_select_tcs): seeds [n, 8]
    float32 and seed_offsets [n_events + 1] int64 on the device."""
    opt = dict(TC_OPTIONS, **(options or {}))
    dev = builder.device
    n_ev = int(seed_offsets.shape[0]) - 1
    if seeds.dtype != torch.float32 or seeds.dim() != 2 or seeds.shape[1] != 8 or not seeds.is_contiguous():
        raise ValueError("seeds must be a contiguous float32 [n, 8] tensor")
    n_md, n_ls, n_t3, n_t5 = objects.counts()
    ob = B.LstObjects(_ptr(objects.md_hits), _ptr(objects.ls_md), _ptr(objects.t3_ls), _ptr(objects.t5_t3),
                      _ptr(objects.t5_score), _ptr(objects.t5_chi2_rphi), _ptr(objects.t5_chi2_rz), None, None,
                      n_md, n_ls, n_t3, n_t5)
    ws_bytes = B.lst_tc_workspace_size(builder.ctx, ob, seeds.shape[0], n_ev)
    ws = torch.empty(ws_bytes + 256, dtype=torch.uint8, device=dev)
    cap = n_t5 + n_t3 + seeds.shape[0] + 1
    kind = torch.empty(cap, dtype=torch.int32, device=dev)
    seed = torch.empty(cap, dtype=torch.int32, device=dev)
    obj = torch.empty(cap, dtype=torch.int32, device=dev)
    counts = torch.zeros(B.TC_COUNTS_LEN, dtype=torch.int64, device=dev)
    out = B.LstTcs(kind.data_ptr(), seed.data_ptr(), obj.data_ptr(), counts.data_ptr(), cap, 0)
    hits = B.LstHits(_ptr(x), _ptr(y), _ptr(z), None, int(x.shape[0]))
    sd = B.LstSeeds(seeds.data_ptr(), seed_offsets.data_ptr(), int(seeds.shape[0]))
    ev = objects.event_offsets
    if n_ev > 1 and ev is None:
        raise ValueError("several events need the batched build's event offsets")
    B.lst_select_tcs(builder.ctx, hits, ob, _ptr(ev.contiguous()) if ev is not None else None, n_ev, sd,
                     B.LstTcOptions(*(opt[k] for k in TC_OPTIONS)), out, (ws.data_ptr() + 255) & ~255, ws_bytes,
                     torch.cuda.current_stream(dev).cuda_stream)
    n = int(out.n)
    return Tcs(kind[:n], seed[:n], obj[:n], counts.cpu().tolist()[:6])


@dataclass
class GraphTcs:
    features: torch.Tensor    # [n_md, 7] float32 node features
    src: torch.Tensor         # [n_ls] int32 edge sources (outer MD)
    dst: torch.Tensor         # [n_ls] int32 edge targets (inner MD, ascending)
    scores: torch.Tensor      # [n_ls] float32 edge scores
    labels: torch.Tensor      # [n_md] int32 component label (smallest MD index)
    n_tc: int                 # components with at least min_mds MDs


def graph_tcs(builder: Builder, classifier: "EdgeClassifier", x, y, z, sensor, objects: Objects,
              threshold: float = 0.5, min_mds: int = 3) -> GraphTcs:
    """Sec. 4's pipeline on a completed build: the MD/LS graph (lst_md_graph),
    edge scores (lst_gnn_score) and track candidates as components of the
    kept edges (lst_graph_components)."""
    dev = builder.device
    n_md, n_ls = objects.counts()[:2]
    feat = torch.empty((n_md, 7), dtype=torch.float32, device=dev)
    src = torch.empty(n_ls, dtype=torch.int32, device=dev)
    dst = torch.empty(n_ls, dtype=torch.int32, device=dev)
    ob = B.LstObjects(_ptr(objects.md_hits), _ptr(objects.ls_md), None, None, None, None, None, None, None,
                      n_md, n_ls, 0, 0)
    hits = B.LstHits(_ptr(x), _ptr(y), _ptr(z), _ptr(sensor), int(x.shape[0]))
    stream = torch.cuda.current_stream(dev).cuda_stream
    B.lst_md_graph(builder.ctx, hits, ob, feat.data_ptr(), src.data_ptr(), dst.data_ptr(), stream)
    scores = classifier.score(feat, src, dst)
    labels = torch.empty(n_md, dtype=torch.int32, device=dev)
    n_tc = torch.zeros(1, dtype=torch.int64, device=dev)
    ws_bytes = B.lst_graph_components_workspace_size(builder.ctx, n_md)
    ws = torch.empty(ws_bytes + 256, dtype=torch.uint8, device=dev)
    B.lst_graph_components(builder.ctx, n_md, src.data_ptr(), dst.data_ptr(), scores.data_ptr(), n_ls, threshold,
                           min_mds, labels.data_ptr(), n_tc.data_ptr(), (ws.data_ptr() + 255) & ~255, ws_bytes, stream)
    return GraphTcs(feat, src, dst, scores, labels, int(n_tc.item()))
