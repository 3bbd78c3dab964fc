"""Seeded edge-classifier weights and synthetic LST-like graphs.

The paper (Sec. 4) names a graph neural network on LST objects as the next
step (nodes are lower-level objects, edges the higher-level objects built
from pairs of them) without fixing an architecture. The model here is an
interaction network:

  h0 = relu(Wb relu(Wa x + ba) + bb)                          node encoder 7 -> 64 -> 64
  e0 = relu(Wc [h0_src, h0_dst] + bc)                          edge init 128 -> 64
  step s = 0, 1 (own weights per step):
    e_{s+1} = e_s + We2 relu(We1 [h_s_src, h_s_dst, e_s] + be1) + be2     192 -> 64 -> 64
    m_v     = sum of e_{s+1} over the edges entering v
    h_{s+1} = h_s + Wn2 relu(Wn1 [h_s, m] + bn1) + bn2                    128 -> 64 -> 64
  score = sigmoid(wh2 . relu(Wh1 e_2 + bh1) + bh2)            edge head 64 -> 32 -> 1

Weights are Xavier-uniform draws with zero biases (no trained weights exist).

Blob v1 (little endian)::

    char[4] "LSTE", u32 version 1, u32 n_in 7, u32 hidden 64, u32 head 32, u32 steps 2
    then f32 arrays in the order of LAYERS below, each weight [out][in] then its bias
"""
from __future__ import annotations

import struct
from dataclasses import dataclass, field

import numpy as np

from .model import xavier

N_IN = 7
HID = 64
HEAD = 32
STEPS = 2

# (name, out, in): every layer is a weight [out][in] followed by a bias [out]
LAYERS = (("enc1", HID, N_IN), ("enc2", HID, HID), ("einit", HID, 2 * HID)) + tuple(
    x for s in range(STEPS) for x in ((f"e{s}a", HID, 3 * HID), (f"e{s}b", HID, HID),
                                       (f"n{s}a", HID, 2 * HID), (f"n{s}b", HID, HID))) + (
    ("head1", HEAD, HID), ("head2", 1, HEAD))


@dataclass
class GnnModel:
    W: dict = field(default_factory=dict)     # name -> [out][in] f64
    b: dict = field(default_factory=dict)     # name -> [out] f64

    def to_blob(self) -> bytes:
        out = [struct.pack("<4sIIIII", b"LSTE", 1, N_IN, HID, HEAD, STEPS)]
        for name, o, i in LAYERS:
            out.append(np.asarray(self.W[name], dtype="<f4").reshape(o, i).tobytes())
            out.append(np.asarray(self.b[name], dtype="<f4").reshape(o).tobytes())
        return b"".join(out)

    def rounded(self) -> "GnnModel":
        """The weights as the device holds them (FP32)."""
        return GnnModel({k: v.astype(np.float32).astype(np.float64) for k, v in self.W.items()},
                        {k: v.astype(np.float32).astype(np.float64) for k, v in self.b.items()})


def make_gnn_model(seed=(3, 2), zero: bool = False, bias: float = 0.0) -> GnnModel:
    rng = np.random.Generator(np.random.PCG64(np.random.SeedSequence(list(seed))))
    m = GnnModel()
    for name, o, i in LAYERS:
        m.W[name] = np.zeros((o, i)) if zero else xavier(rng, o, i)
        m.b[name] = np.full(o, float(bias))
    return m


@dataclass
class Graph:
    x: np.ndarray        # [N, 7] f32 node features
    src: np.ndarray      # [E] i32
    dst: np.ndarray      # [E] i32, sorted ascending

    @property
    def n_nodes(self) -> int:
        return int(self.x.shape[0])

    @property
    def n_edges(self) -> int:
        return int(self.src.shape[0])


def make_graph(n_nodes: int = 200_000, n_edges: int = 1_000_000, n_layers: int = 5, window: int = 2000,
               seed=(3, 3)) -> Graph:
    """LST-like graph: nodes in n_layers equal "layers" (segments by layer),
    edges only between consecutive layers (triplets chain segments outward);
    an edge's target is uniform within +-window of the source's aligned index
    in the next layer, restricted to that layer (the locality of detector
    neighbours). Features ~ N(0, 1). Edges are sorted by (dst, src)."""
    rng = np.random.Generator(np.random.PCG64(np.random.SeedSequence(list(seed))))
    per = n_nodes // n_layers
    n_nodes = per * n_layers
    x = rng.standard_normal((n_nodes, N_IN)).astype(np.float32)
    pairs = n_layers - 1
    lay = rng.integers(0, pairs, size=n_edges)
    s_loc = rng.integers(0, per, size=n_edges)
    # target uniform over the part of [s - window, s + window] inside the layer
    # (drawing there instead of clipping keeps the layer's edge nodes from
    # collecting every overflow: in-degrees stay Poisson-like)
    lo = np.maximum(s_loc - window, 0)
    hi = np.minimum(s_loc + window, per - 1)
    d_loc = lo + (rng.random(n_edges) * (hi - lo + 1)).astype(np.int64)
    d_loc = np.minimum(d_loc, hi)
    src = (lay * per + s_loc).astype(np.int64)
    dst = ((lay + 1) * per + d_loc).astype(np.int64)
    order = np.lexsort((src, dst))
    return Graph(x, src[order].astype(np.int32), dst[order].astype(np.int32))
