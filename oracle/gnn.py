"""FP64 oracle of the edge classifier (test infrastructure: only tests, the
smoke check and the CPU baseline of the benchmark may use it).

The paper (Sec. 4) proposes a GNN that classifies the edges of a graph built
from LST objects and gives no architecture. The reading implemented here is
an interaction network, written out step by step with numpy in FP64:

  h0 = relu(Wb relu(Wa x + ba) + bb)
  e0 = relu(Wc [h0_src, h0_dst] + bc)
  for each of the two message-passing steps (own weights per step):
    e <- e + We2 relu(We1 [h_src, h_dst, e] + be1) + be2
    m_v = sum of e over the edges whose dst is v
    h <- h + Wn2 relu(Wn1 [h, m] + bn1) + bn2
  score = sigmoid(wh2 . relu(Wh1 e + bh1) + bh2)

Weights are passed as dicts of arrays ([out][in]) named as in the model blob.
"""
from __future__ import annotations

import numpy as np


def _relu(v):
    return np.maximum(v, 0.0)


def _lin(W, b, name, v):
    return v @ np.asarray(W[name], np.float64).T + np.asarray(b[name], np.float64)


def edge_scores(W: dict, b: dict, x, src, dst, steps: int = 2, return_state: bool = False):
    """Scores [E] of every edge (src[i] -> dst[i]) of the graph with node features x [N, 7]."""
    x = np.asarray(x, np.float64)
    src = np.asarray(src, np.int64)
    dst = np.asarray(dst, np.int64)
    n = x.shape[0]
    h = _relu(_lin(W, b, "enc2", _relu(_lin(W, b, "enc1", x))))
    e = _relu(_lin(W, b, "einit", np.concatenate([h[src], h[dst]], axis=1)))
    for s in range(steps):
        upd = _lin(W, b, f"e{s}b", _relu(_lin(W, b, f"e{s}a", np.concatenate([h[src], h[dst], e], axis=1))))
        e = e + upd
        m = np.zeros((n, e.shape[1]))
        np.add.at(m, dst, e)
        h = h + _lin(W, b, f"n{s}b", _relu(_lin(W, b, f"n{s}a", np.concatenate([h, m], axis=1))))
    z = _lin(W, b, "head2", _relu(_lin(W, b, "head1", e)))[:, 0]
    score = 1.0 / (1.0 + np.exp(-z))
    if return_state:
        return score, h, e
    return score
