"""FP64 oracle of the LST-built graph and of its track candidates (test
infrastructure: only tests, the smoke check and the CPU baseline of the
benchmark may use it).

Sec. 4 proposes building a GNN's input graph with LST, MDs as nodes and LSs as
edges, and producing TCs from the classified graph; it fixes neither the node
features nor how TCs are read off. The reading implemented here:

 1. Nodes: every MD. Seven features of MD (anchor hit A, other hit O), all
    local to the MD: r_A / 100, phi_A / pi, z_A / 100 (cm; phi by atan2),
    10 alpha (alpha = angle from the radial direction at the chord midpoint
    M = (A + O) / 2 to the chord O - A, in the transverse plane: the MD's bend),
    eta_MD = asinh((z_O - z_A) / (r_O - r_A)) clipped to [-5, 5] (the chord's
    pseudorapidity; +-5 when r_O = r_A), is_endcap (0 / 1), layer / 11.
 2. Edges: every LS (inner MD a, outer MD b) as the edge b -> a, so that the
    edges entering a node are the segments starting at it.
 3. Edge scores: the edge classifier (oracle/gnn.py).
 4. TCs: the connected components of the graph of the edges with score >=
    threshold, labelled by their smallest MD index; a component is a TC when
    it has at least min_mds MDs.
"""
from __future__ import annotations

import math

import numpy as np
import scipy.sparse as sp
from scipy.sparse.csgraph import connected_components


def md_features(x, y, z, sensor, md_hits, kind, layer):
    """Step 1: [n_md, 7] float64 node features. kind / layer indexed by module."""
    n = md_hits.shape[0]
    X = np.zeros((n, 7))
    for i in range(n):
        a, o = int(md_hits[i, 0]), int(md_hits[i, 1])
        xa, ya, za = float(x[a]), float(y[a]), float(z[a])
        xo, yo, zo = float(x[o]), float(y[o]), float(z[o])
        ra, ro = math.hypot(xa, ya), math.hypot(xo, yo)
        mx, my = 0.5 * (xa + xo), 0.5 * (ya + yo)
        dx, dy = xo - xa, yo - ya
        alpha = math.atan2(mx * dy - my * dx, mx * dx + my * dy)
        dr = ro - ra
        if dr == 0.0:
            eta = math.copysign(5.0, zo - za) if zo != za else 0.0
        else:
            eta = max(-5.0, min(5.0, math.asinh((zo - za) / dr)))
        m = int(sensor[a]) // 2
        X[i] = (ra / 100.0, math.atan2(ya, xa) / math.pi, za / 100.0, 10.0 * alpha, eta,
                float(kind[m] != 0), float(layer[m]) / 11.0)
    return X


def ls_edges(ls_md):
    """Step 2: (src, dst) = (outer MD, inner MD) of every LS."""
    ls_md = np.asarray(ls_md)
    return ls_md[:, 1].astype(np.int64), ls_md[:, 0].astype(np.int64)


def components(n_nodes, src, dst, scores, threshold):
    """Step 4: component label (smallest node index) of every node over the
    edges with score >= threshold."""
    keep = np.asarray(scores, np.float64) >= threshold
    s, d = np.asarray(src)[keep], np.asarray(dst)[keep]
    g = sp.coo_matrix((np.ones(len(s)), (s, d)), shape=(n_nodes, n_nodes))
    _, lab = connected_components(g, directed=True, connection="weak")
    lab = np.asarray(lab)
    # relabel every component by its smallest node
    first = np.full(lab.max() + 1 if len(lab) else 0, n_nodes)
    np.minimum.at(first, lab, np.arange(n_nodes))
    return first[lab]


def track_candidates(labels, min_mds):
    """The components with at least min_mds nodes: {label: sorted node list}."""
    out = {}
    for v, l in enumerate(np.asarray(labels).tolist()):
        out.setdefault(l, []).append(v)
    return {l: v for l, v in out.items() if len(v) >= min_mds}
