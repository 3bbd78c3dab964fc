"""GPU-vs-oracle comparison of object sets (test infrastructure).

Objects are compared as sets of hit-index keys:
  MD = (anchor hit, other hit); LS = (MD, MD); T3 = (MD, MD, MD); T5 = 5 MDs.
Each object in the symmetric difference of a stage is classified:
  inherited - one of its component objects is itself in the previous stage's
              symmetric difference;
  marginal  - recomputed in FP64 by the oracle, the cut that decides the
              disagreement lies within a relative 1e-5 of its threshold
              (GPU-only objects: every cut the oracle fails is within the band;
              oracle-only objects: some cut is within the band);
  violation - anything else. The parity bar is zero violations.
"""
from __future__ import annotations

from dataclasses import dataclass, field

import numpy as np

from oracle import oracle as O

MARGIN = 1e-5


def gpu_keys(h):
    """Host objects of the GPU library -> key sets and per-T5 score dicts."""
    md = [tuple(r) for r in h.md_hits.tolist()]
    ls = [(md[a], md[b]) for a, b in h.ls_md.tolist()]
    t3 = [tuple(md[k] for k in row) for row in h.t3_mds().tolist()]
    t5 = [tuple(md[k] for k in row) for row in h.t5_mds().tolist()]
    return md, ls, t3, t5


def oracle_keys(r: O.Result):
    md = [tuple(r_) for r_ in r.md.tolist()]
    ls = [(md[a], md[b]) for a, b in r.ls.tolist()]
    t3 = [tuple(md[k] for k in row) for row in r.t3_mds().tolist()]
    t5 = [tuple(md[k] for k in row) for row in r.t5_mds().tolist()]
    return md, ls, t3, t5


@dataclass
class StageReport:
    n_gpu: int
    n_oracle: int
    inherited: int = 0
    marginal: int = 0
    violation: int = 0
    duplicates: int = 0
    examples: list = field(default_factory=list)


def _components(stage, key):
    if stage == 1:
        return []
    if stage == 2:
        return list(key)                 # MD keys
    if stage == 3:
        return [(key[0], key[1]), (key[1], key[2])]   # LS keys
    return [key[:3], key[2:]]            # T3 keys


def _hits(key, stage):
    if stage == 1:
        return list(key)
    return [h for md in key for h in md]


def compare(geom: O.Geom, model: O.Model, ev, gpu_host, orc: O.Result, mode: int = 0,
            score_min: float = float("nan")):
    g = gpu_keys(gpu_host)
    o = oracle_keys(orc)
    reports = []
    prev_diff = set()
    for stage in (1, 2, 3, 4):
        gs, os_ = set(g[stage - 1]), set(o[stage - 1])
        rep = StageReport(len(g[stage - 1]), len(o[stage - 1]))
        rep.duplicates = len(g[stage - 1]) - len(gs)
        diff = gs ^ os_
        for key in diff:
            if any(c in prev_diff for c in _components(stage, key)):
                rep.inherited += 1
                continue
            cv = O.cut_values(geom, model, ev.x, ev.y, ev.z, ev.sensor, stage, _hits(key, stage), mode,
                              score_min)
            near = cv.marginal(MARGIN)
            fails = ~cv.passes()
            if key in gs:      # GPU kept it, the oracle rejects it
                ok = bool(np.all(near[fails])) and bool(np.any(fails))
            else:              # the oracle keeps it, the GPU rejected it
                ok = bool(np.any(near))
            if ok:
                rep.marginal += 1
            else:
                rep.violation += 1
                if len(rep.examples) < 5:
                    rep.examples.append((key, "gpu" if key in gs else "oracle", cv.v.tolist(), cv.t.tolist()))
        reports.append(rep)
        prev_diff = diff
    return reports


def score_errors(gpu_host, orc: O.Result):
    """max / mean |score_gpu - score_oracle| and chi2 relative errors over the common T5s."""
    g = gpu_keys(gpu_host)[3]
    o = oracle_keys(orc)[3]
    oi = {k: i for i, k in enumerate(o)}
    ds, dr, dz, n = [], [], [], 0
    for i, k in enumerate(g):
        j = oi.get(k)
        if j is None:
            continue
        n += 1
        ds.append(abs(float(gpu_host.t5_score[i]) - orc.score[j]))
        dr.append(abs(float(gpu_host.t5_chi2_rphi[i]) - orc.chi2_rphi[j]) / max(1e-3, abs(orc.chi2_rphi[j])))
        dz.append(abs(float(gpu_host.t5_chi2_rz[i]) - orc.chi2_rz[j]) / max(1e-3, abs(orc.chi2_rz[j])))
    f = lambda a: (float(np.max(a)) if a else 0.0, float(np.mean(a)) if a else 0.0)
    return dict(n_common=n, score=f(ds), chi2_rphi_rel=f(dr), chi2_rz_rel=f(dz))


def feature_errors(gpu_host, orc: O.Result, angle_cols=()):
    """Per feature column: max |f_gpu - f_oracle| / max(1, |f_oracle|) over the
    common T5s; columns in angle_cols are compared modulo 2 pi."""
    g = gpu_keys(gpu_host)[3]
    o = oracle_keys(orc)[3]
    oi = {k: i for i, k in enumerate(o)}
    pairs = [(i, oi[k]) for i, k in enumerate(g) if k in oi]
    if not pairs:
        return np.zeros(42)
    gi, oj = (np.array(v) for v in zip(*pairs))
    a = gpu_host.t5_feat[gi].astype(np.float64)
    b = orc.feat[oj]
    d = a - b
    ang = list(angle_cols)
    if ang:
        d[:, ang] = np.remainder(d[:, ang] + np.pi, 2 * np.pi) - np.pi
    return np.max(np.abs(d) / np.maximum(1.0, np.abs(b)), axis=0)
