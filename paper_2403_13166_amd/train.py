"""T5-DNN training on synthetic truth, its working point, and the efficiency
and fake rate it gives (paper Sec. 2 and Sec. 3; matching rule of Sec. 1).

What the paper fixes and what is read here:
  * the training set is every T5 the builder makes with the circle-fit
    heuristic cut removed (Sec. 2), i.e. the DNN-mode T5s;
  * a T5 is real when more than 75 % of its hits belong to one simulated
    track (the matching rule of Sec. 1 applied to the T5's 10 hits: at least
    8 hits); noise hits count in the denominator and belong to no track;
  * binary cross entropy, the set shuffled and split 80 / 20 into training
    and testing (Sec. 2), the 42 -> 32 -> 32 -> 1 architecture of the model
    blob (ReLU, sigmoid output);
  * the working point is the score threshold that keeps the same fraction of
    real T5s as the pre-DNN selection (the chi2_rphi cut) keeps, so that the
    fake rates compare at matched efficiency (Sec. 3).
Reading: the optimiser is Adam (the paper names none), the standardisation
constants of the blob are the training set's mean and standard deviation.

The features are the builder's own (the GPU path's 42 inputs, FP32, before
standardisation); training itself is a small offline numpy loop, not part
of the per-event path. The trained weights are written as a model blob that
lst_load_model reads like any other.
"""
from __future__ import annotations

import argparse
import json
import sys
import time
from dataclasses import dataclass

import numpy as np

from .synth.model import Model, N_FEAT, N_H1, N_H2

REAL_FRACTION = 0.75      # a T5 is real with more than this fraction of its hits from one track


def t5_truth(md_hits: np.ndarray, t5_mds: np.ndarray, truth: np.ndarray):
    """Per T5: (is_real, matched track id or -1). md_hits [n_md, 2] hit
    indices, t5_mds [n_t5, 5] MD indices, truth [n_hits] track id (-1 noise)."""
    n = len(t5_mds)
    if n == 0:
        return np.zeros(0, bool), np.zeros(0, np.int64)
    hits = md_hits[t5_mds].reshape(n, 10)
    tr = np.sort(truth[hits].astype(np.int64), axis=1)
    # longest run of equal non-negative ids in each sorted row
    best = np.zeros(n, np.int64)
    best_id = np.full(n, -1, np.int64)
    run = np.ones(n, np.int64)
    for k in range(10):
        if k > 0:
            same = tr[:, k] == tr[:, k - 1]
            run = np.where(same, run + 1, 1)
        better = (tr[:, k] >= 0) & (run > best)
        best = np.where(better, run, best)
        best_id = np.where(better, tr[:, k], best_id)
    real = best > REAL_FRACTION * 10
    return real, np.where(real, best_id, -1)


# ------------------------------------------------------------------ the MLP

def init_params(seed) -> dict:
    """Xavier-uniform weights, zero biases (the blob's initialisation)."""
    rng = np.random.Generator(np.random.PCG64(np.random.SeedSequence(list(seed))))

    def xavier(o, i):
        lim = np.sqrt(6.0 / (i + o))
        return rng.uniform(-lim, lim, size=(o, i))
    return {"W1": xavier(N_H1, N_FEAT), "b1": np.zeros(N_H1), "W2": xavier(N_H2, N_H1), "b2": np.zeros(N_H2),
            "w3": xavier(1, N_H2)[0], "b3": np.zeros(1)}


def forward(P: dict, xs: np.ndarray):
    """xs: standardised inputs [n, 42]. Returns the pre-activations and logits."""
    a1 = xs @ P["W1"].T + P["b1"]
    h1 = np.maximum(a1, 0.0)
    a2 = h1 @ P["W2"].T + P["b2"]
    h2 = np.maximum(a2, 0.0)
    logit = h2 @ P["w3"] + P["b3"][0]
    return a1, h1, a2, h2, logit


def bce_loss(logit: np.ndarray, y: np.ndarray) -> float:
    """Mean binary cross entropy of sigmoid(logit) against labels y, written
    with log(1 + e^-|z|) so that large logits stay finite."""
    z = logit
    return float(np.mean(np.maximum(z, 0) - z * y + np.log1p(np.exp(-np.abs(z)))))


def bce_grad(P: dict, xs: np.ndarray, y: np.ndarray) -> dict:
    """Gradient of the mean binary cross entropy w.r.t. every parameter."""
    a1, h1, a2, h2, logit = forward(P, xs)
    g = (1.0 / (1.0 + np.exp(-logit)) - y) / len(y)        # d loss / d logit
    grad = {"w3": h2.T @ g, "b3": np.array([g.sum()])}
    d2 = np.outer(g, P["w3"]) * (a2 > 0)
    grad["W2"] = d2.T @ h1
    grad["b2"] = d2.sum(0)
    d1 = (d2 @ P["W2"]) * (a1 > 0)
    grad["W1"] = d1.T @ xs
    grad["b1"] = d1.sum(0)
    return grad


@dataclass
class TrainResult:
    model: Model
    history: list            # (epoch, train loss, test loss)
    test_index: np.ndarray   # rows of the dataset held out for testing


def fit(X: np.ndarray, y: np.ndarray, epochs: int = 30, batch: int = 1024, lr: float = 1e-3, seed=(6, 0),
        test_fraction: float = 0.2, log=None) -> TrainResult:
    """Shuffle, split 80 / 20, standardise with the training rows' mean and
    standard deviation, and minimise binary cross entropy with Adam."""
    X = np.asarray(X, np.float64)
    y = np.asarray(y, np.float64)
    rng = np.random.Generator(np.random.PCG64(np.random.SeedSequence(list(seed) + [1])))
    perm = rng.permutation(len(y))
    n_test = int(round(test_fraction * len(y)))
    te, tr = perm[:n_test], perm[n_test:]
    mu = X[tr].mean(0)
    sd = X[tr].std(0)
    sd = np.where(sd > 1e-6, sd, 1.0)
    # the blob stores FP32 constants; standardise with exactly those
    mu, sd = mu.astype(np.float32).astype(np.float64), sd.astype(np.float32).astype(np.float64)
    xs = (X - mu) / sd
    P = init_params(seed)
    m = {k: np.zeros_like(v) for k, v in P.items()}
    v = {k: np.zeros_like(v_) for k, v_ in P.items()}
    b1, b2, eps, step = 0.9, 0.999, 1e-8, 0
    history = []
    for ep in range(epochs):
        order = rng.permutation(tr)
        for s in range(0, len(order), batch):
            bi = order[s:s + batch]
            g = bce_grad(P, xs[bi], y[bi])
            step += 1
            for k in P:
                m[k] = b1 * m[k] + (1 - b1) * g[k]
                v[k] = b2 * v[k] + (1 - b2) * g[k] ** 2
                P[k] -= lr * (m[k] / (1 - b1 ** step)) / (np.sqrt(v[k] / (1 - b2 ** step)) + eps)
        ltr = bce_loss(forward(P, xs[tr])[4], y[tr])
        lte = bce_loss(forward(P, xs[te])[4], y[te]) if len(te) else float("nan")
        history.append((ep, ltr, lte))
        if log:
            log(f"epoch {ep}: train loss {ltr:.4f}, test loss {lte:.4f}")
    f32 = lambda a: np.asarray(a, np.float32)
    model = Model(f32(mu), f32(sd), f32(P["W1"]), f32(P["b1"]), f32(P["W2"]), f32(P["b2"]), f32(P["w3"]),
                  float(np.float32(P["b3"][0])))
    return TrainResult(model, history, te)


def predict(model: Model, X: np.ndarray) -> np.ndarray:
    """FP64 forward of a blob's model on raw (untransformed-by-mu/sd) features."""
    P = {"W1": model.W1.astype(np.float64), "b1": model.b1.astype(np.float64),
         "W2": model.W2.astype(np.float64), "b2": model.b2.astype(np.float64),
         "w3": model.w3.astype(np.float64), "b3": np.array([model.b3])}
    xs = (np.asarray(X, np.float64) - model.mu.astype(np.float64)) / model.sd.astype(np.float64)
    return 1.0 / (1.0 + np.exp(-forward(P, xs)[4]))


# ------------------------------------------------------ working point and rates

def working_point(score_real: np.ndarray, target_eff: float) -> float:
    """Largest threshold t such that the fraction of real T5s with score >= t
    is at least target_eff."""
    s = np.sort(np.asarray(score_real))[::-1]
    if len(s) == 0:
        return float("nan")
    k = int(np.ceil(target_eff * len(s)))
    k = min(max(k, 1), len(s))
    return float(s[k - 1])


def rates(keep: np.ndarray, real: np.ndarray, track: np.ndarray, tracks_all: np.ndarray):
    """T5-level real efficiency, fraction of fakes kept, fake fraction of the
    kept set; track-level efficiency over the tracks with a real T5."""
    keep = np.asarray(keep, bool)
    real = np.asarray(real, bool)
    found = np.unique(track[keep & real])
    return {"real_t5_efficiency": float(keep[real].mean()) if real.any() else float("nan"),
            "fakes_kept": float(keep[~real].mean()) if (~real).any() else float("nan"),
            "fake_fraction_of_selected": float((~real[keep]).mean()) if keep.any() else float("nan"),
            "track_efficiency": float(len(np.intersect1d(found, tracks_all)) / max(1, len(tracks_all)))}


# ---------------------------------------------------------- GPU data collection

def collect(builder, events, event_key=0):
    """Build every event on the GPU (DNN mode, FP32 features) and return the
    dataset: features [n, 42], real labels, matched track ids (made unique
    per event), chi2_rphi, and the per-event keys of reconstructable tracks."""
    from .runtime import to_device
    from . import binding as B
    Xs, ys, ts, cs, tr_all = [], [], [], [], []
    for i, ev in enumerate(events):
        o = builder.build(*to_device(ev, builder.device), mode=B.LST_MODE_DNN, precision=B.LST_PREC_F32,
                          with_features=True).to_host()
        real, tid = t5_truth(o.md_hits, o.t5_mds(), ev.truth)
        key = np.where(tid >= 0, (event_key + i) * 10_000_000 + tid, -1)
        Xs.append(o.t5_feat.astype(np.float64)); ys.append(real); ts.append(key); cs.append(o.t5_chi2_rphi)
        tr_all.append(np.unique(key[real]))
    cat = lambda a, d: np.concatenate(a) if a else np.zeros(d)
    return (np.concatenate(Xs) if Xs else np.zeros((0, N_FEAT)), cat(ys, 0).astype(bool), cat(ts, 0).astype(np.int64),
            cat(cs, 0).astype(np.float64), cat(tr_all, 0).astype(np.int64))


def compare_selections(score, chi2_rphi, real, track, tracks_all, chi2_cut: float):
    """Pre-DNN selection (chi2_rphi cut) against the DNN at the working point
    that matches the pre-DNN real-T5 efficiency."""
    pre = chi2_rphi <= chi2_cut
    pre_r = rates(pre, real, track, tracks_all)
    thr = working_point(score[real], pre_r["real_t5_efficiency"])
    dnn_r = rates(score >= thr, real, track, tracks_all)
    return {"working_point": thr, "pre_dnn": pre_r, "dnn": dnn_r,
            "fake_reduction": pre_r["fakes_kept"] / max(dnn_r["fakes_kept"], 1e-12)}


def main(argv=None):
    ap = argparse.ArgumentParser(description="Train the T5-DNN on synthetic PU200-like events")
    ap.add_argument("--train-events", type=int, default=40)
    ap.add_argument("--eval-events", type=int, default=10)
    ap.add_argument("--epochs", type=int, default=30)
    ap.add_argument("--out", default=None, help="write the trained model blob here")
    ap.add_argument("--report", default=None, help="write the JSON report here")
    a = ap.parse_args(argv)
    from .runtime import Builder
    from .synth import events as E, geometry as G, model as M
    geo = G.make_geometry(True)
    log = lambda m: print(m, file=sys.stderr, flush=True)
    b = Builder(geo.to_blob(), M.make_model().to_blob(), 0)
    t0 = time.perf_counter()
    train_evs = [E.make_event(geo, E.PU200, (5, e)) for e in range(a.train_events)]
    X, y, trk, c2, _ = collect(b, train_evs, 0)
    t_collect = time.perf_counter() - t0
    log(f"{len(y)} T5s from {a.train_events} events, {y.mean():.3f} real ({t_collect:.1f} s)")
    t0 = time.perf_counter()
    res = fit(X, y, epochs=a.epochs, log=log)
    t_fit = time.perf_counter() - t0
    te = res.test_index
    p_te = predict(res.model, X[te])
    held = compare_selections(p_te, c2[te], y[te], trk[te], np.unique(trk[te][y[te]]), geo.params["chi2_rphi_max"])
    # unseen events, scored by the GPU with the trained blob
    b.close()
    b = Builder(geo.to_blob(), res.model.to_blob(), 0)
    eval_evs = [E.make_event(geo, E.PU200, (5, 1000 + e)) for e in range(a.eval_events)]
    from .runtime import to_device
    from . import binding as B
    scores, c2e, ye, tre, tall = [], [], [], [], []
    for i, ev in enumerate(eval_evs):
        o = b.build(*to_device(ev, b.device), mode=B.LST_MODE_DNN, precision=B.LST_PREC_BF16).to_host()
        real, tid = t5_truth(o.md_hits, o.t5_mds(), ev.truth)
        key = np.where(tid >= 0, (1000 + i) * 10_000_000 + tid, -1)
        scores.append(o.t5_score); c2e.append(o.t5_chi2_rphi); ye.append(real); tre.append(key)
        tall.append(np.unique(key[real]))
    b.close()
    cat = np.concatenate
    unseen = compare_selections(cat(scores).astype(np.float64), cat(c2e).astype(np.float64), cat(ye), cat(tre),
                                cat(tall), geo.params["chi2_rphi_max"])
    report = {"train_events": a.train_events, "eval_events": a.eval_events, "t5_total": int(len(y)),
              "real_fraction": float(y.mean()), "epochs": a.epochs, "collect_s": t_collect, "fit_s": t_fit,
              "loss_history": [[int(e), float(l1), float(l2)] for e, l1, l2 in res.history],
              "held_out_20pct": held, "unseen_events_gpu_bf16": unseen}
    print(json.dumps(report), flush=True)
    if a.report:
        with open(a.report, "w") as f:
            json.dump(report, f, indent=1)
    if a.out:
        with open(a.out, "wb") as f:
            f.write(res.model.to_blob())


if __name__ == "__main__":
    main()
