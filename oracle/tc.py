"""FP64 oracle of track-candidate selection and duplicate removal (test
infrastructure: only tests, the smoke check and the CPU baseline of the
benchmark may use it).

The paper (Sec. 1 and Table 1, steps 5-8) matches pixel seeds (pLS) to the
outer-tracker objects and forms four mutually exclusive kinds of track
candidates (TC), longest first: pT5 (T5 matched to a seed), T5 (not matched),
pT3 (T3 not in a pT5, matched to a seed) and pLS (seeds in neither); unused
seeds are kept. It names duplicate removal as a later step (Sec. 2) without
defining either step's criteria, so this module implements the following
reading, step by step, per event:

 1. Helix parameters of an outer-tracker object (T5 or T3) from the anchor
    hits A (first MD) and E (last MD) on a circle through the beam line:
    c = |A x E| / (r_A r_E |E - A|), sgn = sign(A x E) (+1 when 0),
    kappa = sgn c, phi0 = atan2(y_A, x_A) - sgn asin(c r_A) (wrapped to
    (-pi, pi]), s_X = asin(c r_X) / c (r_X at c = 0), cot = (z_E - z_A) /
    (s_E - s_A), z0 = z_A - s_A cot. An object with s_E <= s_A or c r >= 1 has
    no parameters and matches no seed.
 2. Match chi2 of seed p and object o (options taken as FP32 numbers, as the
    library receives them): the sum over kappa, phi0 (difference
    wrapped to (-pi, pi]), cot and z0 of (p_i - o_i)^2 / (sigma_p,i^2 +
    sigma_o,i^2), with the seed's own sigmas and the object sigmas of the
    options (sigma_kappa,o = kappa_rel |kappa_o| + kappa_abs). A pair matches
    when chi2 <= chi2_max.
 3. pT5: a seed and a T5 form a pT5 when each is the other's best match; best
    = smallest chi2 rounded to FP32, ties to the smaller index.
 4. T5 TCs: the T5s that are not in a pT5.
 5. pT3: the same mutual best match between the seeds not in a pT5 and the
    T3s that are not one of the two T3s of a pT5's T5.
 6. pLS TCs: the seeds in no pT5 and no pT3.
 7. Duplicate removal among the TCs that have outer-tracker MDs (pT5 and T5:
    the T5's five MDs, pT3: the T3's three): two TCs are duplicates when they
    share more than half of the smaller one's MDs. A TC is removed when it has
    a duplicate of higher priority. Priority: kind (pT5, then T5, then pT3),
    then quality (T5: higher DNN score, or lower r-phi fit chi2 when there is
    no score; pT3: lower match chi2 rounded to FP32), then the smaller object
    index. pLS TCs are never removed.

TC kinds: 0 pT5, 1 T5, 2 pT3, 3 pLS. Each TC is (kind, seed or -1, object
index or -1): the T5 index for pT5 / T5, the T3 index for pT3.
"""
from __future__ import annotations

import math
from dataclasses import dataclass

import numpy as np
import scipy.sparse as sp

K_PT5, K_T5, K_PT3, K_PLS = 0, 1, 2, 3


@dataclass
class TcOptions:
    chi2_max: float = 20.0
    kappa_abs: float = 5e-6
    kappa_rel: float = 0.05
    phi0: float = 2e-3
    cot: float = 5e-3
    z0: float = 0.3


def object_params(x, y, z, md_hits, obj_mds):
    """Step 1. obj_mds [n, k] MD indices (first and last used); returns
    params [n, 4] (kappa, phi0, cot, z0) and valid [n]."""
    n = obj_mds.shape[0]
    P = np.full((n, 4), np.nan)
    valid = np.zeros(n, bool)
    for i in range(n):
        a = md_hits[obj_mds[i, 0], 0]
        e = md_hits[obj_mds[i, -1], 0]
        xa, ya, za = float(x[a]), float(y[a]), float(z[a])
        xe, ye, ze = float(x[e]), float(y[e]), float(z[e])
        ra, re = math.hypot(xa, ya), math.hypot(xe, ye)
        cr = xa * ye - ya * xe
        c = abs(cr) / (ra * re * math.hypot(xe - xa, ye - ya))
        sgn = -1.0 if cr < 0 else 1.0
        if not (c * ra < 1.0 and c * re < 1.0):
            continue
        sa = math.asin(c * ra) / c if c > 0 else ra
        se = math.asin(c * re) / c if c > 0 else re
        if not se > sa:
            continue
        cot = (ze - za) / (se - sa)
        phi0 = math.atan2(ya, xa) - sgn * math.asin(c * ra)
        phi0 = (phi0 + math.pi) % (2.0 * math.pi) - math.pi
        P[i] = (sgn * c, phi0, cot, za - sa * cot)
        valid[i] = True
    return P, valid


def _f32(v):
    """Options are single-precision numbers (as the library receives them)."""
    return float(np.float32(v))


def chi2_matrix(seeds, P, valid, opt: TcOptions):
    """Step 2: [n_seeds, n_obj] chi2 (inf where the object has no parameters)."""
    opt = TcOptions(*(_f32(getattr(opt, k)) for k in TcOptions.__dataclass_fields__))
    s = np.asarray(seeds, np.float64)
    C = np.full((s.shape[0], P.shape[0]), np.inf)
    if not s.shape[0] or not P.shape[0]:
        return C
    so = np.stack([opt.kappa_rel * np.abs(P[:, 0]) + opt.kappa_abs, np.full(len(P), opt.phi0),
                   np.full(len(P), opt.cot), np.full(len(P), opt.z0)], axis=1)
    tot = np.zeros((s.shape[0], P.shape[0]))
    for k in range(4):
        d = s[:, k][:, None] - P[:, k][None, :]
        if k == 1:
            d = (d + math.pi) % (2.0 * math.pi) - math.pi
        tot += d * d / (s[:, 4 + k][:, None] ** 2 + so[:, k][None, :] ** 2)
    C[:, valid] = tot[:, valid]
    return C


def _key(c):
    """Ranking value of a chi2: rounded to FP32."""
    return np.asarray(c, np.float64).astype(np.float32)


def mutual_best(C, chi2_max, seed_ok, obj_ok):
    """Step 3 / 5: pairs (p, o) that are each other's best match. Entries
    outside the eligible rows / columns or above chi2_max do not match."""
    ns, no = C.shape
    M = np.where((C <= chi2_max) & seed_ok[:, None] & obj_ok[None, :], C, np.inf)
    K = _key(M)
    best_o = np.full(ns, -1)
    for p in range(ns):
        if np.isfinite(K[p]).any():
            best_o[p] = int(np.argmin(K[p]))          # first minimum = smallest index
    best_p = np.full(no, -1)
    for o in range(no):
        if np.isfinite(K[:, o]).any():
            best_p[o] = int(np.argmin(K[:, o]))
    return [(p, int(best_o[p])) for p in range(ns) if best_o[p] >= 0 and best_p[best_o[p]] == p]


@dataclass
class TcResult:
    tcs: list                 # kept TCs: (kind, seed, obj)
    before: list              # TCs before duplicate removal
    chi2: dict                # (kind, seed, obj) -> match chi2 (pT5, pT3)


def select_event(x, y, z, md_hits, t3_mds, t5_mds, t5_t3, t5_quality, seeds, opt: TcOptions = TcOptions()):
    """Steps 1-7 on one event. t3_mds [n3, 3], t5_mds [n5, 5] MD indices,
    t5_t3 [n5, 2] T3 indices, t5_quality [n5] (lower = better), seeds [ns, 8]."""
    ns = seeds.shape[0]
    n5, n3 = t5_mds.shape[0], t3_mds.shape[0]
    P5, v5 = object_params(x, y, z, md_hits, t5_mds)
    P3, v3 = object_params(x, y, z, md_hits, t3_mds)
    C5 = chi2_matrix(seeds, P5, v5, opt)
    pt5 = mutual_best(C5, _f32(opt.chi2_max), np.ones(ns, bool), np.ones(n5, bool))
    seed_used = np.zeros(ns, bool)
    t5_used = np.zeros(n5, bool)
    t3_used = np.zeros(n3, bool)
    for p, t in pt5:
        seed_used[p] = True
        t5_used[t] = True
        t3_used[t5_t3[t, 0]] = True
        t3_used[t5_t3[t, 1]] = True
    C3 = chi2_matrix(seeds, P3, v3, opt)
    pt3 = mutual_best(C3, _f32(opt.chi2_max), ~seed_used, ~t3_used)
    for p, t in pt3:
        seed_used[p] = True
    tcs = [(K_PT5, p, t) for p, t in sorted(pt5, key=lambda v: v[1])]
    tcs += [(K_T5, -1, t) for t in range(n5) if not t5_used[t]]
    tcs += [(K_PT3, p, t) for p, t in sorted(pt3, key=lambda v: v[1])]
    tcs += [(K_PLS, p, -1) for p in range(ns) if not seed_used[p]]
    # match chi2 of the pairs, rounded to FP32 as in the ranking
    chi2 = {(K_PT5, p, t): float(_key(C5[p, t])) for p, t in pt5}
    chi2.update({(K_PT3, p, t): float(_key(C3[p, t])) for p, t in pt3})
    # step 7
    ot = [i for i, tc in enumerate(tcs) if tc[0] != K_PLS]
    mds = [t5_mds[tcs[i][2]] if tcs[i][0] in (K_PT5, K_T5) else t3_mds[tcs[i][2]] for i in ot]
    keyv = []
    for i in ot:
        kind, p, o = tcs[i]
        q = chi2[tcs[i]] if kind == K_PT3 else float(t5_quality[o])
        keyv.append((kind, q, o))
    drop = set()
    if ot:
        n_md = int(md_hits.shape[0])
        rows = np.concatenate([np.full(len(m), j) for j, m in enumerate(mds)])
        cols = np.concatenate([np.asarray(m) for m in mds])
        inc = sp.csr_matrix((np.ones(len(rows)), (rows, cols)), shape=(len(ot), n_md))
        shared = (inc @ inc.T).tocoo()
        for a, b, v in zip(shared.row, shared.col, shared.data):
            if a == b:
                continue
            if v > min(len(mds[a]), len(mds[b])) / 2 and keyv[b] < keyv[a]:
                drop.add(ot[a])
    kept = [tc for i, tc in enumerate(tcs) if i not in drop]
    return TcResult(kept, tcs, chi2)


def t5_quality(score, chi2_rphi):
    """Quality (lower = better) of T5s for duplicate removal: -score, or the
    r-phi chi2 where there is no score."""
    score = np.asarray(score, np.float64)
    return np.where(np.isfinite(score), -score, np.asarray(chi2_rphi, np.float64))
