"""Seeded synthetic pixel seeds (pLS) for track-candidate selection.

The paper's pixel seeds come from an upstream tracking iteration on the inner
tracker (Sec. 1, Table 1 step 0), which the synthetic detector does not model.
They are stood in for by helix parameters of the generated tracks, measured
with Gaussian resolution, plus a fraction of fake seeds:

  * a track yields a seed with probability `eff`;
  * parameters (the same helix description the selection uses for
    outer-tracker objects): kappa = signed half-curvature, kappa = -q k_B /
    (2 pT) (the sign is that of A x B for two points A, B of the track at
    increasing radius), phi0 = direction at the beam line, cot = cot(theta) =
    sinh(eta), z0 = z of the vertex;
  * each seed carries its resolutions: sigma_kappa = KAPPA_REL |kappa| +
    KAPPA_ABS, sigma_phi0, sigma_cot, sigma_z0, and the measured value is the
    truth plus a normal deviate of that width;
  * fake seeds (n_fake = fake_frac * n_tracks) have kappa uniform in
    [-c_max, c_max], phi0 uniform, cot uniform in [-5.5, 5.5], z0 ~ N(0, 5 cm).

Seeds are shuffled. This module holds input generation only: no step of the
selection itself.
"""
from __future__ import annotations

import math
from dataclasses import dataclass

import numpy as np

KAPPA_REL, KAPPA_ABS = 0.02, 2e-6      # 1/cm
SIGMA_PHI0 = 1e-3                      # rad
SIGMA_COT = 2e-3
SIGMA_Z0 = 0.05                        # cm

# parameter columns of a seed record
N_SEED_COLS = 8    # kappa, phi0, cot, z0, sigma_kappa, sigma_phi0, sigma_cot, sigma_z0


@dataclass
class Seeds:
    params: np.ndarray   # [n, 8] float32
    track: np.ndarray    # [n] int32 generating track (-1: fake)

    @property
    def n(self) -> int:
        return int(self.params.shape[0])


def _wrap(phi):
    return (phi + math.pi) % (2.0 * math.pi) - math.pi


def true_params(geo, tracks: np.ndarray) -> np.ndarray:
    """[n, 4] float64 (kappa, phi0, cot, z0) of generated tracks (q, pt, eta, phi0, zv)."""
    kb = geo.params["k_b"]
    q, pt, eta, phi0, zv = (tracks[:, i] for i in range(5))
    return np.stack([-q * kb / (2.0 * pt), _wrap(phi0), np.sinh(eta), zv], axis=1)


def make_seeds(geo, ev, rng: np.random.Generator, eff: float = 0.9, fake_frac: float = 0.05) -> Seeds:
    truth = true_params(geo, ev.tracks)
    keep = rng.random(truth.shape[0]) < eff
    tp = truth[keep]
    tid = np.nonzero(keep)[0].astype(np.int32)
    n_fake = int(round(fake_frac * truth.shape[0]))
    cmax = geo.c_max()
    fk = np.stack([rng.uniform(-cmax, cmax, n_fake), rng.uniform(-math.pi, math.pi, n_fake),
                   rng.uniform(-5.5, 5.5, n_fake), rng.normal(0.0, 5.0, n_fake)], axis=1)
    p = np.concatenate([tp, fk], axis=0)
    tid = np.concatenate([tid, np.full(n_fake, -1, np.int32)])
    sig = np.stack([KAPPA_REL * np.abs(p[:, 0]) + KAPPA_ABS, np.full(len(p), SIGMA_PHI0),
                    np.full(len(p), SIGMA_COT), np.full(len(p), SIGMA_Z0)], axis=1)
    meas = p + rng.normal(0.0, 1.0, p.shape) * sig
    meas[:, 1] = _wrap(meas[:, 1])
    order = rng.permutation(len(p))
    params = np.concatenate([meas, sig], axis=1)[order].astype(np.float32)
    return Seeds(np.ascontiguousarray(params), tid[order])


def concat_seeds(seeds):
    """Concatenate per-event seeds into one [n, 8] array plus int64 offsets."""
    off = np.zeros(len(seeds) + 1, np.int64)
    for i, s in enumerate(seeds):
        off[i + 1] = off[i] + s.n
    params = np.concatenate([s.params for s in seeds], axis=0) if seeds else np.zeros((0, 8), np.float32)
    return np.ascontiguousarray(params, np.float32), off
