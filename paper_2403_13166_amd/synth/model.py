"""Seeded T5-DNN weights and feature normalisation (the "model blob").

Sec. 2 of the paper fixes the architecture: a two-hidden-layer MLP with 32
nodes per layer and a binary (sigmoid) output trained with cross entropy. The
trained weights are not published, so the weights here are Xavier/Glorot
uniform draws, biases zero, seeded; the normalisation constants are fixed from
the detector's coordinate ranges (no data-dependent fit), so nothing here
depends on either implementation of the method.

Blob v1 (little endian)::

    char[4] "LSTM", u32 version 1, u32 n_in, u32 n_h1, u32 n_h2, u32 reserved
    f32 mu[n_in], f32 sd[n_in],
    f32 W1[n_h1][n_in], f32 b1[n_h1], f32 W2[n_h2][n_h1], f32 b2[n_h2],
    f32 w3[n_h2], f32 b3
"""
from __future__ import annotations

import math
import struct
from dataclasses import dataclass

import numpy as np

N_FEAT = 42
N_H1 = 32
N_H2 = 32

# Feature layout (index -> meaning); the transforms are applied before the
# (x - mu) / sd standardisation that the model blob carries.
FEATURE_NAMES = tuple(
    [f"{a}_{q}" for a in "ABCDE" for q in ("r", "phi", "z", "eta", "layer", "is_endcap")]
    + ["log_pt_t3in", "log_r_t3in", "log_pt_t3out", "log_r_t3out", "log_pt_t5", "eta_t5",
       "phi_t5", "log_r_bridge", "log1p_chi2_rphi", "log1p_chi2_rz", "abs_d0", "z0_fit"])
assert len(FEATURE_NAMES) == N_FEAT


def _t5_norm():
    mu = np.zeros(N_FEAT); sd = np.ones(N_FEAT)
    for a in range(5):
        mu[6 * a:6 * a + 6] = (65.0, 0.0, 0.0, 0.0, 6.0, 0.5)
        sd[6 * a:6 * a + 6] = (30.0, 1.8, 100.0, 1.4, 3.2, 0.5)
    mu[30:42] = (math.log(3.0), math.log(250.0), math.log(3.0), math.log(250.0), math.log(3.0),
                 0.0, 0.0, math.log(250.0), 1.5, 1.5, 0.5, 0.0)
    sd[30:42] = (1.0, 1.0, 1.0, 1.0, 1.0, 1.4, 1.8, 1.0, 1.5, 1.5, 1.0, 7.0)
    return mu, sd


@dataclass
class Model:
    mu: np.ndarray
    sd: np.ndarray
    W1: np.ndarray
    b1: np.ndarray
    W2: np.ndarray
    b2: np.ndarray
    w3: np.ndarray
    b3: float

    def to_blob(self) -> bytes:
        f = lambda a: np.asarray(a, dtype="<f4").ravel().tobytes()
        head = struct.pack("<4sIIIII", b"LSTM", 1, N_FEAT, N_H1, N_H2, 0)
        return b"".join([head, f(self.mu), f(self.sd), f(self.W1), f(self.b1), f(self.W2),
                         f(self.b2), f(self.w3), f([self.b3])])


def xavier(rng, fan_out, fan_in):
    lim = math.sqrt(6.0 / (fan_in + fan_out))
    return rng.uniform(-lim, lim, size=(fan_out, fan_in))


def make_model(seed=(3, 1), standardise: bool = True, zero: bool = False, b3: float = 0.0) -> Model:
    """T5-DNN 42 -> 32 -> 32 -> 1. standardise=False gives mu = 0, sd = 1 (inputs
    already N(0, 1)); zero=True zeroes every weight (output sigmoid(b3))."""
    rng = np.random.Generator(np.random.PCG64(np.random.SeedSequence(list(seed))))
    W1 = xavier(rng, N_H1, N_FEAT)
    W2 = xavier(rng, N_H2, N_H1)
    w3 = xavier(rng, 1, N_H2)[0]
    if zero:
        W1[:] = 0; W2[:] = 0; w3[:] = 0
    mu, sd = _t5_norm() if standardise else (np.zeros(N_FEAT), np.ones(N_FEAT))
    # store what the blob stores (f32) so every consumer sees identical values
    r = lambda a: np.asarray(a, np.float32)
    return Model(r(mu), r(sd), r(W1), r(np.zeros(N_H1)), r(W2), r(np.zeros(N_H2)), r(w3),
                 float(np.float32(b3)))


def make_scoring_inputs(n: int, seed=(3, 0)) -> np.ndarray:
    """Standalone scoring workload: n x 42 features drawn from N(0, 1), f32."""
    rng = np.random.Generator(np.random.PCG64(np.random.SeedSequence(list(seed))))
    return rng.standard_normal((n, N_FEAT), dtype=np.float32)
