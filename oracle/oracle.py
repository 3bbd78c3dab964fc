"""ctypes front end of the FP64 oracle (test infrastructure only).

Objects are returned as numpy arrays in the oracle's own numbering and also as
hit-index keys (MD = (anchor, other); LS = 2 MD keys; T3 = 3 MD keys; T5 = 5 MD
keys), which is how results are compared with the GPU library.
"""
from __future__ import annotations

import ctypes as C
import os
from dataclasses import dataclass

import numpy as np

from .build import LIB, build

_lib = None


def lib():
    global _lib
    if _lib is None:
        if not os.path.exists(LIB):
            build()
        L = C.CDLL(LIB)
        vp = C.c_void_p
        L.orc_geom_load.restype = vp
        L.orc_geom_load.argtypes = [C.c_char_p, C.c_size_t]
        L.orc_geom_free.argtypes = [vp]
        L.orc_model_load.restype = vp
        L.orc_model_load.argtypes = [C.c_char_p, C.c_size_t]
        L.orc_model_free.argtypes = [vp]
        L.orc_build.restype = C.c_int
        L.orc_build.argtypes = [vp, vp, vp, vp, vp, vp, C.c_int64, C.c_int, C.c_double,
                                C.POINTER(vp)]
        L.orc_result_free.argtypes = [vp]
        L.orc_result_count.restype = C.c_int64
        L.orc_result_count.argtypes = [vp, C.c_int]
        L.orc_result_copy.argtypes = [vp] + [vp] * 8
        L.orc_cut_values.restype = C.c_int
        L.orc_cut_values.argtypes = [vp, vp, vp, vp, vp, vp, C.c_int64, C.c_int, vp, C.c_int,
                                     C.c_double, vp, vp, vp, vp, vp, vp]
        L.orc_cut_values_d.restype = C.c_int
        L.orc_cut_values_d.argtypes = [vp, vp, vp, vp, vp, vp, C.c_int, C.c_int, C.c_double,
                                       vp, vp, vp, vp, vp, vp]
        L.orc_mlp.argtypes = [vp, vp, C.c_int64, vp]
        L.orc_circle_fit.argtypes = [vp, vp, vp, C.c_int, vp]
        L.orc_line_fit.argtypes = [vp, vp, vp, C.c_int, vp]
        _lib = L
    return _lib


def _p(a: np.ndarray):
    return a.ctypes.data_as(C.c_void_p)


class Geom:
    def __init__(self, blob: bytes):
        self._blob = blob
        self.h = lib().orc_geom_load(blob, len(blob))
        if not self.h:
            raise ValueError("oracle rejected geometry blob")

    def __del__(self):
        if getattr(self, "h", None) and _lib is not None:
            _lib.orc_geom_free(self.h)
            self.h = None


class Model:
    def __init__(self, blob: bytes):
        self._blob = blob
        self.h = lib().orc_model_load(blob, len(blob))
        if not self.h:
            raise ValueError("oracle rejected model blob")

    def __del__(self):
        if getattr(self, "h", None) and _lib is not None:
            _lib.orc_model_free(self.h)
            self.h = None


@dataclass
class Result:
    md: np.ndarray       # [n_md, 2] hit indices (anchor, other)
    ls: np.ndarray       # [n_ls, 2] md indices
    t3: np.ndarray       # [n_t3, 2] ls indices
    t5: np.ndarray       # [n_t5, 2] t3 indices
    chi2_rphi: np.ndarray
    chi2_rz: np.ndarray
    score: np.ndarray
    feat: np.ndarray     # [n_t5, 42]

    def counts(self):
        return (len(self.md), len(self.ls), len(self.t3), len(self.t5))

    # hit-index keys
    def md_keys(self):
        return [tuple(r) for r in self.md.tolist()]

    def ls_mds(self):
        return self.ls

    def t3_mds(self):
        """[n_t3, 3] MD indices (A, B, C)."""
        return np.stack([self.ls[self.t3[:, 0], 0], self.ls[self.t3[:, 0], 1],
                         self.ls[self.t3[:, 1], 1]], axis=1) if len(self.t3) else np.zeros((0, 3), np.int32)

    def t5_mds(self):
        """[n_t5, 5] MD indices (A..E)."""
        if not len(self.t5):
            return np.zeros((0, 5), np.int32)
        t3m = self.t3_mds()
        a = t3m[self.t5[:, 0]]
        b = t3m[self.t5[:, 1]]
        return np.concatenate([a, b[:, 1:]], axis=1)


def build_objects(geom: Geom, model: Model | None, x, y, z, sensor, mode: int = 0,
                  score_min: float = float("nan")) -> Result:
    x = np.ascontiguousarray(x, np.float32); y = np.ascontiguousarray(y, np.float32)
    z = np.ascontiguousarray(z, np.float32); sensor = np.ascontiguousarray(sensor, np.int32)
    L = lib()
    res = C.c_void_p()
    rc = L.orc_build(geom.h, model.h if model else None, _p(x), _p(y), _p(z), _p(sensor),
                     int(x.shape[0]), int(mode), float(score_min), C.byref(res))
    if rc != 0:
        raise ValueError(f"oracle build failed ({rc})")
    try:
        n = [L.orc_result_count(res, s) for s in (1, 2, 3, 4)]
        md = np.zeros((n[0], 2), np.int32); ls = np.zeros((n[1], 2), np.int32)
        t3 = np.zeros((n[2], 2), np.int32); t5 = np.zeros((n[3], 2), np.int32)
        cr = np.zeros(n[3]); cz = np.zeros(n[3]); sc = np.zeros(n[3]); ft = np.zeros((n[3], 42))
        L.orc_result_copy(res, _p(md), _p(ls), _p(t3), _p(t5), _p(cr), _p(cz), _p(sc), _p(ft))
    finally:
        L.orc_result_free(res)
    return Result(md, ls, t3, t5, cr, cz, sc, ft)


@dataclass
class CutValues:
    v: np.ndarray
    t: np.ndarray
    strict: np.ndarray
    detail: np.ndarray | None = None
    feat: np.ndarray | None = None
    score: float = float("nan")

    def passes(self) -> np.ndarray:
        with np.errstate(invalid="ignore"):
            return np.where(self.strict.astype(bool), self.v < self.t, self.v <= self.t)

    def all_pass(self) -> bool:
        return bool(np.all(self.passes()))

    def marginal(self, rel: float = 1e-5) -> np.ndarray:
        with np.errstate(invalid="ignore"):
            return np.abs(self.v - self.t) <= rel * np.abs(self.t)


def cut_values(geom: Geom, model: Model | None, x, y, z, sensor, stage: int, hits,
               mode: int = 0, score_min: float = float("nan")) -> CutValues:
    x = np.ascontiguousarray(x, np.float32); y = np.ascontiguousarray(y, np.float32)
    z = np.ascontiguousarray(z, np.float32); sensor = np.ascontiguousarray(sensor, np.int32)
    h = np.ascontiguousarray(hits, np.int64)
    v = np.zeros(16); t = np.zeros(16); st = np.zeros(16, np.int32)
    det = np.zeros(7); ft = np.zeros(42); sc = np.zeros(1)
    n = lib().orc_cut_values(geom.h, model.h if model else None, _p(x), _p(y), _p(z), _p(sensor),
                             int(x.shape[0]), int(stage), _p(h), int(mode), float(score_min),
                             _p(v), _p(t), _p(st), _p(det), _p(ft), _p(sc))
    if n < 0:
        raise ValueError("bad candidate")
    if stage == 4:
        return CutValues(v[:n], t[:n], st[:n], det, ft, float(sc[0]))
    return CutValues(v[:n], t[:n], st[:n])


def cut_values_exact(geom: Geom, model: Model | None, x, y, z, sensor, stage: int,
                     mode: int = 0, score_min: float = float("nan")) -> CutValues:
    """Cut values of one candidate whose hits are given in FP64, in candidate order."""
    x = np.ascontiguousarray(x, np.float64); y = np.ascontiguousarray(y, np.float64)
    z = np.ascontiguousarray(z, np.float64); sensor = np.ascontiguousarray(sensor, np.int32)
    v = np.zeros(16); t = np.zeros(16); st = np.zeros(16, np.int32)
    det = np.zeros(7); ft = np.zeros(42); sc = np.zeros(1)
    n = lib().orc_cut_values_d(geom.h, model.h if model else None, _p(x), _p(y), _p(z), _p(sensor),
                               int(stage), int(mode), float(score_min), _p(v), _p(t), _p(st),
                               _p(det), _p(ft), _p(sc))
    if n < 0:
        raise ValueError("bad candidate")
    if stage == 4:
        return CutValues(v[:n], t[:n], st[:n], det, ft, float(sc[0]))
    return CutValues(v[:n], t[:n], st[:n])


def mlp(model: Model, X: np.ndarray) -> np.ndarray:
    X = np.ascontiguousarray(X, np.float32)
    out = np.zeros(X.shape[0])
    lib().orc_mlp(model.h, _p(X), int(X.shape[0]), _p(out))
    return out


def circle_fit(x, y, sig=None):
    """-> (xm, ym, A, B, C, D, R, chi2): natural form over centred coordinates."""
    x = np.ascontiguousarray(x, np.float64); y = np.ascontiguousarray(y, np.float64)
    sig = np.ones_like(x) if sig is None else np.ascontiguousarray(sig, np.float64)
    res = np.zeros(8)
    lib().orc_circle_fit(_p(x), _p(y), _p(sig), int(x.shape[0]), _p(res))
    return res


def line_fit(s, z, sig):
    """-> (t, z0, chi2)."""
    s = np.ascontiguousarray(s, np.float64); z = np.ascontiguousarray(z, np.float64)
    sig = np.ascontiguousarray(sig, np.float64)
    res = np.zeros(3)
    lib().orc_line_fit(_p(s), _p(z), _p(sig), int(s.shape[0]), _p(res))
    return res
