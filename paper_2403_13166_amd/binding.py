"""ctypes binding of the C ABI in include/lst.h (argument marshalling only).

Every function here has the name of the C entry point it wraps. Loading fails
loudly (RuntimeError) when the HIP library has not been built: there is no
fallback implementation.
"""
from __future__ import annotations

import ctypes as C
import os

HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(HERE, "liblst.so")

LST_OK = 0
LST_E_INVAL = -1
LST_E_STATE = -2
LST_E_CAPACITY = -3
LST_E_HIP = -4
LST_E_NOMEM = -5

LST_MODE_DNN = 0
LST_MODE_PRE_DNN = 1
LST_PREC_F32 = 0
LST_PREC_BF16 = 1
LST_ASYNC = 1
LST_DTYPE_F32 = 0
LST_DTYPE_BF16 = 1
LST_COUNTS_LEN = 8
LST_NOALLOC_SCRATCH_MIB = 128   # static scratch of lst_build_objects_noalloc (include/lst.h)
LST_COUNT_ERR = 4
LST_COUNT_MAXCAND = 5
N_FEATURES = 42

EXPORTED = ("lst_create", "lst_destroy", "lst_load_geometry", "lst_load_model", "lst_workspace_size",
            "lst_build_objects", "lst_build_objects_noalloc", "lst_build_objects_batched", "lst_score", "lst_status_string",
            "lst_last_error", "lst_set_timing", "lst_set_fail_stage", "lst_stage_times", "lst_get_tuning",
            "lst_set_tuning",
            "lst_load_gnn", "lst_gnn_workspace_size", "lst_gnn_score", "lst_tc_workspace_size", "lst_select_tcs",
            "lst_md_graph", "lst_graph_components_workspace_size", "lst_graph_components")


class LstHits(C.Structure):
    _fields_ = [("x", C.c_void_p), ("y", C.c_void_p), ("z", C.c_void_p), ("sensor", C.c_void_p),
                ("n", C.c_int64)]


class LstCaps(C.Structure):
    _fields_ = [("hits", C.c_int64), ("events", C.c_int64), ("md", C.c_int64), ("ls", C.c_int64),
                ("t3", C.c_int64), ("t5", C.c_int64), ("cand", C.c_int64)]


class LstObjects(C.Structure):
    _fields_ = [("md_hits", C.c_void_p), ("ls_md", C.c_void_p), ("t3_ls", C.c_void_p),
                ("t5_t3", C.c_void_p), ("t5_score", C.c_void_p), ("t5_chi2_rphi", C.c_void_p),
                ("t5_chi2_rz", C.c_void_p), ("t5_feat", C.c_void_p), ("counts_dev", C.c_void_p),
                ("n_md", C.c_int64), ("n_ls", C.c_int64), ("n_t3", C.c_int64), ("n_t5", C.c_int64)]


class LstOptions(C.Structure):
    _fields_ = [("mode", C.c_int32), ("precision", C.c_int32), ("score_min", C.c_float),
                ("flags", C.c_int32)]


class LstTuning(C.Structure):
    _fields_ = [("bin_split", C.c_int32), ("tile_per", C.c_int32 * 5), ("eval_blocks", C.c_int32),
                ("t3_masks", C.c_int32)]

    def as_dict(self) -> dict:
        return {"bin_split": self.bin_split, "tile_per": list(self.tile_per), "eval_blocks": self.eval_blocks,
                "t3_masks": self.t3_masks}

    @staticmethod
    def from_dict(d: dict) -> "LstTuning":
        t = LstTuning()
        t.bin_split = int(d["bin_split"])
        for i, v in enumerate(d["tile_per"]):
            t.tile_per[i] = int(v)
        t.eval_blocks = int(d["eval_blocks"])
        t.t3_masks = int(d.get("t3_masks", T3_MASKS_DEFAULT))
        return t


class LstSeeds(C.Structure):
    _fields_ = [("params", C.c_void_p), ("event_off", C.c_void_p), ("n", C.c_int64)]


class LstTcOptions(C.Structure):
    _fields_ = [("chi2_max", C.c_float), ("sigma_kappa_abs", C.c_float), ("sigma_kappa_rel", C.c_float),
                ("sigma_phi0", C.c_float), ("sigma_cot", C.c_float), ("sigma_z0", C.c_float)]


class LstTcs(C.Structure):
    _fields_ = [("kind", C.c_void_p), ("seed", C.c_void_p), ("obj", C.c_void_p), ("counts_dev", C.c_void_p),
                ("cap", C.c_int64), ("n", C.c_int64)]


TC_COUNTS_LEN = 8
TC_KINDS = ("pT5", "T5", "pT3", "pLS")


class LstError(RuntimeError):
    def __init__(self, status: int, msg: str):
        super().__init__(f"{msg} (status {status})")
        self.status = status


_lib = None


def lib():
    """The loaded HIP library; raises if it is not built."""
    global _lib
    if _lib is None:
        if not os.path.exists(LIB_PATH):
            raise RuntimeError(f"LST HIP library not built: {LIB_PATH} is missing "
                               "(run __graft_entry__.build() or paper_2403_13166_amd/build_lib.py)")
        L = C.CDLL(LIB_PATH)
        vp, i32, i64 = C.c_void_p, C.c_int32, C.c_int64
        L.lst_create.argtypes = [C.c_int, C.POINTER(vp)]
        L.lst_create.restype = i32
        L.lst_destroy.argtypes = [vp]
        L.lst_destroy.restype = None
        L.lst_load_geometry.argtypes = [vp, C.c_char_p, C.c_size_t]
        L.lst_load_geometry.restype = i32
        L.lst_load_model.argtypes = [vp, C.c_char_p, C.c_size_t]
        L.lst_load_model.restype = i32
        L.lst_workspace_size.argtypes = [vp, C.POINTER(LstCaps), C.POINTER(C.c_size_t)]
        L.lst_workspace_size.restype = i32
        L.lst_build_objects.argtypes = [vp, C.POINTER(LstHits), C.POINTER(LstOptions), C.POINTER(LstCaps),
                                        C.POINTER(LstObjects), vp, C.c_size_t, vp]
        L.lst_build_objects.restype = i32
        L.lst_build_objects_noalloc.argtypes = [vp, C.POINTER(LstHits), C.POINTER(LstOptions),
                                                C.POINTER(LstCaps), C.POINTER(LstObjects), vp]
        L.lst_build_objects_noalloc.restype = i32
        L.lst_build_objects_batched.argtypes = [vp, C.POINTER(LstHits), vp, i32, C.POINTER(LstOptions),
                                                C.POINTER(LstCaps), C.POINTER(LstObjects), vp, vp,
                                                C.c_size_t, vp]
        L.lst_build_objects_batched.restype = i32
        L.lst_score.argtypes = [vp, vp, i32, i64, vp, i32, vp]
        L.lst_score.restype = i32
        L.lst_set_timing.argtypes = [vp, i32]
        L.lst_set_timing.restype = i32
        L.lst_set_fail_stage.argtypes = [vp, i32]
        L.lst_set_fail_stage.restype = i32
        L.lst_stage_times.argtypes = [vp, vp, i32]
        L.lst_stage_times.restype = i32
        L.lst_load_gnn.argtypes = [vp, C.c_char_p, C.c_size_t]
        L.lst_load_gnn.restype = i32
        L.lst_gnn_workspace_size.argtypes = [vp, i64, i64, C.POINTER(C.c_size_t)]
        L.lst_gnn_workspace_size.restype = i32
        L.lst_gnn_score.argtypes = [vp, vp, i64, vp, vp, i64, vp, vp, C.c_size_t, i32, vp]
        L.lst_gnn_score.restype = i32
        L.lst_tc_workspace_size.argtypes = [vp, C.POINTER(LstObjects), i64, i32, C.POINTER(C.c_size_t)]
        L.lst_tc_workspace_size.restype = i32
        L.lst_select_tcs.argtypes = [vp, C.POINTER(LstHits), C.POINTER(LstObjects), vp, i32, C.POINTER(LstSeeds),
                                     C.POINTER(LstTcOptions), C.POINTER(LstTcs), vp, C.c_size_t, vp]
        L.lst_select_tcs.restype = i32
        L.lst_md_graph.argtypes = [vp, C.POINTER(LstHits), C.POINTER(LstObjects), vp, vp, vp, vp]
        L.lst_md_graph.restype = i32
        L.lst_graph_components_workspace_size.argtypes = [vp, i64, C.POINTER(C.c_size_t)]
        L.lst_graph_components_workspace_size.restype = i32
        L.lst_graph_components.argtypes = [vp, i64, vp, vp, vp, i64, C.c_float, i32, vp, vp, vp, C.c_size_t, vp]
        L.lst_graph_components.restype = i32
        L.lst_get_tuning.argtypes = [vp, C.POINTER(LstTuning)]
        L.lst_get_tuning.restype = i32
        L.lst_set_tuning.argtypes = [vp, C.POINTER(LstTuning)]
        L.lst_set_tuning.restype = i32
        L.lst_status_string.argtypes = [i32]
        L.lst_status_string.restype = C.c_char_p
        L.lst_last_error.argtypes = [vp]
        L.lst_last_error.restype = C.c_char_p
        _lib = L
    return _lib


def _check(ctx, status: int, what: str):
    if status != LST_OK:
        detail = lib().lst_last_error(ctx).decode() if ctx else ""
        raise LstError(status, f"{what}: {lib().lst_status_string(status).decode()}: {detail}")


def lst_create(device: int = 0):
    h = C.c_void_p()
    _check(None, lib().lst_create(int(device), C.byref(h)), "lst_create")
    return h


def lst_destroy(ctx) -> None:
    lib().lst_destroy(ctx)


def lst_load_geometry(ctx, blob: bytes) -> None:
    _check(ctx, lib().lst_load_geometry(ctx, blob, len(blob)), "lst_load_geometry")


def lst_load_model(ctx, blob: bytes) -> None:
    _check(ctx, lib().lst_load_model(ctx, blob, len(blob)), "lst_load_model")


def lst_workspace_size(ctx, caps: LstCaps) -> int:
    n = C.c_size_t()
    _check(ctx, lib().lst_workspace_size(ctx, C.byref(caps), C.byref(n)), "lst_workspace_size")
    return int(n.value)


def lst_build_objects(ctx, hits: LstHits, opts: LstOptions, caps: LstCaps, out: LstObjects, ws: int,
                      ws_bytes: int, stream: int, check: bool = True) -> int:
    st = lib().lst_build_objects(ctx, C.byref(hits), C.byref(opts), C.byref(caps), C.byref(out), ws,
                                 ws_bytes, stream)
    if check:
        _check(ctx, st, "lst_build_objects")
    return st


def lst_build_objects_noalloc(ctx, hits: LstHits, opts: LstOptions, caps: LstCaps, out: LstObjects,
                              stream: int, check: bool = True) -> int:
    st = lib().lst_build_objects_noalloc(ctx, C.byref(hits), C.byref(opts), C.byref(caps), C.byref(out), stream)
    if check:
        _check(ctx, st, "lst_build_objects_noalloc")
    return st


def lst_build_objects_batched(ctx, hits: LstHits, event_offsets_dev: int, n_events: int, opts: LstOptions,
                              caps: LstCaps, out: LstObjects, event_obj_offsets_dev: int, ws: int,
                              ws_bytes: int, stream: int, check: bool = True) -> int:
    st = lib().lst_build_objects_batched(ctx, C.byref(hits), event_offsets_dev, int(n_events), C.byref(opts),
                                         C.byref(caps), C.byref(out), event_obj_offsets_dev, ws, ws_bytes,
                                         stream)
    if check:
        _check(ctx, st, "lst_build_objects_batched")
    return st


def lst_score(ctx, X_dev: int, x_dtype: int, n: int, scores_dev: int, precision: int, stream: int) -> None:
    _check(ctx, lib().lst_score(ctx, X_dev, int(x_dtype), int(n), scores_dev, int(precision), stream),
           "lst_score")


# eval-only windows of the MD, LS and T3 stages ("md", "ls", "t3") and the
# whole stages ("md_all", "ls_all", "t3_all")
STAGE_WINDOWS = ("build", "bin", "md", "ls", "t3", "t5", "score", "md_all", "ls_all", "t3_all")


def lst_set_timing(ctx, enable: bool) -> None:
    _check(ctx, lib().lst_set_timing(ctx, int(bool(enable))), "lst_set_timing")


# stages of the build that failure injection can stop before (0: off)
FAIL_STAGES = ("off", "bin", "md", "ls", "t3", "t5", "score")


def lst_set_fail_stage(ctx, stage: int) -> None:
    _check(ctx, lib().lst_set_fail_stage(ctx, int(stage)), "lst_set_fail_stage")


def lst_stage_times(ctx) -> dict:
    """ms per stage window of the most recent completed build (stream synchronised)."""
    buf = (C.c_float * len(STAGE_WINDOWS))()
    _check(ctx, lib().lst_stage_times(ctx, buf, len(STAGE_WINDOWS)), "lst_stage_times")
    return dict(zip(STAGE_WINDOWS, list(buf)))


def lst_load_gnn(ctx, blob: bytes) -> None:
    _check(ctx, lib().lst_load_gnn(ctx, blob, len(blob)), "lst_load_gnn")


def lst_gnn_workspace_size(ctx, n_nodes: int, n_edges: int) -> int:
    n = C.c_size_t()
    _check(ctx, lib().lst_gnn_workspace_size(ctx, int(n_nodes), int(n_edges), C.byref(n)), "lst_gnn_workspace_size")
    return int(n.value)


def lst_gnn_score(ctx, x_dev: int, n_nodes: int, src_dev: int, dst_dev: int, n_edges: int, scores_dev: int,
                  ws: int, ws_bytes: int, flags: int, stream: int, check: bool = True) -> int:
    st = lib().lst_gnn_score(ctx, x_dev, int(n_nodes), src_dev, dst_dev, int(n_edges), scores_dev, ws, ws_bytes,
                             int(flags), stream)
    if check:
        _check(ctx, st, "lst_gnn_score")
    return st


# tile sizes each stage is compiled for (candidates per thread): MD, LS, T3, T5 pre, T5 fit
TILE_CHOICES = ((2, 4, 8), (2, 4, 8), (1, 2, 4), (1, 2, 4), (1, 2))
T3_MASKS_DEFAULT = 8


def lst_get_tuning(ctx) -> dict:
    t = LstTuning()
    _check(ctx, lib().lst_get_tuning(ctx, C.byref(t)), "lst_get_tuning")
    return t.as_dict()


def lst_set_tuning(ctx, tuning: dict | None) -> None:
    """Set launch shapes ({"bin_split", "tile_per": [5], "eval_blocks", "t3_masks"}, t3_masks optional);
    None restores the defaults."""
    if tuning is None:
        _check(ctx, lib().lst_set_tuning(ctx, None), "lst_set_tuning")
    else:
        t = LstTuning.from_dict(tuning)
        _check(ctx, lib().lst_set_tuning(ctx, C.byref(t)), "lst_set_tuning")


def lst_status_string(status: int) -> str:
    return lib().lst_status_string(int(status)).decode()


def lst_last_error(ctx) -> str:
    return lib().lst_last_error(ctx).decode()


def lst_tc_workspace_size(ctx, objects: LstObjects, n_seeds: int, n_events: int) -> int:
    n = C.c_size_t()
    _check(ctx, lib().lst_tc_workspace_size(ctx, C.byref(objects), int(n_seeds), int(n_events), C.byref(n)),
           "lst_tc_workspace_size")
    return int(n.value)


def lst_select_tcs(ctx, hits: LstHits, objects: LstObjects, event_obj_offsets_dev: int, n_events: int,
                   seeds: LstSeeds, opt: LstTcOptions, out: LstTcs, ws: int, ws_bytes: int, stream: int,
                   check: bool = True) -> int:
    st = lib().lst_select_tcs(ctx, C.byref(hits), C.byref(objects), event_obj_offsets_dev, int(n_events),
                              C.byref(seeds), C.byref(opt), C.byref(out), ws, ws_bytes, stream)
    if check:
        _check(ctx, st, "lst_select_tcs")
    return st


def lst_md_graph(ctx, hits: LstHits, objects: LstObjects, features_dev: int, src_dev: int, dst_dev: int,
                 stream: int) -> None:
    _check(ctx, lib().lst_md_graph(ctx, C.byref(hits), C.byref(objects), features_dev, src_dev, dst_dev, stream),
           "lst_md_graph")


def lst_graph_components_workspace_size(ctx, n_nodes: int) -> int:
    n = C.c_size_t()
    _check(ctx, lib().lst_graph_components_workspace_size(ctx, int(n_nodes), C.byref(n)),
           "lst_graph_components_workspace_size")
    return int(n.value)


def lst_graph_components(ctx, n_nodes: int, src_dev: int, dst_dev: int, scores_dev: int, n_edges: int,
                         threshold: float, min_mds: int, labels_dev: int, n_tc_dev: int, ws: int, ws_bytes: int,
                         stream: int, check: bool = True) -> int:
    st = lib().lst_graph_components(ctx, int(n_nodes), src_dev, dst_dev, scores_dev, int(n_edges), float(threshold),
                                    int(min_mds), labels_dev, n_tc_dev, ws, ws_bytes, stream)
    if check:
        _check(ctx, st, "lst_graph_components")
    return st
