"""ctypes declarations of libnbgpu's C ABI (include/nb.h).

Loading fails loudly: there is no fallback implementation of any entry point.
"""
from __future__ import annotations

import ctypes
import os

_PKG = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(_PKG, "libnbgpu.so")

NB_OK = 0
STATUS_NAMES = {
    -1: "NB_EINVAL", -2: "NB_EOVERFLOW", -3: "NB_EMINFILES", -4: "NB_ENOMODEL",
    -5: "NB_EDATA", -6: "NB_ENOMEM", -7: "NB_EHIP", -8: "NB_EREJECTED",
}

MULTINOMIAL, BERNOULLI, GAUSSIAN = 0, 1, 2
X_U8, X_I32, X_FP8 = 0, 1, 2
W_F32, W_BF16 = 0, 1
TRAIN_ASYNC = 1
PLAN_TUNE, PLAN_STATIC, PLAN_STREAM = 1, 2, 4
SERVE_DEVICE_INPUTS, SERVE_SIMULATE = 1, 2


class NbModel(ctypes.Structure):
    _fields_ = [("kind", ctypes.c_int32), ("n_classes", ctypes.c_int32),
                ("n_features", ctypes.c_int32), ("trained", ctypes.c_int32),
                ("dev", ctypes.c_void_p)]


class NbLayout(ctypes.Structure):
    _fields_ = [("total_bytes", ctypes.c_size_t), ("padded_features", ctypes.c_int32),
                ("form_rows", ctypes.c_int32),
                ("off_status", ctypes.c_size_t), ("off_class_totals", ctypes.c_size_t),
                ("off_class_sums", ctypes.c_size_t), ("off_counts", ctypes.c_size_t),
                ("off_log_theta", ctypes.c_size_t), ("off_log_1m_theta", ctypes.c_size_t),
                ("off_weight", ctypes.c_size_t), ("off_bias", ctypes.c_size_t),
                ("off_form_f32", ctypes.c_size_t), ("off_form_bf16", ctypes.c_size_t),
                ("off_form_bias", ctypes.c_size_t), ("alpha", ctypes.c_double),
                ("off_sumsq", ctypes.c_size_t), ("off_mean", ctypes.c_size_t), ("off_var", ctypes.c_size_t),
                ("off_form2_f32", ctypes.c_size_t),
                ("off_form2_bf16", ctypes.c_size_t), ("off_epsilon", ctypes.c_size_t)]


class NbGroup(ctypes.Structure):
    _fields_ = [("model", ctypes.c_int32), ("reserved", ctypes.c_int32), ("x", ctypes.c_void_p),
                ("n", ctypes.c_int64), ("ld", ctypes.c_int64), ("labels", ctypes.c_void_p),
                ("log_post", ctypes.c_void_p), ("scores", ctypes.c_void_p)]


class NbGroupPlanInfo(ctypes.Structure):
    _fields_ = [("tile_rows", ctypes.c_int32), ("n_items", ctypes.c_int32), ("grid", ctypes.c_int32),
                ("tuned", ctypes.c_int32), ("n_files", ctypes.c_int64), ("rows_per_block", ctypes.c_int32),
                ("lds_bytes", ctypes.c_int32), ("schedule", ctypes.c_int32),
                ("staged", ctypes.c_int32)]


class NbRequest(ctypes.Structure):
    _fields_ = [("model", ctypes.c_int32), ("status", ctypes.c_int32), ("x", ctypes.c_void_p),
                ("n", ctypes.c_int64), ("arrival_s", ctypes.c_double), ("labels_host", ctypes.c_void_p),
                ("log_post_host", ctypes.c_void_p), ("done_s", ctypes.c_double)]


class NbServeCfg(ctypes.Structure):
    _fields_ = [("arena", ctypes.c_void_p), ("arena_bytes", ctypes.c_size_t),
                ("max_batch_requests", ctypes.c_int32), ("n_streams", ctypes.c_int32),
                ("xtype", ctypes.c_int32), ("wtype", ctypes.c_int32), ("flags", ctypes.c_int32),
                ("reserved", ctypes.c_int32), ("sim_batch_s", ctypes.c_double),
                ("sim_bytes_per_s", ctypes.c_double)]


class NbServeStats(ctypes.Structure):
    _fields_ = [("p50_s", ctypes.c_double), ("p99_s", ctypes.c_double), ("mean_s", ctypes.c_double),
                ("max_s", ctypes.c_double), ("makespan_s", ctypes.c_double), ("files_per_s", ctypes.c_double),
                ("bytes_per_s", ctypes.c_double), ("served", ctypes.c_int64), ("rejected", ctypes.c_int64),
                ("batches", ctypes.c_int64), ("peak_arena_bytes", ctypes.c_int64),
                ("max_in_flight", ctypes.c_int32), ("reserved", ctypes.c_int32)]


_i32, _i64, _sz, _vp, _d = ctypes.c_int32, ctypes.c_int64, ctypes.c_size_t, ctypes.c_void_p, ctypes.c_double
_PM = ctypes.POINTER(NbModel)
_PG = ctypes.POINTER(NbGroup)

# name -> (restype, argtypes); every symbol include/nb.h declares
SIGNATURES = {
    "nb_version": (ctypes.c_char_p, []),
    "nb_last_error": (ctypes.c_char_p, []),
    "nb_model_bytes": (_sz, [_i32, _i32]),
    "nb_model_layout": (ctypes.c_int, [_i32, _i32, ctypes.POINTER(NbLayout)]),
    "nb_train_workspace_bytes": (_sz, [_i32, _i32, _i64, _i32]),
    "nb_train": (ctypes.c_int, [_PM, _vp, _i32, _i64, _i64, _vp, _d, _i32, _vp, _sz, _i32, _vp]),
    "nb_model_status": (ctypes.c_int, [_PM, _vp]),
    "nb_score": (ctypes.c_int, [_PM, _vp, _i32, _i64, _i64, _i32, _vp, _vp, _vp, _vp]),
    "nb_quantize_fp8": (ctypes.c_int, [_vp, _i64, _i32, _i64, _vp, _i64, _vp]),
    "nb_select_features": (ctypes.c_int, [_PM, _i32, _i32, _vp, _i64, _vp]),
    "nb_model_select_workspace_bytes": (_sz, [_i32, _i32]),
    "nb_model_select": (ctypes.c_int, [_PM, _vp, _i32, _d, _PM, _vp, _sz, _i32, _vp]),
    "nb_gather_features": (ctypes.c_int, [_vp, _i32, _i64, _i32, _i64, _vp, _i32, _vp, _i64, _vp, _vp]),
    "nb_model_expand": (ctypes.c_int, [_PM, _vp, _PM, _i32, _vp]),
    "nb_route_groups": (ctypes.c_int, [_vp, _i32, _i32, _i32, _vp]),
    "nb_score_groups_workspace_bytes": (_sz, [_PM, _i32, _PG, _i32, _i32, _i32, _i32]),
    "nb_score_groups": (ctypes.c_int, [_PM, _i32, _PG, _i32, _i32, _i32, _i32, _vp, _sz, _vp]),
    "nb_score_groups_static": (ctypes.c_int, [_PM, _i32, _PG, _i32, _i32, _i32, _i32, _vp]),
    "nb_group_plan_create": (ctypes.c_int, [_PM, _i32, _PG, _i32, _i32, _i32, _i32, _i32, _vp,
                                            ctypes.POINTER(_vp)]),
    "nb_group_plan_update": (ctypes.c_int, [_vp, _PM, _i32, _PG, _i32, _vp]),
    "nb_group_plan_launch": (ctypes.c_int, [_vp, _vp]),
    "nb_group_plan_query": (ctypes.c_int, [_vp, ctypes.POINTER(NbGroupPlanInfo)]),
    "nb_group_plan_destroy": (ctypes.c_int, [_vp]),
    "nb_serve": (ctypes.c_int, [_PM, _i32, ctypes.POINTER(NbRequest), _i64, ctypes.POINTER(NbServeCfg),
                                ctypes.POINTER(NbServeStats)]),
    "nb_probe_sink_words": (_i32, []),
    "nb_probe_read": (ctypes.c_int, [_vp, _i64, _vp, _vp]),
}

_lib = None


def load():
    """Load libnbgpu.so (built in-tree by paper_1905_13746_amd.build)."""
    global _lib
    if _lib is not None:
        return _lib
    if not os.path.exists(LIB_PATH):
        raise ImportError(f"{LIB_PATH} is not built: run `python -m paper_1905_13746_amd.build` "
                          "(there is no fallback implementation)")
    lib = ctypes.CDLL(LIB_PATH)
    for name, (res, args) in SIGNATURES.items():
        fn = getattr(lib, name)
        fn.restype = res
        fn.argtypes = args
    _lib = lib
    return lib


class NBError(RuntimeError):
    def __init__(self, code: int, where: str):
        msg = load().nb_last_error().decode(errors="replace")
        super().__init__(f"{where}: {STATUS_NAMES.get(code, code)}: {msg}")
        self.code = code


def check(code: int, where: str):
    if code != NB_OK:
        raise NBError(code, where)
    return code
