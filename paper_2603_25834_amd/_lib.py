"""ctypes binding of ``libaslam.so`` (the C-ABI declared in include/aslam.h).

Argument marshalling only: every step of the hot path runs in the library's
HIP kernels.  Loading fails loudly when the library has not been built.
"""
from __future__ import annotations

import ctypes
import os

_HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(_HERE, "libaslam.so")

ASL_OK = 0
ERRORS = {-1: "ASL_EINVAL", -2: "ASL_ENOMEM", -3: "ASL_EHIP", -4: "ASL_ESTATE", -5: "ASL_ENOTIMPL"}

FORM_PLAIN = 0
FORM_FUSED = 1

FIELD_BELIEF, FIELD_POSE, FIELD_EST, FIELD_COV, FIELD_RHO_Q, FIELD_HIT_CELL, FIELD_ENTROPY_Q, \
    FIELD_STEP, FIELD_FLAGS, FIELD_TERMS, FIELD_COUNTERS, FIELD_U_PREV, FIELD_VISIT_LAST, FIELD_DRAWS, \
    FIELD_MATCH = range(15)


class AslamError(RuntimeError):
    def __init__(self, code: int, msg: str):
        super().__init__(f"{ERRORS.get(code, code)}: {msg}")
        self.code = code


class EnvConfig(ctypes.Structure):
    _fields_ = [
        ("n_rays", ctypes.c_int32), ("loop_closure", ctypes.c_int32),
        ("lc_gap", ctypes.c_int32), ("episode_len", ctypes.c_int32),
        ("cell_m", ctypes.c_float), ("r_max_m", ctypes.c_float), ("dt", ctypes.c_float),
        ("v_max", ctypes.c_float), ("w_max", ctypes.c_float),
        ("sigma_x", ctypes.c_float), ("sigma_y", ctypes.c_float), ("sigma_th", ctypes.c_float),
        ("var0_xy", ctypes.c_float), ("var0_th", ctypes.c_float),
        ("lc_cell_m", ctypes.c_float), ("lc_radius_m", ctypes.c_float), ("lc_sigma_m", ctypes.c_float),
        ("l_hit", ctypes.c_float), ("l_miss", ctypes.c_float), ("l_clamp", ctypes.c_float),
        ("w_entropy", ctypes.c_float), ("w_dopt", ctypes.c_float), ("lambda_col", ctypes.c_float),
        ("fov_steps", ctypes.c_int32), ("reward_mode", ctypes.c_int32),
        ("r_min_m", ctypes.c_float), ("range_sigma_m", ctypes.c_float), ("range_quant_m", ctypes.c_float),
        ("d_crash_m", ctypes.c_float), ("d_full_m", ctypes.c_float),
        ("lambda_explore", ctypes.c_float), ("lambda_abs", ctypes.c_float), ("lambda_delta", ctypes.c_float),
        ("u_hi", ctypes.c_float), ("kappa", ctypes.c_float),
        ("noise_seed", ctypes.c_uint64),
        ("slam_backend", ctypes.c_int32), ("lag_len", ctypes.c_int32), ("gn_iters", ctypes.c_int32),
        ("csm_W", ctypes.c_int32), ("csm_V", ctypes.c_int32), ("csm_step_xy_q", ctypes.c_int32),
        ("csm_step_h", ctypes.c_int32), ("scan_sigma_xy_m", ctypes.c_float), ("scan_sigma_th", ctypes.c_float),
        ("int_weight_floor", ctypes.c_float),
    ]


class CsmConfig(ctypes.Structure):
    _fields_ = [("W", ctypes.c_int32), ("V", ctypes.c_int32), ("step_xy_q", ctypes.c_int32), ("step_h", ctypes.c_int32)]


class ExecConfig(ctypes.Structure):
    _fields_ = [(n, ctypes.c_int32) for n in ("form", "threads", "band_rows", "grid", "record_rays", "lds_bytes",
                                              "mark_seg")]


_P = ctypes.c_void_p
_I32 = ctypes.c_int32
_I64 = ctypes.c_int64
_U64 = ctypes.c_uint64

# name -> (restype, argtypes); every function of include/aslam.h
SIGNATURES = {
    "aslam_last_error": (ctypes.c_char_p, []),
    "aslam_device_info": (ctypes.c_int, [_P, _P]),
    "aslam_env_create": (ctypes.c_int, [ctypes.POINTER(EnvConfig), _I32, _P, ctypes.POINTER(_P)]),
    "aslam_env_destroy": (ctypes.c_int, [_P]),
    "aslam_env_world_words": (_I64, [_P]),
    "aslam_env_cells": (_I64, [_P]),
    "aslam_env_noise_width": (_I32, [_P]),
    "aslam_env_observe_bridge": (ctypes.c_int, [_P, _P, _P, _I32, _P, _P, _P, _I64, _I64, _P]),
    "aslam_env_visit_cells": (_I64, [_P]),
    "aslam_env_set_exec": (ctypes.c_int, [_P, ctypes.POINTER(ExecConfig)]),
    "aslam_env_get_exec": (ctypes.c_int, [_P, ctypes.POINTER(ExecConfig)]),
    "aslam_env_reset": (ctypes.c_int, [_P, _P, _P, _P, _P]),
    "aslam_env_step": (ctypes.c_int, [_P, _P, _P, _P, _P, _P, _P]),
    "aslam_env_observe": (ctypes.c_int, [_P, _P, _P, _I32, _P, _P, _P]),
    "aslam_env_read": (ctypes.c_int, [_P, _I32, _P, _P]),
    "aslam_env_graph_build": (ctypes.c_int, [_P, _I32, _P, _I64, _P, _I64, _P, _I64, _P, _I64, _P, _I64]),
    "aslam_env_graph_launch": (ctypes.c_int, [_P, _P]),
    "aslam_policy_num_params": (_I64, [_I32]),
    "aslam_policy_param_count": (_I64, [_P]),
    "aslam_policy_act_rnn": (ctypes.c_int, [_P, _P, _I32, _P, _P, _P, _I32, _P, _P, _P, _U64, _U64, _P, _P, _P, _P, _P,
                                            _P]),
    "aslam_policy_backward_seq": (ctypes.c_int, [_P, _P, _P, _P, _P, _I32, _I32, _P, _I32, _P, _P, _P, _P, _P, _P, _P,
                                                 _P, _P]),
    "aslam_policy_create": (ctypes.c_int, [ctypes.c_void_p, ctypes.POINTER(_P)]),
    "aslam_policy_destroy": (ctypes.c_int, [_P]),
    "aslam_policy_forward": (ctypes.c_int, [_P, _P, _P, _P, _P, _I32, _P, _P, _P]),
    "aslam_policy_backward": (ctypes.c_int, [_P, _P, _P, _P, _P, _I32, _P, _P, _P, _P, _P, _P, _P]),
    "aslam_policy_sample": (ctypes.c_int, [_P, _P, _P, _P, _U64, _U64, _I32, _P, _P, _P]),
    "aslam_permutation": (ctypes.c_int, [_I32, _U64, _U64, _P, _P, _I64, _P]),
    "aslam_permutation_work_bytes": (_I64, [_I32]),
    "aslam_policy_prepare": (ctypes.c_int, [_P, _P, _P]),
    "aslam_policy_forward_noalloc": (ctypes.c_int, [_P, _I32, _P, _P, _P, _I32, _P, _P, _P]),
    "aslam_policy_noalloc_limits": (_I64, [_P, _P]),
    "aslam_policy_backward_rows": (ctypes.c_int, [_P, _P, _P, _P, _P, _P, _I32, _P, _P, _P, _P, _P, _P, _P]),
    "aslam_policy_act": (ctypes.c_int, [_P, _P, _I32, _P, _P, _P, _I32, _P, _U64, _U64, _P, _P, _P, _P, _P]),
    "aslam_gather_rows": (ctypes.c_int, [_P, _I64, _P, _I32, _P, _P]),
    "aslam_gae": (ctypes.c_int, [_P, _P, _P, _P, _I32, _I32, ctypes.c_float, ctypes.c_float, _P, _P, _P]),
    "aslam_adam": (ctypes.c_int, [_P, _P, _P, _P, _I64, _I32, ctypes.c_float, ctypes.c_float, ctypes.c_float,
                                  ctypes.c_float, _P]),
    "aslam_slam_create": (ctypes.c_int, [ctypes.POINTER(_P)]),
    "aslam_slam_destroy": (ctypes.c_int, [_P]),
    "aslam_csm_match": (ctypes.c_int, [_P, _P, _P, _P, _I32, _I32, _P, _P, _I32, _P, ctypes.POINTER(CsmConfig), _P,
                                       _P]),
    "aslam_csm_factor": (ctypes.c_int, [_P, _P, _I32, ctypes.POINTER(CsmConfig), ctypes.c_double, ctypes.c_double,
                                        ctypes.c_double, ctypes.c_double, _P, _P, _P]),
    "aslam_csm_integrate": (ctypes.c_int, [_P, _P, _P, _P, _I32, _P, _P, _I32, _P, _I32, _I32, _P, ctypes.POINTER(CsmConfig),
                                            ctypes.c_double, _I32, _I32, _I32, _P, _P]),
    "aslam_fixedlag_solve": (ctypes.c_int, [_I32, _I32, _P, _P, _P, _P, _I32, _P, _P, _P]),
}

_lib = None


def lib():
    """Load libaslam.so; raises when it is missing (no fallback path exists)."""
    global _lib
    if _lib is None:
        if not os.path.exists(LIB_PATH):
            raise RuntimeError(f"{LIB_PATH} is not built; run __graft_entry__.build() first")
        L = ctypes.CDLL(LIB_PATH)
        for name, (res, args) in SIGNATURES.items():
            f = getattr(L, name)
            f.restype = res
            f.argtypes = args
        _lib = L
    return _lib


def check(rc: int) -> None:
    if rc != ASL_OK:
        msg = lib().aslam_last_error()
        raise AslamError(rc, msg.decode() if msg else "")


class PolicyConfig(ctypes.Structure):
    _fields_ = [("n_scan", ctypes.c_int32), ("max_batch", ctypes.c_int32), ("clip_eps", ctypes.c_float),
                ("c_value", ctypes.c_float), ("c_entropy", ctypes.c_float), ("recurrent", ctypes.c_int32),
                ("precision", ctypes.c_int32)]
