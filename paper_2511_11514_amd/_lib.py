"""ctypes declarations of libct.so (the C ABI in include/ct.h).

Loading fails loudly if the library has not been built: there is no fallback
implementation of any entry point.
"""
from __future__ import annotations

import ctypes
import os
from ctypes import POINTER, c_char_p, c_double, c_float, c_int32, c_int64, c_size_t, c_uint32, c_void_p

HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(HERE, "libct.so")

CT_OK = 0
CT_WARN_NOT_CONVERGED = 1
CT_E_ARG = -1
CT_E_SHAPE = -2
CT_E_NONFINITE = -3
CT_E_WORKSPACE = -4
CT_E_HIP = -5
CT_E_UNSUPPORTED = -6
CT_E_CAPTURE = -7
CT_E_DEVICE = -8

CT_DEBIAS = 1
CT_GRAD_W = 2
CT_VALUE = 4
CT_WARM_START = 8
CT_REF_CACHED = 16
CT_SAFE_LSE = 32
CT_ONE_STREAM = 64
CT_PERSISTENT = 128
CT_FUSED = 256
CT_UNFUSED = 512
CT_DIFFERENCE = 1024
CT_TINY = 2048
CT_MESH = 4096

CT_DYN_DOUBLE_INTEGRATOR = 0
CT_DYN_UNICYCLE = 1
CT_FLOW_SINKHORN = 0
CT_FLOW_SVGD = 1
CT_FLOW_SVGD_GRID = 2


class SinkhornOpts(ctypes.Structure):
    _fields_ = [("d", c_int32), ("iters", c_int32), ("eps", c_float), ("flags", c_uint32)]


class GMMDesc(ctypes.Structure):
    _fields_ = [("K", c_int32), ("weights", c_void_p), ("means", c_void_p), ("sigmas", c_void_p),
                ("floor", c_float)]


class GridDesc(ctypes.Structure):
    _fields_ = [("n", c_int32 * 3), ("lo", c_float * 3), ("hi", c_float * 3), ("u", c_void_p),
                ("floor", c_float)]


class PlanProblem(ctypes.Structure):
    _fields_ = [("dynamics", c_int32), ("d", c_int32), ("T", c_int64), ("dt", c_double),
                ("s0", POINTER(c_double))]


class PlanOpts(ctypes.Structure):
    _fields_ = [("flow", c_int32), ("outer", c_int32), ("step", c_double), ("Q", POINTER(c_double)),
                ("R", POINTER(c_double)), ("sk", SinkhornOpts), ("svgd_h", c_float),
                ("grid", POINTER(GridDesc))]


class CtError(RuntimeError):
    def __init__(self, fn: str, code: int, msg: str):
        super().__init__(f"{fn} failed with status {code}: {msg}")
        self.code = code


_lib = None

P = c_void_p
PD = POINTER(c_double)
PI64 = POINTER(c_int64)

_SIGS = {
    "ct_last_error": (c_char_p, []),
    "ct_version": (c_char_p, []),
    "ct_sinkhorn_workspace_size": (c_size_t, [c_int64, c_int64, POINTER(SinkhornOpts)]),
    "ct_sinkhorn_grad": (c_int32, [P, c_int64, P, P, c_int64, POINTER(SinkhornOpts), P, P, P, P, P,
                                   P, P, c_size_t, P]),
    "ct_sinkhorn_static_scratch_bytes": (c_size_t, []),
    "ct_sinkhorn_grad_static": (c_int32, [P, c_int64, P, P, c_int64, POINTER(SinkhornOpts), P, P,
                                          P, P, P, P, P]),
    "ct_status_sync": (c_int32, [P, c_float, POINTER(c_uint32), POINTER(c_uint32),
                                 POINTER(c_float), P]),
    "ct_sinkhorn_batched_workspace_size": (c_size_t, [c_int32, PI64, PI64, POINTER(SinkhornOpts)]),
    "ct_sinkhorn_batched_prepare": (c_int32, [c_int32, PI64, PI64, POINTER(SinkhornOpts), P,
                                              c_size_t, P]),
    "ct_sinkhorn_grad_batched": (c_int32, [c_int32, PI64, PI64, P, P, P, POINTER(SinkhornOpts), P,
                                           P, P, P, c_size_t, P]),
    "ct_svgd_workspace_size": (c_size_t, [c_int64, c_int32]),
    "ct_svgd_grad": (c_int32, [P, c_int64, c_int32, POINTER(GMMDesc), c_float, P, P, P, P,
                               c_size_t, P]),
    "ct_svgd_grad_score": (c_int32, [P, c_int64, c_int32, P, c_float, P, P, P, c_size_t, P]),
    "ct_grid_score": (c_int32, [P, c_int64, c_int32, POINTER(GridDesc), P, P]),
    "ct_grid_samples_workspace_size": (c_size_t, [POINTER(GridDesc), c_int32]),
    "ct_grid_samples": (c_int32, [POINTER(GridDesc), c_int32, P, P, PI64, P, c_size_t, P]),
    "ct_lqr_track": (c_int32, [c_int64, c_int32, c_int32, c_double, PD, PD, PD, PD, PD, PD, PD]),
    "ct_plan_workspace_size": (c_size_t, [POINTER(PlanProblem), POINTER(PlanOpts), c_int64]),
    "ct_plan": (c_int32, [POINTER(PlanProblem), POINTER(PlanOpts), P, P, c_int64, POINTER(GMMDesc),
                          PD, PD, PD, P, c_size_t, P]),
    "ct_plan_ensemble_workspace_size": (c_size_t, [POINTER(PlanProblem), POINTER(PlanOpts),
                                                   c_int32, c_int64, c_int32]),
    "ct_plan_ensemble": (c_int32, [POINTER(PlanProblem), POINTER(PlanOpts), c_int32, P, P, c_int64,
                                   PD, PD, PD, POINTER(c_int32), P, c_size_t, P]),
    "ct_autotune_sinkhorn": (c_int32, [c_int64, c_int64, POINTER(SinkhornOpts), P, c_size_t, P]),
    "ct_tuning_count": (c_int32, []),
    "ct_tuning_entry": (c_int32, [c_int32, POINTER(c_int32)]),
    "ct_tuning_save": (c_int32, [c_char_p]),
    "ct_tuning_load": (c_int32, [c_char_p]),
    "ct_tuning_clear": (None, []),
    "ct_profile_enable": (c_int32, [c_int32]),
    "ct_profile_count": (c_int32, []),
    "ct_profile_read": (c_int32, [c_int32, POINTER(c_int32), PD, POINTER(c_float)]),
    "ct_profile_clear": (None, []),
    "ct_probe_workspace_size": (c_size_t, []),
    "ct_probe_alu_rates": (c_int32, [PD, P, c_size_t, P]),
}


def lib() -> ctypes.CDLL:
    """The loaded libct.so (raises if it has not been built)."""
    global _lib
    if _lib is None:
        if not os.path.exists(LIB_PATH):
            raise ImportError(f"libct.so not found at {LIB_PATH}: build it with "
                              "`python -m paper_2511_11514_amd.build` (no fallback exists)")
        L = ctypes.CDLL(LIB_PATH)
        for name, (res, args) in _SIGS.items():
            fn = getattr(L, name)
            fn.restype = res
            fn.argtypes = args
        _lib = L
    return _lib


def check(fn: str, status: int) -> None:
    if status != CT_OK:
        msg = lib().ct_last_error().decode(errors="replace")
        raise CtError(fn, status, msg)
