"""ctypes view of the C ABI declared in include/dmatch.h (argument marshalling only).

The shared library is built in place by ``paper_1601_06274_amd.build``.  Loading
fails loudly when it is missing: there is no fallback implementation.
"""
from __future__ import annotations

import ctypes
import os

HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(HERE, "libdmatch.so")

DM_OK = 0
DM_F32 = 0
DM_F16 = 1
DM_MINORANT_ITERATIVE = 0
DM_MINORANT_NAIVE = 1
DM_MINORANT_HIERARCHICAL = 2

PROF_KINDS = {"sweep_h": 0, "sweep_v": 1, "sweep_final": 2, "sweep_opt": 3, "bounds": 4, "cost_volume": 5,
              "refine_linearize": 6, "refine_iter": 7, "other": 8, "adjoint_h": 9, "adjoint_v": 10,
              "adjoint_final": 11, "record_h": 12, "record_v": 13, "census": 14, "lr_check": 15, "flow_cost": 16,
              "flow_project": 17}

STATUS_NAMES = {
    0: "DM_OK", -1: "DM_ERR_NULL", -2: "DM_ERR_SHAPE", -3: "DM_ERR_PARAM", -4: "DM_ERR_DTYPE",
    -5: "DM_ERR_WORKSPACE", -6: "DM_ERR_UNSUPPORTED", -7: "DM_ERR_HIP",
}


class DmShape(ctypes.Structure):
    _fields_ = [("W", ctypes.c_int), ("H", ctypes.c_int), ("K", ctypes.c_int)]


class DmCostParams(ctypes.Structure):
    _fields_ = [("window", ctypes.c_int), ("trunc", ctypes.c_float), ("lambda_pw", ctypes.c_float),
                ("contrast_sigma", ctypes.c_float)]


class DmDiscreteParams(ctypes.Structure):
    _fields_ = [("n_iters", ctypes.c_int), ("n_half_steps", ctypes.c_int), ("trunc_T", ctypes.c_int),
                ("minorant", ctypes.c_int), ("max_pass", ctypes.c_int), ("gamma", ctypes.c_float * 8),
                ("warm_start", ctypes.c_int), ("tile_lanes", ctypes.c_int), ("labels_per_lane", ctypes.c_int),
                ("tile_lanes_v", ctypes.c_int), ("labels_per_lane_v", ctypes.c_int), ("keep_checkpoints", ctypes.c_int),
                ("recompute_selections", ctypes.c_int)]


class DmRefineParams(ctypes.Structure):
    _fields_ = [("C", ctypes.c_float), ("eps", ctypes.c_float), ("delta", ctypes.c_float), ("h", ctypes.c_float),
                ("tau", ctypes.c_float), ("sigma", ctypes.c_float), ("n_warps", ctypes.c_int), ("n_iters", ctypes.c_int),
                ("keep_tape", ctypes.c_int)]


class DmFlowShape(ctypes.Structure):
    _fields_ = [("W", ctypes.c_int), ("H", ctypes.c_int), ("K1", ctypes.c_int), ("K2", ctypes.c_int),
                ("off1", ctypes.c_int), ("off2", ctypes.c_int)]


class DmInstance(ctypes.Structure):
    _fields_ = [("s", DmShape), ("cost", ctypes.c_void_p), ("w_h", ctypes.c_void_p), ("w_v", ctypes.c_void_p),
                ("labels", ctypes.c_void_p), ("dual", ctypes.c_void_p), ("u", ctypes.c_void_p),
                ("bounds", ctypes.c_void_p), ("minmarg", ctypes.c_void_p)]


class DmGradInstance(ctypes.Structure):
    _fields_ = [("s", DmShape)] + [(k, ctypes.c_void_p) for k in (
        "cost", "w_h", "w_v", "labels", "dual", "minmarg", "bounds", "u", "grad_minmarg", "grad_bounds", "grad_u",
        "grad_cost", "grad_w_h", "grad_w_v")]


class DmError(RuntimeError):
    def __init__(self, fn: str, status: int, detail: str):
        super().__init__(f"{fn} failed: {STATUS_NAMES.get(status, status)}: {detail}")
        self.status = status


_lib = None

# (name, restype, argtypes) for every exported symbol declared in include/dmatch.h
_VP = ctypes.c_void_p
_SIGNATURES = [
    ("dm_build_cost_volume", ctypes.c_int,
     [_VP, _VP, DmShape, ctypes.POINTER(DmCostParams), ctypes.c_int, _VP, _VP, _VP, _VP]),
    ("dm_build_cost_volume_census", ctypes.c_int,
     [_VP, _VP, DmShape, ctypes.POINTER(DmCostParams), ctypes.c_int, ctypes.c_int, _VP, _VP, _VP, _VP]),
    ("dm_lr_check", ctypes.c_int,
     [_VP, _VP, ctypes.c_int, ctypes.c_int, ctypes.c_float, ctypes.c_float, _VP, _VP]),
    ("dm_solve_discrete_workspace", ctypes.c_size_t, [DmShape, ctypes.c_int, ctypes.POINTER(DmDiscreteParams)]),
    ("dm_solve_discrete", ctypes.c_int,
     [_VP, ctypes.c_int, _VP, _VP, DmShape, ctypes.POINTER(DmDiscreteParams), _VP, _VP, _VP, _VP, _VP, _VP,
      ctypes.c_size_t, _VP]),
    ("dm_solve_discrete_noalloc_limit", ctypes.c_size_t, []),
    ("dm_solve_discrete_noalloc", ctypes.c_int,
     [_VP, ctypes.c_int, _VP, _VP, DmShape, ctypes.POINTER(DmDiscreteParams), _VP, _VP, _VP, _VP, _VP, _VP]),
    ("dm_default_tile", ctypes.c_int, [ctypes.c_int, ctypes.POINTER(ctypes.c_int), ctypes.POINTER(ctypes.c_int)]),
    ("dm_autotune_tiles", ctypes.c_int, [DmShape, ctypes.c_int, ctypes.POINTER(DmDiscreteParams), _VP]),
    ("dm_solve_discrete_backward_workspace", ctypes.c_size_t, [DmShape, ctypes.POINTER(DmDiscreteParams)]),
    ("dm_solve_discrete_backward", ctypes.c_int,
     [_VP, _VP, _VP, ctypes.c_int, _VP, _VP, DmShape, ctypes.POINTER(DmDiscreteParams), _VP, _VP,
      ctypes.c_size_t, _VP, _VP, _VP, ctypes.c_int, _VP, ctypes.c_size_t, _VP]),
    ("dm_refine_continuous_workspace", ctypes.c_size_t, [DmShape, ctypes.POINTER(DmRefineParams)]),
    ("dm_refine_continuous", ctypes.c_int,
     [_VP, ctypes.c_int, _VP, _VP, _VP, DmShape, ctypes.POINTER(DmRefineParams), _VP, _VP, ctypes.c_size_t, _VP]),
    ("dm_build_flow_cost_volume", ctypes.c_int,
     [_VP, _VP, DmFlowShape, ctypes.POINTER(DmCostParams), ctypes.c_int, _VP, _VP, _VP, _VP]),
    ("dm_flow_project", ctypes.c_int, [_VP, ctypes.c_int, DmFlowShape, _VP, _VP, _VP]),
    ("dm_refine_flow_workspace", ctypes.c_size_t, [DmFlowShape, ctypes.POINTER(DmRefineParams)]),
    ("dm_refine_flow", ctypes.c_int,
     [_VP, ctypes.c_int, _VP, _VP, _VP, _VP, DmFlowShape, ctypes.POINTER(DmRefineParams), _VP, _VP, _VP,
      ctypes.c_size_t, _VP]),
    ("dm_profiler_enable", ctypes.c_int, [ctypes.c_uint]),
    ("dm_profiler_query", ctypes.c_int,
     [ctypes.c_int, ctypes.POINTER(ctypes.c_longlong), ctypes.POINTER(ctypes.c_double), ctypes.POINTER(ctypes.c_double)]),
    ("dm_refine_continuous_backward_workspace", ctypes.c_size_t, [DmShape, ctypes.POINTER(DmRefineParams)]),
    ("dm_refine_continuous_backward", ctypes.c_int,
     [_VP, _VP, ctypes.c_int, _VP, _VP, DmShape, ctypes.POINTER(DmRefineParams), _VP, ctypes.c_size_t, _VP, _VP, _VP,
      ctypes.c_int, _VP, ctypes.c_size_t, _VP]),
    ("dm_plan_batched", ctypes.c_int,
     [ctypes.POINTER(DmInstance), ctypes.c_int, ctypes.c_int, ctypes.POINTER(DmDiscreteParams),
      ctypes.POINTER(DmRefineParams), ctypes.POINTER(ctypes.c_void_p)]),
    ("dm_plan_batched_grad", ctypes.c_int,
     [ctypes.POINTER(DmGradInstance), ctypes.c_int, ctypes.c_int, ctypes.POINTER(DmDiscreteParams),
      ctypes.POINTER(DmRefineParams), ctypes.c_int, ctypes.POINTER(ctypes.c_void_p)]),
    ("dm_run_batched", ctypes.c_int, [_VP, _VP]),
    ("dm_plan_device_bytes", ctypes.c_size_t, [_VP]),
    ("dm_plan_destroy", None, [_VP]),
    ("dm_status_string", ctypes.c_char_p, [ctypes.c_int]),
    ("dm_last_error_message", ctypes.c_char_p, []),
    ("dm_version", ctypes.c_char_p, []),
]


def exported_names():
    return [n for n, _, _ in _SIGNATURES]


def lib():
    """Load libdmatch.so (once).  Raises if it has not been built."""
    global _lib
    if _lib is None:
        if not os.path.exists(LIB_PATH):
            raise ImportError(f"{LIB_PATH} is missing: build it with `python -m paper_1601_06274_amd.build`")
        L = ctypes.CDLL(LIB_PATH)
        for name, res, args in _SIGNATURES:
            if hasattr(L, name):
                f = getattr(L, name)
                f.restype = res
                f.argtypes = args
        _lib = L
    return _lib


def check(fn: str, status: int):
    if status != DM_OK:
        detail = lib().dm_last_error_message().decode(errors="replace")
        raise DmError(fn, status, detail)
