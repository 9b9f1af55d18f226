"""ctypes loader for libstereo.so (the gfx950 HIP library).

There is no fallback: if the library is missing or cannot be loaded this
module raises, so nothing can silently run on another path.
"""
from __future__ import annotations

import ctypes
import os
from ctypes import (POINTER, Structure, c_char_p, c_double, c_float, c_int,
                    c_int32, c_int64, c_size_t, c_void_p)

import torch  # noqa: F401  -- load torch's HIP runtime first; the library shares it

LIB_PATH = os.path.join(os.path.dirname(os.path.abspath(__file__)), "libstereo.so")

OK = 0
STATUS = {0: "ok", 1: "invalid argument", 2: "unsupported", 3: "workspace too small",
          4: "HIP error", 5: "not converged"}
U8, F32 = 0, 1


class StereoParams(Structure):
    _fields_ = [
        ("width", c_int32), ("height", c_int32),
        ("pitch_ref", c_int64), ("pitch_tar", c_int64),
        ("dtype", c_int),
        ("num_disp", c_int32), ("delta_p", c_float),
        ("perspective", c_int32), ("plane", c_double * 3),
        ("ncc_radius", c_int32), ("bil_radius", c_int32),
        ("sigma_s", c_float), ("sigma_r", c_float),
        ("lr_delta", c_float), ("lr_check", c_int32),
        ("softargmin_T", c_float),
    ]


class RoadFit(Structure):
    _fields_ = [
        ("psi", c_double), ("alpha0", c_double), ("alpha1", c_double),
        ("e_min", c_double), ("plane", c_double * 3), ("n_points", c_double),
        ("iters", c_int32), ("converged", c_int32), ("flat", c_int32),
        ("pad_", c_int32),
    ]


class PlaneState(Structure):
    _fields_ = [("plane", c_double * 3), ("psi", c_double), ("frames", c_int32),
                ("pad_", c_int32)]


class BatchItem(Structure):
    _fields_ = [("plan", c_void_p), ("ref", c_void_p), ("tar", c_void_p),
                ("dint_R", c_void_p), ("valid", c_void_p), ("disp", c_void_p)]


class StereoError(RuntimeError):
    def __init__(self, status, message):
        super().__init__(f"{STATUS.get(status, status)}: {message}")
        self.status = status


# name -> (restype, argtypes); every function in include/stereo.h
SIGNATURES = {
    "stereo_status_string": (c_char_p, [c_int]),
    "stereo_last_error": (c_char_p, []),
    "stereo_version": (c_char_p, []),
    "stereo_plan_create": (c_int, [POINTER(StereoParams), POINTER(c_void_p)]),
    "stereo_plan_destroy": (c_int, [c_void_p]),
    "stereo_plan_workspace_bytes": (c_int, [c_void_p, POINTER(c_size_t)]),
    "stereo_plan_get_params": (c_int, [c_void_p, POINTER(StereoParams)]),
    "stereo_plan_set_tuning": (c_int, [c_void_p, c_char_p, c_int32]),
    "stereo_plan_get_tuning": (c_int, [c_void_p, c_char_p, POINTER(c_int32)]),
    "stereo_warp": (c_int, [c_void_p, c_void_p, c_void_p, c_void_p]),
    "stereo_cost_volume": (c_int, [c_void_p, c_void_p, c_void_p, c_void_p, c_void_p,
                                   c_void_p, c_size_t, c_void_p]),
    "stereo_bilateral_aggregate": (c_int, [c_void_p, c_void_p, c_int, c_int64, c_void_p,
                                           c_void_p, c_void_p]),
    "stereo_wta_subpixel": (c_int, [c_void_p, c_void_p, c_void_p, c_void_p, c_void_p]),
    "stereo_lr_check": (c_int, [c_void_p, c_void_p, c_void_p, c_void_p, c_void_p,
                                c_void_p, c_void_p]),
    "stereo_match": (c_int, [c_void_p, c_void_p, c_void_p, c_void_p, c_void_p, c_void_p,
                             c_void_p, c_void_p, c_void_p, c_size_t, c_void_p]),
    "stereo_match_profiled": (c_int, [c_void_p, c_void_p, c_void_p, c_void_p, c_void_p,
                                      c_void_p, c_void_p, c_void_p, c_void_p, c_size_t,
                                      c_void_p, c_void_p]),
    "stereo_road_transform": (c_int, [c_void_p, c_void_p, c_void_p, c_double, c_double,
                                      c_double, c_int32, c_float, c_void_p, c_void_p,
                                      c_void_p, c_size_t, c_void_p]),
    "stereo_road_transform_noalloc": (c_int, [c_void_p, c_void_p, c_void_p, c_double,
                                              c_double, c_double, c_int32, c_float, c_void_p,
                                              c_void_p, c_void_p]),
    "stereo_match_tracked": (c_int, [c_void_p, c_void_p, c_void_p, c_void_p, c_void_p, c_void_p,
                                     c_void_p, c_void_p, c_void_p, c_void_p, c_size_t,
                                     c_void_p]),
    "stereo_road_transform_tracked": (c_int, [c_void_p, c_void_p, c_void_p, c_double, c_double,
                                              c_int32, c_float, c_void_p, c_void_p, c_void_p,
                                              c_void_p, c_size_t, c_void_p]),
    "stereo_plan_set_homography": (c_int, [c_void_p, c_void_p]),
    "stereo_damage_mask": (c_int, [c_void_p, c_void_p, c_float, c_float, c_void_p, c_void_p]),
    "stereo_soft_forward": (c_int, [c_void_p, c_void_p, c_void_p, POINTER(c_double), c_void_p,
                                    c_void_p, c_void_p, c_size_t, c_void_p]),
    "stereo_backward": (c_int, [c_void_p, c_void_p, c_void_p, POINTER(c_double), c_void_p,
                                c_void_p, c_void_p, c_void_p, c_void_p, c_void_p, c_size_t,
                                c_void_p]),
    "stereo_backward_profiled": (c_int, [c_void_p, c_void_p, c_void_p, POINTER(c_double),
                                         c_void_p, c_void_p, c_void_p, c_void_p, c_void_p,
                                         c_void_p, c_size_t, c_void_p, c_void_p]),
    "stereo_photometric_l1": (c_int, [c_void_p, c_void_p, c_void_p, c_void_p, c_void_p,
                                      c_void_p, c_size_t, c_void_p]),
    "stereo_photometric_l1_bwd": (c_int, [c_void_p, c_void_p, c_void_p, c_void_p, c_double,
                                          c_void_p, c_void_p, c_void_p, c_void_p, c_size_t,
                                          c_void_p]),
    "stereo_batch_create": (c_int, [POINTER(BatchItem), c_int32, POINTER(c_void_p)]),
    "stereo_batch_workspace_bytes": (c_int, [c_void_p, POINTER(c_size_t)]),
    "stereo_batch_set_tuning": (c_int, [c_void_p, c_char_p, c_int32]),
    "stereo_batch_get_tuning": (c_int, [c_void_p, c_char_p, POINTER(c_int32)]),
    "stereo_submit_batch": (c_int, [c_void_p, c_void_p, c_size_t, c_void_p]),
    "stereo_submit_batch_profiled": (c_int, [c_void_p, c_void_p, c_size_t, c_void_p, c_void_p]),
    "stereo_batch_instantiate": (c_int, [c_void_p, c_void_p, c_size_t, c_void_p]),
    "stereo_batch_launch": (c_int, [c_void_p, c_void_p]),
    "stereo_batch_destroy": (c_int, [c_void_p]),
    "stereo_plan_autotune": (c_int, [c_void_p, c_void_p, c_void_p, c_void_p, c_size_t, c_void_p,
                                     c_char_p, c_int32, POINTER(c_double)]),
    "stereo_batch_autotune": (c_int, [c_void_p, c_void_p, c_size_t, c_void_p, c_char_p, c_int32,
                                      POINTER(c_double)]),
}

_lib = None


def load():
    global _lib
    if _lib is not None:
        return _lib
    if not os.path.exists(LIB_PATH):
        raise RuntimeError(
            f"{LIB_PATH} not found: build it with `python -m paper_1904_06017_amd.build` "
            "(there is no CPU fallback)")
    lib = ctypes.CDLL(LIB_PATH, mode=ctypes.RTLD_GLOBAL)
    for name, (res, args) in SIGNATURES.items():
        f = getattr(lib, name)
        f.restype = res
        f.argtypes = args
    _lib = lib
    return lib


def check(status):
    if status != OK:
        msg = load().stereo_last_error().decode(errors="replace")
        raise StereoError(status, msg)
    return status
