"""ctypes view of libinrf's C ABI (include/inrf.h): structures, signatures and
status handling.  Argument marshalling only; every step of the render path
runs in the library."""
from __future__ import annotations

import ctypes
import os
from ctypes import POINTER, c_char_p, c_int32, c_int64, c_uint32, c_uint64, c_void_p

HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(HERE, "libinrf.so")

INRF_OK, INRF_E_INVALID, INRF_E_SIZE, INRF_E_BUILD, INRF_E_DEVICE, INRF_E_UNSUPPORTED = 0, -1, -2, -3, -4, -5
INRF_F32, INRF_F16, INRF_BF16 = 0, 1, 2
PREC_FP32, PREC_FP16, PREC_BF16 = 0, 1, 2
MAX_LEVELS, FEATURES, SH_DIM, HIDDEN, OUT = 32, 2, 16, 64, 4
MAX_OBJECTS = 16
MAX_CAMERAS = 16

EXPORTED = [
    "inrf_last_error", "inrf_version", "inrf_psh_params_default", "inrf_build_psh", "inrf_build_psh_keys",
    "inrf_psh_levels", "inrf_psh_level", "inrf_psh_free", "inrf_brick_entries", "inrf_brick_index",
    "inrf_build_bvh", "inrf_bvh_get_info",
    "inrf_bvh_copy", "inrf_bvh_free", "inrf_workspace_size", "inrf_render", "inrf_render_profiled",
    "inrf_forward", "inrf_trace",
    "inrf_encode", "inrf_mlp", "inrf_batch_workspace_size", "inrf_render_batch", "inrf_scene_workspace_size", "inrf_render_scene", "inrf_backward_workspace_size",
    "inrf_backward", "inrf_adam", "inrf_render_nolf", "inrf_shade_nolf", "inrf_camera_rays",
    "inrf_render_static", "inrf_mlp_encoded", "inrf_scene_batch_workspace_size", "inrf_render_scene_batch",
]


class InrfError(RuntimeError):
    def __init__(self, code: int, msg: str):
        super().__init__(f"[{code}] {msg}")
        self.code = code


class PshParams(ctypes.Structure):
    _fields_ = [("seed", c_uint64), ("dilate", c_int32), ("load_pct", c_int32), ("bucket_keys", c_int32),
                ("n_random", c_int32), ("max_restarts", c_int32), ("n_threads", c_int32)]


class PshLevelInfo(ctypes.Structure):
    _fields_ = [("res", c_int32), ("mbar", c_int32), ("rbar", c_int32), ("restarts", c_int32),
                ("n_keys", c_int64), ("n_slots", c_int64), ("n_phi", c_int64)]


class BvhInfo(ctypes.Structure):
    _fields_ = [("n_nodes", c_int64), ("node_bytes", c_int64), ("tri_bytes", c_int64), ("depth", c_int32),
                ("max_leaf", c_int32), ("stack", c_int32), ("pad", c_int32)]


class LevelDesc(ctypes.Structure):
    _fields_ = [("res", c_int32), ("mbar", c_int32), ("rbar", c_int32), ("pad", c_int32),
                ("phi_offset", c_int64), ("slot_offset", c_int64)]


class ModelDesc(ctypes.Structure):
    _fields_ = [("n_levels", c_int32), ("table_dtype", c_int32), ("levels", LevelDesc * MAX_LEVELS),
                ("phi", c_void_p), ("table", c_void_p), ("weights", c_void_p), ("bvh_nodes", c_void_p),
                ("bvh_tris", c_void_p), ("n_tris", c_int64), ("bvh_stack", c_int32), ("bvh_n_nodes", c_int32)]


class CameraDesc(ctypes.Structure):
    _fields_ = [("origin", ctypes.c_float * 3), ("right", ctypes.c_float * 3), ("up", ctypes.c_float * 3),
                ("forward", ctypes.c_float * 3), ("tan_half_fov_y", ctypes.c_float), ("width", c_int32),
                ("height", c_int32)]


class InstanceDesc(ctypes.Structure):
    _fields_ = [("model", ctypes.c_void_p), ("scale", ctypes.c_float), ("rotation", ctypes.c_float * 9),
                ("translation", ctypes.c_float * 3)]


class CubesDesc(ctypes.Structure):
    _fields_ = [("base_res", c_int32), ("cube_res", c_int32), ("index", ctypes.c_void_p),
                ("density", ctypes.c_void_p), ("diffuse", ctypes.c_void_p), ("n_cubes", c_int64),
                ("step", ctypes.c_float), ("t_stop", ctypes.c_float), ("w_min", ctypes.c_float), ("pad", c_int32)]


class AdamParams(ctypes.Structure):
    _fields_ = [("lr", ctypes.c_float), ("beta1", ctypes.c_float), ("beta2", ctypes.c_float),
                ("eps", ctypes.c_float), ("step", c_int64), ("zero_grad", c_int32), ("lazy", c_int32)]


_lib = None


def _declare(lib):
    S = c_int32
    sig = {
        "inrf_last_error": (c_char_p, []),
        "inrf_version": (c_int32, []),
        "inrf_psh_params_default": (None, [POINTER(PshParams)]),
        "inrf_build_psh": (S, [c_void_p, c_int64, c_void_p, c_int64, c_int32, c_void_p, POINTER(PshParams),
                               POINTER(c_void_p)]),
        "inrf_build_psh_keys": (S, [c_int32, c_void_p, c_int64, POINTER(PshParams), POINTER(c_void_p)]),
        "inrf_psh_levels": (c_int32, [c_void_p]),
        "inrf_psh_level": (S, [c_void_p, c_int32, POINTER(PshLevelInfo), c_void_p, c_void_p, c_void_p]),
        "inrf_psh_free": (None, [c_void_p]),
        "inrf_brick_entries": (c_int64, [c_int32]),
        "inrf_brick_index": (S, [c_int32, c_void_p, c_int64, c_void_p]),
        "inrf_build_bvh": (S, [c_void_p, c_int64, c_void_p, c_int64, POINTER(c_void_p)]),
        "inrf_bvh_get_info": (S, [c_void_p, POINTER(BvhInfo)]),
        "inrf_bvh_copy": (S, [c_void_p, c_void_p, c_void_p]),
        "inrf_bvh_free": (None, [c_void_p]),
        "inrf_workspace_size": (c_int64, [c_int64]),
        "inrf_render": (S, [POINTER(ModelDesc), c_int32, POINTER(CameraDesc), c_void_p, c_void_p, c_void_p,
                            c_void_p, c_int64, c_void_p]),
        "inrf_render_profiled": (S, [POINTER(ModelDesc), c_int32, POINTER(CameraDesc), c_void_p, c_void_p,
                                     c_void_p, c_void_p, c_int64, c_void_p, c_void_p]),
        "inrf_forward": (S, [POINTER(ModelDesc), c_int32, c_void_p, c_void_p, c_int64, c_void_p, c_void_p,
                             c_void_p, c_void_p, c_int64, c_void_p]),
        "inrf_trace": (S, [POINTER(ModelDesc), c_void_p, c_void_p, c_int64, c_void_p, c_void_p, c_void_p]),
        "inrf_encode": (S, [POINTER(ModelDesc), c_void_p, c_int64, c_void_p, c_void_p, c_void_p]),
        "inrf_mlp": (S, [POINTER(ModelDesc), c_int32, c_void_p, c_int64, c_void_p, c_void_p]),
        "inrf_batch_workspace_size": (c_int64, [c_int32, c_int64]),
        "inrf_render_batch": (S, [POINTER(ModelDesc), c_int32, POINTER(CameraDesc), c_int32, c_void_p, c_void_p,
                                  c_void_p, c_void_p, c_int64, c_void_p]),
        "inrf_scene_workspace_size": (c_int64, [c_int32, c_int64]),
        "inrf_render_scene": (S, [POINTER(InstanceDesc), c_int32, c_int32, POINTER(CameraDesc), c_void_p, c_void_p,
                                  c_void_p, c_void_p, c_void_p, c_int64, c_void_p]),
        "inrf_backward_workspace_size": (c_int64, [POINTER(ModelDesc), c_int64]),
        "inrf_backward": (S, [POINTER(ModelDesc), c_void_p, c_void_p, c_int64, c_void_p, c_void_p, c_void_p,
                              c_void_p, c_void_p, c_int64, c_void_p]),
        "inrf_adam": (S, [c_void_p, c_void_p, c_void_p, c_void_p, c_int64, POINTER(AdamParams), c_void_p,
                          c_void_p]),
        "inrf_render_nolf": (S, [POINTER(ModelDesc), POINTER(CubesDesc), c_int32, POINTER(CameraDesc), c_void_p,
                                 c_void_p, c_void_p, c_void_p, c_int64, c_void_p]),
        "inrf_shade_nolf": (S, [POINTER(ModelDesc), POINTER(CubesDesc), c_int32, c_void_p, c_void_p, c_void_p,
                                c_int64, c_void_p, c_void_p, c_int64, c_void_p]),
        "inrf_camera_rays": (S, [POINTER(CameraDesc), c_void_p, c_void_p, c_void_p]),
        "inrf_render_static": (S, [POINTER(ModelDesc), c_int32, POINTER(CameraDesc), c_void_p, c_void_p, c_void_p,
                                   c_void_p]),
        "inrf_mlp_encoded": (S, [POINTER(ModelDesc), c_int32, c_void_p, c_void_p, c_int64, c_void_p, c_void_p]),
        "inrf_scene_batch_workspace_size": (c_int64, [c_int32, c_int32, c_int64]),
        "inrf_render_scene_batch": (S, [POINTER(InstanceDesc), c_int32, c_int32, POINTER(CameraDesc), c_int32,
                                        c_void_p, c_void_p, c_void_p, c_void_p, c_void_p, c_int64, c_void_p]),
    }
    for name, (res, args) in sig.items():
        f = getattr(lib, name)
        f.restype = res
        f.argtypes = args


def lib():
    """The loaded library; raises if it has not been built (no fallback)."""
    global _lib
    if _lib is None:
        if not os.path.exists(LIB_PATH):
            raise ImportError(f"{LIB_PATH} is missing: build it with paper_2303_04086_amd.build.build()")
        _lib = ctypes.CDLL(LIB_PATH)
        _declare(_lib)
    return _lib


def check(status: int):
    if status != INRF_OK:
        raise InrfError(status, lib().inrf_last_error().decode())


def ptr(a) -> int:
    """Address of a numpy array or torch tensor (0 for None)."""
    if a is None:
        return 0
    if hasattr(a, "data_ptr"):
        return a.data_ptr()
    return a.ctypes.data
