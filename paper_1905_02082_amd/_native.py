"""ctypes declarations of the C ABI in include/refusion.h.

This module only loads librefusion_hip.so and declares argument types; it
raises if the library is missing (there is no fallback path)."""
from __future__ import annotations

import ctypes
import os

HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(HERE, "librefusion_hip.so")

RF_OK = 0
RF_EINVAL, RF_ENOMEM, RF_EDEVICE, RF_EUNSUPPORTED = -1, -2, -3, -4
RF_FLAG_POOL_FULL = 0x1
RF_FLAG_HASH_FULL = 0x2
RF_FLAG_TRACK_FEW_PIXELS = 0x4
RF_FLAG_TRACK_SINGULAR = 0x8
RF_FLAG_MASK_LIMIT = 0x10
RF_FLAG_TRACK_RANGE = 0x20
RF_DEPTH_U16, RF_DEPTH_F32 = 0, 1
RF_STORAGE_FP32, RF_STORAGE_FP16_U8 = 0, 1

c_void_p, c_int32, c_uint32, c_float, c_double, c_size_t = (
    ctypes.c_void_p, ctypes.c_int32, ctypes.c_uint32, ctypes.c_float, ctypes.c_double, ctypes.c_size_t)


class RfFrame(ctypes.Structure):
    _fields_ = [("fx", c_float), ("fy", c_float), ("cx", c_float), ("cy", c_float),
                ("width", c_int32), ("height", c_int32), ("depth", c_void_p), ("depth_format", c_int32),
                ("depth_scale", c_float), ("rgb", c_void_p)]


class RfMapParams(ctypes.Structure):
    _fields_ = [("voxel_size", c_float), ("truncation", c_float), ("depth_max", c_float),
                ("num_buckets", c_uint32), ("max_blocks", c_uint32), ("max_weight", c_uint32),
                ("carve_stride", c_uint32), ("storage", c_int32), ("max_pixels", c_uint32),
                ("free_blocks", c_int32)]


class RfTrackParams(ctypes.Structure):
    _fields_ = [("levels", c_int32), ("iters_per_level", c_int32), ("w_c", c_float), ("min_valid", c_int32),
                ("lm_lambda", c_double), ("adaptive", c_int32)]


class RfMaskParams(ctypes.Structure):
    _fields_ = [("gamma", c_float), ("theta", c_float)]


class RfTrackStats(ctypes.Structure):
    _fields_ = [("cost", c_double), ("count", c_double), ("iters", c_int32), ("flags", c_uint32),
                ("level_count", c_double * 8)]


class RfJob(ctypes.Structure):
    _fields_ = [("map", c_void_p), ("frame", RfFrame), ("d_pose", c_void_p), ("d_mask", c_void_p),
                ("d_mask_out", c_void_p), ("d_stats", c_void_p)]


EXPORTS = {
    "hashmap_bytes": (c_int32, [ctypes.POINTER(RfMapParams), ctypes.POINTER(c_size_t)]),
    "hashmap_create": (c_int32, [ctypes.POINTER(RfMapParams), c_void_p, c_size_t, c_void_p,
                                 ctypes.POINTER(c_void_p)]),
    "hashmap_destroy": (c_int32, [c_void_p]),
    "hashmap_reset": (c_int32, [c_void_p, c_void_p]),
    "hashmap_allocate": (c_int32, [c_void_p, ctypes.POINTER(RfFrame), c_void_p, c_void_p, c_void_p]),
    "integrate_frame": (c_int32, [c_void_p, ctypes.POINTER(RfFrame), c_void_p, c_void_p, c_void_p]),
    "track_frame": (c_int32, [c_void_p, ctypes.POINTER(RfFrame), ctypes.POINTER(RfTrackParams), c_void_p,
                              c_void_p, c_void_p, c_void_p]),
    "track_normal_equations": (c_int32, [c_void_p, ctypes.POINTER(RfFrame), c_void_p, c_void_p, c_int32,
                                         c_float, c_void_p, c_void_p]),
    "compute_dynamic_mask": (c_int32, [c_void_p, ctypes.POINTER(RfFrame), c_void_p,
                                       ctypes.POINTER(RfMaskParams), c_void_p, c_void_p, c_void_p]),
    "compute_dynamic_mask_static": (c_int32, [c_void_p, ctypes.POINTER(RfFrame), c_void_p,
                                              ctypes.POINTER(RfMaskParams), c_void_p, c_void_p, c_void_p]),
    "compute_dynamic_mask_stages": (c_int32, [c_void_p, ctypes.POINTER(RfFrame), c_void_p,
                                              ctypes.POINTER(RfMaskParams), c_void_p, c_void_p, c_void_p,
                                              c_void_p, c_void_p, c_void_p]),
    "extract_surface": (c_int32, [c_void_p, c_void_p, c_uint32, c_void_p, c_void_p]),
    "extract_mesh": (c_int32, [c_void_p, c_void_p, c_uint32, c_void_p, c_void_p]),
    "raycast_depth": (c_int32, [c_void_p, c_void_p, c_void_p, c_float, c_float, c_float, c_int32, c_void_p,
                                c_void_p]),
    "hashmap_export_free": (c_int32, [c_void_p, c_void_p, c_void_p, c_uint32, c_void_p, c_void_p]),
    "map_status": (c_int32, [c_void_p, c_void_p, ctypes.POINTER(c_uint32), ctypes.POINTER(c_uint32)]),
    "hashmap_frame_blocks": (c_int32, [c_void_p, c_void_p, c_uint32, c_void_p, c_void_p]),
    "hashmap_export": (c_int32, [c_void_p, c_void_p, c_void_p, c_void_p, c_void_p, c_uint32, c_void_p,
                                 c_void_p]),
    "hashmap_import": (c_int32, [c_void_p, c_void_p, c_void_p, c_void_p, c_void_p, c_uint32, c_void_p]),
    "track_frame_batch": (c_int32, [ctypes.POINTER(RfJob), c_int32, ctypes.POINTER(RfTrackParams), c_void_p]),
    "compute_dynamic_mask_batch": (c_int32, [ctypes.POINTER(RfJob), c_int32, ctypes.POINTER(RfMaskParams),
                                             c_void_p]),
    "hashmap_allocate_batch": (c_int32, [ctypes.POINTER(RfJob), c_int32, c_void_p]),
    "integrate_frame_batch": (c_int32, [ctypes.POINTER(RfJob), c_int32, c_void_p]),
    "rf_last_error": (ctypes.c_char_p, []),
    "rf_version": (ctypes.c_char_p, []),
}

_lib = None


def load():
    """Loads the built library (raises if it has not been built)."""
    global _lib
    if _lib is not None:
        return _lib
    if not os.path.exists(LIB_PATH):
        raise RuntimeError("librefusion_hip.so is not built (%s); run __graft_entry__.build() or "
                           "python paper_1905_02082_amd/build.py" % LIB_PATH)
    lib = ctypes.CDLL(LIB_PATH)
    for name, (res, args) in EXPORTS.items():
        fn = getattr(lib, name)
        fn.restype = res
        fn.argtypes = args
    _lib = lib
    return lib
