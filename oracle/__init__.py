"""CPU oracle for the ReFusion per-frame hot path (ctypes over liboracle.so).

TEST INFRASTRUCTURE ONLY: the tests, ``__graft_entry__.smoke()`` and the
benchmark's CPU-baseline leg are the only users.  The GPU product path never
imports this package, and this package never imports the product.

``OracleMap(real_bits=64)`` is the FP64 reference (values in FP64, integer
decisions in FP32); ``real_bits=32`` is the FP32 mirror whose decisions and
values follow the same FP32 operation order as the GPU kernels;
``storage=1`` additionally mirrors FP16 sdf/tau + u8 weight storage.
"""
from __future__ import annotations

import ctypes
import os
import subprocess

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
_LIB_PATH = os.path.join(_HERE, "liboracle.so")
_lib = None

c_void_p, c_int, c_float, c_double, c_int64 = (ctypes.c_void_p, ctypes.c_int, ctypes.c_float,
                                               ctypes.c_double, ctypes.c_int64)


_OMP_PATH = os.path.join(_HERE, "liboracle_omp.so")
_variants = {}


def build(force: bool = True) -> str:
    """Compiles liboracle.so (single thread, what the tests use) and
    liboracle_omp.so (the same source with OpenMP: loops over pixels and
    blocks shared out over threads, sums and insertions kept in the serial
    order, so its results are identical)."""
    src = os.path.join(_HERE, "refusion_oracle.cpp")
    for path, extra in ((_LIB_PATH, []), (_OMP_PATH, ["-fopenmp"])):
        if force or not os.path.exists(path):
            tmp = path + ".tmp%d" % os.getpid()
            subprocess.check_call(["g++", "-O2", "-std=c++17", "-ffp-contract=off", "-fno-fast-math", *extra,
                                   "-shared", "-fPIC", src, "-o", tmp])
            os.replace(tmp, path)
    return _LIB_PATH


class _Frame(ctypes.Structure):
    _fields_ = [("width", ctypes.c_int32), ("height", ctypes.c_int32), ("fx", c_float), ("fy", c_float),
                ("cx", c_float), ("cy", c_float), ("depth", c_void_p), ("depth_u16", ctypes.c_int32),
                ("depth_scale", c_float), ("rgb", c_void_p)]


def _load():
    return load_variant("serial")


def load_variant(kind="serial"):
    """The oracle library: "serial" (liboracle.so) or "omp" (liboracle_omp.so)."""
    global _lib
    if kind in _variants:
        return _variants[kind]
    path = {"serial": _LIB_PATH, "omp": _OMP_PATH}[kind]
    if not os.path.exists(path):
        build(force=False)
    L = ctypes.CDLL(path)
    P = ctypes.POINTER
    sig = {
        "orc_map_new": (c_void_p, [c_int, c_int, c_float, c_float, c_float, c_int, c_int, c_int]),
        "orc_map_num_voxel_blocks": (c_int64, [c_void_p]),
        "orc_export_free": (c_int64, [c_void_p, c_void_p, c_void_p, c_int64]),
        "orc_map_free": (None, [c_void_p]),
        "orc_map_num_blocks": (c_int64, [c_void_p]),
        "orc_allocate": (c_int64, [c_void_p, P(_Frame), c_void_p, c_void_p, c_void_p, c_int64]),
        "orc_integrate": (c_int, [c_void_p, P(_Frame), c_void_p, c_void_p, c_void_p]),
        "orc_normal_equations": (c_int, [c_void_p, P(_Frame), c_void_p, c_void_p, c_int, c_float, c_void_p]),
        "orc_track": (c_int, [c_void_p, P(_Frame), c_void_p, c_void_p, c_int, c_int, c_float, c_int,
                              c_double, c_void_p]),
        "orc_track_lm": (c_int, [c_void_p, P(_Frame), c_void_p, c_void_p, c_int, c_int, c_float, c_int,
                                 c_double, c_void_p, c_void_p]),
        "orc_mask": (c_int, [c_void_p, P(_Frame), c_void_p, c_float, c_float, c_void_p, c_void_p,
                             c_void_p, c_void_p, c_void_p]),
        "orc_export": (c_int64, [c_void_p, c_void_p, c_void_p, c_void_p, c_void_p, c_int64]),
        "orc_import": (c_int, [c_void_p, c_void_p, c_void_p, c_void_p, c_void_p, c_int64]),
        "orc_surface": (c_int64, [c_void_p, c_void_p, c_int64]),
        "orc_mesh": (c_int64, [c_void_p, c_void_p, c_int64]),
        "orc_raycast": (c_int, [c_void_p, P(_Frame), c_void_p, c_double, c_double, c_double, c_int, c_void_p]),
        "orc_se3_exp": (None, [c_void_p, c_void_p]),
        "orc_pose_left_update": (None, [c_void_p, c_void_p]),
        "orc_solve6": (c_int, [c_void_p, c_double, c_void_p]),
        "orc_round_to_half": (c_float, [c_float]),
        "orc_sample": (c_int, [c_void_p, c_void_p, c_void_p]),
        "orc_pixel_terms": (c_int, [c_void_p, c_void_p, c_void_p, c_double, c_void_p]),
        "orc_dda": (c_int64, [c_void_p, c_void_p, c_void_p, c_int64]),
        "orc_floodfill": (None, [c_void_p, c_void_p, c_int, c_int, c_float, c_void_p]),
        "orc_morph3x3": (None, [c_void_p, c_int, c_int, c_int, c_void_p]),
        "orc_set_threads": (None, [c_int]),
        "orc_get_threads": (c_int, []),
    }
    for name, (res, args) in sig.items():
        fn = getattr(L, name)
        fn.restype = res
        fn.argtypes = args
    _variants[kind] = L
    if kind == "serial":
        _lib = L
    return L


def _ptr(a):
    return None if a is None else a.ctypes.data


class Frame:
    """Host-side RGB-D frame: depth (H,W) float32 metres or uint16 + scale;
    rgb (H,W,3) uint8; pinhole fx, fy, cx, cy."""

    def __init__(self, depth, rgb, fx, fy, cx, cy, depth_scale=1.0):
        self.depth = np.ascontiguousarray(depth)
        assert self.depth.dtype in (np.float32, np.uint16)
        self.rgb = np.ascontiguousarray(rgb, dtype=np.uint8)
        self.H, self.W = self.depth.shape
        assert self.rgb.shape == (self.H, self.W, 3)
        self.s = _Frame(self.W, self.H, fx, fy, cx, cy, self.depth.ctypes.data,
                        1 if self.depth.dtype == np.uint16 else 0, depth_scale, self.rgb.ctypes.data)

    def metres(self):
        if self.depth.dtype == np.float32:
            return self.depth
        return self.depth.astype(np.float32) * np.float32(self.s.depth_scale)


def _mask_arg(mask, fr):
    if mask is None:
        return None
    m = np.ascontiguousarray(mask, dtype=np.uint8)
    assert m.shape == (fr.H, fr.W)
    return m


class OracleMap:
    def __init__(self, voxel_size, truncation, depth_max=5.0, max_weight=255, carve_stride=4,
                 real_bits=64, storage=0, lib=None, free_blocks=0):
        self.L = _load() if lib is None else lib
        self.real_bits = real_bits
        self.h = self.L.orc_map_new(real_bits, storage, voxel_size, truncation, depth_max, max_weight,
                                    carve_stride, free_blocks)

    def __del__(self):
        if getattr(self, "h", None):
            self.L.orc_map_free(self.h)
            self.h = None

    @property
    def num_blocks(self):
        return self.L.orc_map_num_blocks(self.h)

    @property
    def num_voxel_blocks(self):
        """Blocks holding voxels (with compact free space: not the free blocks)."""
        return self.L.orc_map_num_voxel_blocks(self.h)

    def export_free(self):
        """Compact free space: (sorted (n,3) int32 keys, (n,) weights) of the free blocks."""
        n = self.L.orc_export_free(self.h, None, None, 0)
        keys = np.zeros((n, 3), np.int32)
        w = np.zeros(n, np.float64)
        self.L.orc_export_free(self.h, keys.ctypes.data, w.ctypes.data, n)
        return keys, w

    def allocate(self, fr: Frame, pose, mask=None):
        """Returns the sorted (n,3) int32 keys of the blocks visited this frame."""
        T = np.ascontiguousarray(pose, np.float64)
        m = _mask_arg(mask, fr)
        n = self.L.orc_allocate(self.h, ctypes.byref(fr.s), T.ctypes.data, _ptr(m), None, 0)
        keys = np.zeros((max(n, 1), 3), np.int32)
        self.L.orc_allocate(self.h, ctypes.byref(fr.s), T.ctypes.data, _ptr(m), keys.ctypes.data, n)
        return keys[:n]

    def integrate(self, fr: Frame, pose, mask=None):
        T = np.ascontiguousarray(pose, np.float64)
        m = _mask_arg(mask, fr)
        counts = np.zeros(3, np.int64)
        self.L.orc_integrate(self.h, ctypes.byref(fr.s), T.ctypes.data, _ptr(m), counts.ctypes.data)
        return counts  # band updates, free-space updates, blocks carved whole (compact free space)

    def normal_equations(self, fr: Frame, pose, level=0, w_c=0.025, mask=None):
        T = np.ascontiguousarray(pose, np.float64)
        m = _mask_arg(mask, fr)
        out = np.zeros(29, np.float64)
        self.L.orc_normal_equations(self.h, ctypes.byref(fr.s), T.ctypes.data, _ptr(m), level, w_c,
                                    out.ctypes.data)
        return out

    def track(self, fr: Frame, pose, levels=3, iters=10, w_c=0.025, min_valid=64, lm_lambda=0.0,
              mask=None):
        T = np.array(pose, np.float64, order="C")
        m = _mask_arg(mask, fr)
        stats = np.zeros(4 + levels, np.float64)
        flags = self.L.orc_track(self.h, ctypes.byref(fr.s), T.ctypes.data, _ptr(m), levels, iters, w_c,
                                 min_valid, lm_lambda, stats.ctypes.data)
        return T, int(flags), stats

    def track_lm(self, fr: Frame, pose, levels=3, iters=10, w_c=0.025, min_valid=64, lambda0=1e-4,
                 mask=None):
        """Levenberg-Marquardt registration (Section III-B's solver; accept /
        reject on the mean cost, lambda /10 and x10).  Returns (pose, flags,
        stats, trace) with trace rows (level, mean cost, count, accepted,
        lambda after the decision), one per evaluation."""
        T = np.array(pose, np.float64, order="C")
        m = _mask_arg(mask, fr)
        stats = np.zeros(4 + levels, np.float64)
        trace = np.zeros((levels * iters, 5), np.float64)
        flags = self.L.orc_track_lm(self.h, ctypes.byref(fr.s), T.ctypes.data, _ptr(m), levels, iters, w_c,
                                    min_valid, lambda0, stats.ctypes.data, trace.ctypes.data)
        return T, int(flags), stats, trace

    def mask(self, fr: Frame, pose, gamma=0.5, theta=0.007):
        """Returns dict(raw, eroded, filled, final, residual) (FP32 mirror only)."""
        assert self.real_bits == 32, "the dynamic mask is an FP32 decision"
        T = np.ascontiguousarray(pose, np.float64)
        out = {k: np.zeros((fr.H, fr.W), np.uint8) for k in ("raw", "eroded", "filled", "final")}
        out["residual"] = np.zeros((fr.H, fr.W), np.float32)
        self.L.orc_mask(self.h, ctypes.byref(fr.s), T.ctypes.data, gamma, theta, out["raw"].ctypes.data,
                        out["eroded"].ctypes.data, out["filled"].ctypes.data, out["final"].ctypes.data,
                        out["residual"].ctypes.data)
        return out

    def export(self):
        """Sorted map: keys (n,3) int32, sdf (n,512) f64, weight (n,512) f64, rgb (n,512,3) u8."""
        n = self.L.orc_export(self.h, None, None, None, None, 0)
        keys = np.zeros((n, 3), np.int32)
        sdf = np.zeros((n, 512), np.float64)
        w = np.zeros((n, 512), np.float64)
        rgb = np.zeros((n, 512, 3), np.uint8)
        if n:
            self.L.orc_export(self.h, keys.ctypes.data, sdf.ctypes.data, w.ctypes.data, rgb.ctypes.data, n)
        return keys, sdf, w, rgb

    def import_(self, keys, sdf, w, rgb):
        keys = np.ascontiguousarray(keys, np.int32)
        sdf = np.ascontiguousarray(sdf, np.float64)
        w = np.ascontiguousarray(w, np.float64)
        rgb = np.ascontiguousarray(rgb, np.uint8)
        n = keys.shape[0]
        assert sdf.shape == (n, 512) and w.shape == (n, 512) and rgb.shape == (n, 512, 3)
        self.L.orc_import(self.h, keys.ctypes.data, sdf.ctypes.data, w.ctypes.data, rgb.ctypes.data, n)

    def surface(self):
        """Zero-crossing points (n,7): x, y, z, r, g, b, edge axis."""
        n = self.L.orc_surface(self.h, None, 0)
        out = np.zeros((max(n, 1), 7), np.float64)
        if n:
            self.L.orc_surface(self.h, out.ctypes.data, n)
        return out[:n]

    def raycast(self, fr: Frame, pose, z_near=0.3, z_far=5.0, far_value=5.0, only_invalid=True):
        """Virtual depth (only_invalid=False) or the frame's depth with its
        zeros filled (only_invalid=True): (H, W) float32 metres."""
        T = np.ascontiguousarray(pose, np.float64)
        out = np.zeros((fr.H, fr.W), np.float32)
        self.L.orc_raycast(self.h, ctypes.byref(fr.s), T.ctypes.data, z_near, z_far, far_value,
                           1 if only_invalid else 0, out.ctypes.data)
        return out

    def mesh(self):
        """Marching-tetrahedra triangles (n,3,3): three vertices x, y, z each."""
        n = self.L.orc_mesh(self.h, None, 0)
        out = np.zeros((max(n, 1), 3, 3), np.float64)
        if n:
            self.L.orc_mesh(self.h, out.ctypes.data, n)
        return out[:n]

    def sample(self, y):
        y = np.ascontiguousarray(y, np.float64)
        out = np.zeros(8, np.float64)
        ok = self.L.orc_sample(self.h, y.ctypes.data, out.ctypes.data)
        return bool(ok), out

    def pixel_terms(self, x_cam, pose, I_pix):
        x = np.ascontiguousarray(x_cam, np.float64)
        T = np.ascontiguousarray(pose, np.float64)
        out = np.zeros(14, np.float64)
        ok = self.L.orc_pixel_terms(self.h, x.ctypes.data, T.ctypes.data, float(I_pix), out.ctypes.data)
        return bool(ok), out


def se3_exp(xi):
    L = _load()
    xi = np.ascontiguousarray(xi, np.float64)
    T = np.zeros(16, np.float64)
    L.orc_se3_exp(xi.ctypes.data, T.ctypes.data)
    return T.reshape(4, 4)


def pose_left_update(xi, pose):
    L = _load()
    xi = np.ascontiguousarray(xi, np.float64)
    T = np.array(pose, np.float64, order="C")
    L.orc_pose_left_update(xi.ctypes.data, T.ctypes.data)
    return T


def solve6(ne, lam=0.0):
    L = _load()
    ne = np.ascontiguousarray(ne, np.float64)
    d = np.zeros(6, np.float64)
    rc = L.orc_solve6(ne.ctypes.data, lam, d.ctypes.data)
    return (d if rc == 0 else None)


def round_to_half(x):
    L = _load()
    return np.float32(L.orc_round_to_half(float(x)))


def dda(q0, q1):
    L = _load()
    q0 = np.ascontiguousarray(q0, np.float32)
    q1 = np.ascontiguousarray(q1, np.float32)
    n = L.orc_dda(q0.ctypes.data, q1.ctypes.data, None, 0)
    out = np.zeros((max(n, 1), 3), np.int32)
    L.orc_dda(q0.ctypes.data, q1.ctypes.data, out.ctypes.data, n)
    return out[:n]


def floodfill(seeds, depth, theta):
    L = _load()
    s = np.ascontiguousarray(seeds, np.uint8)
    D = np.ascontiguousarray(depth, np.float32)
    H, W = s.shape
    out = np.zeros_like(s)
    L.orc_floodfill(s.ctypes.data, D.ctypes.data, W, H, theta, out.ctypes.data)
    return out


def morph3x3(mask, erode):
    L = _load()
    m = np.ascontiguousarray(mask, np.uint8)
    H, W = m.shape
    out = np.zeros_like(m)
    L.orc_morph3x3(m.ctypes.data, W, H, 1 if erode else 0, out.ctypes.data)
    return out


def process_frame(omap: OracleMap, fr: Frame, pose_prev, k, levels, iters, w_c=0.025, gamma=0.5,
                  theta=0.007, min_valid=64, dynamic=True, mask_map: OracleMap | None = None,
                  times: dict | None = None):
    """One frame of the method (Fig. 2 order): initial registration, residual
    mask, registration without masked pixels, allocation, integration.  Frame 0
    only allocates and integrates at ``pose_prev``.  ``mask_map`` (FP32 mirror
    holding the same map) supplies the FP32 mask decision when omap is FP64.
    ``times`` (optional) accumulates the seconds of each stage (track1, mask,
    track2, allocate, integrate, and mirror: the FP32 mirror's fusion)."""
    import time
    clock = [time.perf_counter()]

    def lap(stage):
        if times is not None:
            t = time.perf_counter()
            times[stage] = times.get(stage, 0.0) + t - clock[0]
            clock[0] = t
    if k == 0:
        omap.allocate(fr, pose_prev)
        omap.integrate(fr, pose_prev)
        if mask_map is not None and mask_map is not omap:
            mask_map.allocate(fr, pose_prev)
            mask_map.integrate(fr, pose_prev)
        return np.array(pose_prev), None
    T1, _, _ = omap.track(fr, pose_prev, levels, iters, w_c, min_valid)
    lap("track1")
    mask = None
    T = T1
    if dynamic:
        mm = mask_map if mask_map is not None else omap
        mask = mm.mask(fr, T1, gamma, theta)["final"]
        lap("mask")
        T, _, _ = omap.track(fr, T1, levels, iters, w_c, min_valid, mask=mask)
        lap("track2")
    omap.allocate(fr, T, mask)
    lap("allocate")
    omap.integrate(fr, T, mask)
    lap("integrate")
    if mask_map is not None and mask_map is not omap:
        mask_map.allocate(fr, T, mask)
        mask_map.integrate(fr, T, mask)
        lap("mirror")
    return T, mask
