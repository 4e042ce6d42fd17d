"""ReFusion per-frame hot path on MI355X (gfx950): Python binding.

Every step runs in the HIP kernels of librefusion_hip.so through the C ABI of
include/refusion.h; this module marshals arguments and owns device buffers
through torch tensors (device memory and streams only).  There is no CPU
fallback: on a machine without the built library or a GPU the calls raise.

Per frame (the order of the paper's Fig. 2, Sec. III):
    track (no mask) -> dynamic mask -> track (masked) -> allocate -> integrate
"""
from __future__ import annotations

import ctypes
import dataclasses

import torch

from . import _native as N
from ._native import (RF_DEPTH_F32, RF_DEPTH_U16, RF_FLAG_HASH_FULL, RF_FLAG_MASK_LIMIT,  # noqa: F401
                      RF_FLAG_POOL_FULL, RF_FLAG_TRACK_FEW_PIXELS, RF_FLAG_TRACK_RANGE, RF_FLAG_TRACK_SINGULAR,
                      RF_STORAGE_FP16_U8, RF_STORAGE_FP32)

__all__ = ["MapParams", "TrackParams", "MaskParams", "Frame", "Map", "Session", "Pipeline", "process_batch",
           "GraphStep", "VirtualDepth", "RefusionError", "hashmap_bytes", "lib"]


class RefusionError(RuntimeError):
    pass


def lib():
    return N.load()


def _check(rc, what):
    if rc != N.RF_OK:
        msg = N.load().rf_last_error().decode(errors="replace")
        raise RefusionError("%s failed (status %d): %s" % (what, rc, msg))


def _ptr(t):
    return None if t is None else ctypes.c_void_p(t.data_ptr())


def _stream(stream=None):
    s = torch.cuda.current_stream() if stream is None else stream
    return ctypes.c_void_p(s.cuda_stream)


def _dev(t, name, dtype=None, shape=None):
    if not isinstance(t, torch.Tensor) or not t.is_cuda:
        raise RefusionError("%s must be a CUDA (HIP) tensor" % name)
    if not t.is_contiguous():
        raise RefusionError("%s must be contiguous" % name)
    if dtype is not None and t.dtype != dtype:
        raise RefusionError("%s must be %s, got %s" % (name, dtype, t.dtype))
    if shape is not None and tuple(t.shape) != tuple(shape):
        raise RefusionError("%s must have shape %s, got %s" % (name, tuple(shape), tuple(t.shape)))
    return t


@dataclasses.dataclass
class MapParams:
    voxel_size: float
    truncation: float
    depth_max: float = 5.0
    num_buckets: int = 1 << 20
    max_blocks: int = 1 << 18
    max_weight: int = 255
    carve_stride: int = 4
    storage: str = "fp32"            # "fp32" | "fp16"
    max_pixels: int = 640 * 480
    free_blocks: bool = False        # compact free space (blocks carved whole, free blocks without voxels)

    def c(self):
        st = {"fp32": N.RF_STORAGE_FP32, "fp16": N.RF_STORAGE_FP16_U8}[self.storage]
        return N.RfMapParams(self.voxel_size, self.truncation, self.depth_max, self.num_buckets, self.max_blocks,
                             self.max_weight, self.carve_stride, st, self.max_pixels, 1 if self.free_blocks else 0)


@dataclasses.dataclass
class TrackParams:
    levels: int = 3
    iters_per_level: int = 10
    w_c: float = 0.025          # photometric weight (Table I)
    min_valid: int = 64
    lm_lambda: float = 0.0      # 0: Gauss-Newton; with adaptive, the starting lambda
    adaptive: bool = False      # Levenberg-Marquardt accept / reject with adaptive lambda

    def c(self):
        return N.RfTrackParams(self.levels, self.iters_per_level, self.w_c, self.min_valid, self.lm_lambda,
                               1 if self.adaptive else 0)


@dataclasses.dataclass
class MaskParams:
    gamma: float = 0.5          # residual threshold weight (Table I)
    theta: float = 0.007        # flood-fill threshold (Table I)

    def c(self):
        return N.RfMaskParams(self.gamma, self.theta)


def hashmap_bytes(params: MapParams) -> int:
    n = ctypes.c_size_t(0)
    p = params.c()
    _check(N.load().hashmap_bytes(ctypes.byref(p), ctypes.byref(n)), "hashmap_bytes")
    return int(n.value)


class Frame:
    """An RGB-D frame in device memory: depth (H,W) uint16 (x depth_scale m)
    or float32 (m); rgb (H,W,3) uint8."""

    def __init__(self, depth: torch.Tensor, rgb: torch.Tensor, fx, fy, cx, cy, depth_scale=0.001):
        _dev(depth, "depth")
        if depth.dtype == torch.uint16 if hasattr(torch, "uint16") else False:
            fmt = N.RF_DEPTH_U16
        elif depth.dtype == torch.int16:
            fmt = N.RF_DEPTH_U16   # raw 16-bit words reinterpreted as unsigned by the kernels
        elif depth.dtype == torch.float32:
            fmt = N.RF_DEPTH_F32
        else:
            raise RefusionError("depth must be uint16/int16 (millimetre words) or float32 metres")
        if depth.dim() != 2:
            raise RefusionError("depth must be (H, W)")
        H, W = depth.shape
        _dev(rgb, "rgb", torch.uint8, (H, W, 3))
        self.depth, self.rgb = depth, rgb
        self.fx, self.fy, self.cx, self.cy, self.depth_scale = fx, fy, cx, cy, depth_scale
        self.W, self.H = int(W), int(H)
        self.s = N.RfFrame(fx, fy, cx, cy, self.W, self.H, depth.data_ptr(), fmt,
                           depth_scale if fmt == N.RF_DEPTH_U16 else 1.0, rgb.data_ptr())

    @staticmethod
    def from_numpy(depth, rgb, fx, fy, cx, cy, depth_scale=0.001, device="cuda"):
        import numpy as np
        if depth.dtype == np.uint16:
            d = torch.from_numpy(np.ascontiguousarray(depth).view(np.int16)).to(device)
        else:
            d = torch.from_numpy(np.ascontiguousarray(depth, np.float32)).to(device)
        c = torch.from_numpy(np.ascontiguousarray(rgb, np.uint8)).to(device)
        return Frame(d, c, fx, fy, cx, cy, depth_scale)


class Map:
    """A voxel-block TSDF in a device arena owned by this object."""

    def __init__(self, params: MapParams, device="cuda", stream=None):
        self.params = params
        self.L = N.load()
        nbytes = hashmap_bytes(params)
        self.arena = torch.empty(nbytes + 256, dtype=torch.uint8, device=device)
        base = self.arena.data_ptr()
        off = (-base) % 256
        self._arena_ptr = ctypes.c_void_p(base + off)
        self.arena_bytes = nbytes
        self.c_params = params.c()
        h = ctypes.c_void_p(0)
        _check(self.L.hashmap_create(ctypes.byref(self.c_params), self._arena_ptr, nbytes, _stream(stream),
                                     ctypes.byref(h)), "hashmap_create")
        self.h = h
        self.device = self.arena.device

    def __del__(self):
        h = getattr(self, "h", None)
        if h is not None and h.value:
            self.L.hashmap_destroy(h)
            self.h = None

    # ---- per-frame steps
    def allocate(self, frame: Frame, pose: torch.Tensor, mask=None, stream=None):
        _dev(pose, "pose", torch.float64, (4, 4))
        if mask is not None:
            _dev(mask, "mask", torch.uint8, (frame.H, frame.W))
        _check(self.L.hashmap_allocate(self.h, ctypes.byref(frame.s), _ptr(pose), _ptr(mask), _stream(stream)),
               "hashmap_allocate")

    def integrate(self, frame: Frame, pose: torch.Tensor, mask=None, stream=None):
        _dev(pose, "pose", torch.float64, (4, 4))
        if mask is not None:
            _dev(mask, "mask", torch.uint8, (frame.H, frame.W))
        _check(self.L.integrate_frame(self.h, ctypes.byref(frame.s), _ptr(pose), _ptr(mask), _stream(stream)),
               "integrate_frame")

    def track(self, frame: Frame, pose: torch.Tensor, tp: TrackParams, mask=None, stats=None, stream=None):
        """Registers the frame; pose (device float64 4x4) is updated in place.
        stats: optional device tensor of >= 11 float64 (rf_track_stats)."""
        _dev(pose, "pose", torch.float64, (4, 4))
        if mask is not None:
            _dev(mask, "mask", torch.uint8, (frame.H, frame.W))
        if stats is not None:
            _dev(stats, "stats")
            if stats.numel() * stats.element_size() < ctypes.sizeof(N.RfTrackStats):
                raise RefusionError("stats buffer too small")
        c = tp.c()
        _check(self.L.track_frame(self.h, ctypes.byref(frame.s), ctypes.byref(c), _ptr(mask), _ptr(pose),
                                  _ptr(stats), _stream(stream)), "track_frame")

    def normal_equations(self, frame: Frame, pose: torch.Tensor, level=0, w_c=0.025, mask=None, stream=None):
        _dev(pose, "pose", torch.float64, (4, 4))
        out = torch.empty(29, dtype=torch.float64, device=self.device)
        if mask is not None:
            _dev(mask, "mask", torch.uint8, (frame.H, frame.W))
        _check(self.L.track_normal_equations(self.h, ctypes.byref(frame.s), _ptr(mask), _ptr(pose), level, w_c,
                                             _ptr(out), _stream(stream)), "track_normal_equations")
        return out

    def dynamic_mask(self, frame: Frame, pose: torch.Tensor, mp: MaskParams, out=None, residual=None,
                     stages=False, stream=None):
        _dev(pose, "pose", torch.float64, (4, 4))
        shape = (frame.H, frame.W)
        if out is None:
            out = torch.empty(shape, dtype=torch.uint8, device=self.device)
        _dev(out, "out", torch.uint8, shape)
        if residual is not None:
            _dev(residual, "residual", torch.float32, shape)
        c = mp.c()
        if not stages:
            _check(self.L.compute_dynamic_mask(self.h, ctypes.byref(frame.s), _ptr(pose), ctypes.byref(c),
                                               _ptr(out), _ptr(residual), _stream(stream)), "compute_dynamic_mask")
            return out
        raw = torch.empty(shape, dtype=torch.uint8, device=self.device)
        ero = torch.empty_like(raw)
        fil = torch.empty_like(raw)
        _check(self.L.compute_dynamic_mask_stages(self.h, ctypes.byref(frame.s), _ptr(pose), ctypes.byref(c),
                                                  _ptr(raw), _ptr(ero), _ptr(fil), _ptr(out), _ptr(residual),
                                                  _stream(stream)), "compute_dynamic_mask_stages")
        return {"raw": raw, "eroded": ero, "filled": fil, "final": out}

    # ---- inspection
    def status(self, stream=None):
        f, n = ctypes.c_uint32(0), ctypes.c_uint32(0)
        _check(self.L.map_status(self.h, _stream(stream), ctypes.byref(f), ctypes.byref(n)), "map_status")
        return int(f.value), int(n.value)

    def frame_blocks(self, stream=None):
        cap = self.params.num_buckets
        keys = torch.empty((cap, 3), dtype=torch.int32, device=self.device)
        cnt = torch.zeros(1, dtype=torch.int32, device=self.device)
        _check(self.L.hashmap_frame_blocks(self.h, _ptr(keys), cap, _ptr(cnt), _stream(stream)),
               "hashmap_frame_blocks")
        n = int(cnt.item())
        return keys[:n]

    def export(self, stream=None):
        """All blocks: keys (n,3) int32, sdf (n,512) f32, weight (n,512) f32,
        rgb (n,512,3) u8 (device tensors, pool order)."""
        _, n = self.status(stream)
        keys = torch.empty((max(n, 1), 3), dtype=torch.int32, device=self.device)
        sdf = torch.empty((max(n, 1), 512), dtype=torch.float32, device=self.device)
        w = torch.empty_like(sdf)
        rgb = torch.empty((max(n, 1), 512, 3), dtype=torch.uint8, device=self.device)
        cnt = torch.zeros(1, dtype=torch.int32, device=self.device)
        _check(self.L.hashmap_export(self.h, _ptr(keys), _ptr(sdf), _ptr(w), _ptr(rgb), n, _ptr(cnt),
                                     _stream(stream)), "hashmap_export")
        return keys[:n], sdf[:n], w[:n], rgb[:n]

    def import_(self, keys, sdf, weight, rgb, stream=None):
        n = int(keys.shape[0])
        _dev(keys, "keys", torch.int32, (n, 3))
        _dev(sdf, "sdf", torch.float32, (n, 512))
        _dev(weight, "weight", torch.float32, (n, 512))
        _dev(rgb, "rgb", torch.uint8, (n, 512, 3))
        _check(self.L.hashmap_import(self.h, _ptr(keys), _ptr(sdf), _ptr(weight), _ptr(rgb), n, _stream(stream)),
               "hashmap_import")

    def surface(self, cap=None, stream=None):
        """Zero-crossing points (n,7) float32: x, y, z, r, g, b, axis."""
        if cap is None:
            _, nb = self.status(stream)
            cap = max(1024, nb * 512 * 3 // 4)
        pts = torch.empty((cap, 7), dtype=torch.float32, device=self.device)
        cnt = torch.zeros(1, dtype=torch.int32, device=self.device)
        _check(self.L.extract_surface(self.h, _ptr(pts), cap, _ptr(cnt), _stream(stream)), "extract_surface")
        n = int(cnt.item())
        if n > cap:
            return self.surface(cap=n, stream=stream)
        return pts[:n]

    def raycast(self, frame: Frame, pose: torch.Tensor, z_near=0.3, z_far=None, far_value=None, only_invalid=True,
                out=None, stream=None):
        """Virtual depth of the model seen from pose (float64 4x4 device):
        (H, W) float32 metres.  only_invalid: the frame's depth with its zeros
        replaced by the virtual depth (far_value where no surface is met)."""
        _dev(pose, "pose", torch.float64, (4, 4))
        z_far = self.params.depth_max if z_far is None else z_far
        far_value = self.params.depth_max if far_value is None else far_value
        if out is None:
            out = torch.empty((frame.H, frame.W), dtype=torch.float32, device=self.device)
        _dev(out, "out", torch.float32, (frame.H, frame.W))
        _check(self.L.raycast_depth(self.h, ctypes.byref(frame.s), _ptr(pose), z_near, z_far, far_value,
                                    1 if only_invalid else 0, _ptr(out), _stream(stream)), "raycast_depth")
        return out

    def mesh(self, cap=None, stream=None):
        """Marching-tetrahedra triangle mesh of the zero level set: (n, 3, 3)
        float32 device tensor (three vertices x, y, z per triangle, facing the
        positive side).  cap: triangle capacity of the first attempt."""
        if cap is None:
            _, nb = self.status(stream)
            cap = max(1024, nb * 256)
        tris = torch.empty((cap, 3, 3), dtype=torch.float32, device=self.device)
        cnt = torch.zeros(1, dtype=torch.int32, device=self.device)
        _check(self.L.extract_mesh(self.h, _ptr(tris), cap, _ptr(cnt), _stream(stream)), "extract_mesh")
        n = int(cnt.item())
        if n > cap:
            return self.mesh(cap=n, stream=stream)
        return tris[:n]

    def export_free(self, stream=None):
        """Compact free space: (keys (n,3) int32, weights (n,) float32) of the
        free blocks, on the device, in no particular order."""
        cnt = torch.zeros(1, dtype=torch.int32, device=self.device)
        _check(self.L.hashmap_export_free(self.h, None, None, 0, _ptr(cnt), _stream(stream)), "hashmap_export_free")
        n = int(cnt.item())
        keys = torch.empty((max(n, 1), 3), dtype=torch.int32, device=self.device)
        w = torch.empty(max(n, 1), dtype=torch.float32, device=self.device)
        _check(self.L.hashmap_export_free(self.h, _ptr(keys), _ptr(w), n, _ptr(cnt), _stream(stream)),
               "hashmap_export_free")
        return keys[:n], w[:n]

    def _state_words(self):
        off = (-self.arena.data_ptr()) % 256
        return self.arena[off:off + 88].clone().cpu().view(torch.int64)

    def stats_counts(self):
        """(band, free) voxel updates of the last integration (device state)."""
        v = self._state_words()
        return int(v[4].item()), int(v[5].item())

    def cumulative_counts(self):
        """Since creation: (band updates, free-space updates, listed blocks
        integrated, integrations, listed blocks carved whole)."""
        v = self._state_words()
        return tuple(int(v[i].item()) for i in range(6, 11))

    def num_keys(self):
        """Blocks in the hash table (with compact free space: free blocks too)."""
        v = self._state_words()
        return int(v[3].item()) >> 32


class Session:
    """One reconstruction session: a map plus its device-resident pose, mask
    and tracking statistics.  Frames advance through process_batch."""

    def __init__(self, params: MapParams, initial_pose, device="cuda"):
        self.map = Map(params, device)
        self.pose = torch.as_tensor(initial_pose, dtype=torch.float64).to(device).contiguous()
        self.mask = None
        self.stats = torch.zeros(16, dtype=torch.float64, device=device)
        self.k = 0

    def _mask_for(self, frame):
        if self.mask is None or tuple(self.mask.shape) != (frame.H, frame.W):
            self.mask = torch.empty((frame.H, frame.W), dtype=torch.uint8, device=self.pose.device)
        return self.mask


def _jobs(sessions, frames, mask=False, mask_out=False, stats=False):
    arr = (N.RfJob * len(sessions))()
    for i, (s, f) in enumerate(zip(sessions, frames)):
        j = arr[i]
        j.map = s.map.h
        j.frame = f.s
        j.d_pose = s.pose.data_ptr()
        j.d_mask = s.mask.data_ptr() if (mask and s.mask is not None) else None
        j.d_mask_out = s._mask_for(f).data_ptr() if mask_out else None
        j.d_stats = s.stats.data_ptr() if stats else None
    return arr


def _stages(sessions, frames, tp: TrackParams, mp: MaskParams, dynamic, stream):
    """The five stages of one step (the paper's Fig. 2 order) as callables that
    enqueue their launch sets on `stream`:

        registration without mask -> dynamic mask -> registration with mask
        -> block allocation -> integration

    A session whose first frame this is (k == 0) is only allocated and
    integrated at its initial pose."""
    if len(sessions) != len(frames):
        raise RefusionError("one frame per session")
    L = N.load()
    st = _stream(stream)
    run = [i for i, s in enumerate(sessions) if s.k > 0]
    rs = [sessions[i] for i in run]
    rf_ = [frames[i] for i in run]
    tpc, mpc = tp.c(), mp.c()

    def track1():
        if rs:
            _check(L.track_frame_batch(_jobs(rs, rf_, stats=True), len(rs), ctypes.byref(tpc), st),
                   "track_frame_batch")

    def mask():
        if rs and dynamic:
            _check(L.compute_dynamic_mask_batch(_jobs(rs, rf_, mask_out=True), len(rs), ctypes.byref(mpc), st),
                   "compute_dynamic_mask_batch")

    def track2():
        if rs and dynamic:
            _check(L.track_frame_batch(_jobs(rs, rf_, mask=True, stats=True), len(rs), ctypes.byref(tpc), st),
                   "track_frame_batch")

    def allocate_jobs():
        jobs = _jobs(sessions, frames)
        for i, s in enumerate(sessions):
            use = dynamic and s.k > 0 and s.mask is not None
            jobs[i].d_mask = s.mask.data_ptr() if use else None
        return jobs

    def allocate():
        _check(L.hashmap_allocate_batch(allocate_jobs(), len(sessions), st), "hashmap_allocate_batch")

    def integrate():
        _check(L.integrate_frame_batch(allocate_jobs(), len(sessions), st), "integrate_frame_batch")

    return [track1, mask, track2, allocate, integrate]


def process_batch(sessions, frames, tp: TrackParams, mp: MaskParams, dynamic=True, stream=None, events=None):
    """One step of the method for several sessions at once (one frame each),
    one launch set per stage (the paper's Fig. 2 order):

        registration without mask -> dynamic mask -> registration with mask
        -> block allocation -> integration

    A session's first frame is only allocated and integrated at its initial
    pose.  Every result is the same as processing the session alone.
    events: optional 6 torch.cuda.Event recorded on the stream before, between
    and after the five stages (for timing)."""
    tstream = stream if stream is not None else torch.cuda.current_stream()
    fns = _stages(sessions, frames, tp, mp, dynamic, tstream)
    if events is not None:
        events[0].record(tstream)
    for i, fn in enumerate(fns):
        fn()
        if events is not None:
            events[i + 1].record(tstream)
    for s in sessions:
        s.k += 1


class GraphStep:
    """process_batch recorded once as HIP graphs and replayed per step.

    A frame costs about seventy launches, most of them the short tracking
    iterations, so replaying a recorded graph removes most of the per-launch
    submission cost.  Kernel arguments (the frame's buffers among them) are
    fixed when recording, so the graphs read staging frames that this object
    owns; each call copies the step's frames into them on the stream first.
    The epoch that stamps allocated blocks advances on the device, so every
    replay does exactly what an eager step does (the GPU tests check each
    replay against eager steps bit for bit).

    Record after every session's first frame; frames must keep the staging
    frames' size, depth format and intrinsics.  split=True records one graph
    per stage so that events can be placed between the stages."""

    def __init__(self, sessions, frames_like, tp: TrackParams, mp: MaskParams, dynamic=True, split=False):
        if any(s.k == 0 for s in sessions):
            raise RefusionError("record a graph step after each session's first frame")
        if len(sessions) != len(frames_like):
            raise RefusionError("one frame per session")
        self.sessions = list(sessions)
        self.split = split
        self.staging = [Frame(torch.empty_like(f.depth), torch.empty_like(f.rgb), f.fx, f.fy, f.cx, f.cy,
                              f.depth_scale) for f in frames_like]
        for s, f in zip(self.sessions, self.staging):
            s._mask_for(f)
        side = torch.cuda.Stream()
        side.wait_stream(torch.cuda.current_stream())
        torch.cuda.synchronize()
        fns = _stages(self.sessions, self.staging, tp, mp, dynamic, side)
        groups = [[fn] for fn in fns] if split else [fns]
        self.graphs = []
        for grp in groups:
            g = torch.cuda.CUDAGraph()
            with torch.cuda.graph(g, stream=side):
                for fn in grp:
                    fn()
            self.graphs.append(g)
        torch.cuda.synchronize()

    def __call__(self, frames, stream=None, events=None):
        """Runs one step on `frames` (one per session).  events: optional 6
        torch.cuda.Event; with split=False only the first and last are recorded.
        The staging copies run between the first two."""
        if len(frames) != len(self.staging):
            raise RefusionError("one frame per session")
        for f, g in zip(frames, self.staging):
            if (f.depth.shape != g.depth.shape or f.depth.dtype != g.depth.dtype or f.s.fx != g.s.fx
                    or f.s.fy != g.s.fy or f.s.cx != g.s.cx or f.s.cy != g.s.cy
                    or f.s.depth_scale != g.s.depth_scale):
                raise RefusionError("frame does not match the recorded staging frame")
        stream = stream if stream is not None else torch.cuda.current_stream()
        with torch.cuda.stream(stream):
            if events is not None:
                events[0].record(stream)
            for f, g in zip(frames, self.staging):
                g.depth.copy_(f.depth, non_blocking=True)
                g.rgb.copy_(f.rgb, non_blocking=True)
            for i, gr in enumerate(self.graphs):
                gr.replay()
                if events is not None and self.split:
                    events[i + 1].record(stream)
            if events is not None and not self.split:
                events[5].record(stream)
        for s in self.sessions:
            s.k += 1


class VirtualDepth:
    """The second way of the paper to treat invalid depth (Sec. III-E): frames
    are collected n at a time; a temporary model is fused from them at their
    registered poses and cast from each pose, and each frame's zero depths are
    replaced by the virtual depth, or far_value where the rays meet no
    surface.  push() returns the n refined frames (float32 metres, same
    colour) once n have been collected, so the model they feed lags n frames.
    The temporary model reuses one arena."""

    def __init__(self, params: MapParams, n=10, z_near=0.3, far_value=None, device="cuda"):
        self.n = n
        self.z_near = z_near
        self.far_value = params.depth_max if far_value is None else far_value
        self.temp = Map(params, device)
        self.pending = []

    def push(self, frame: Frame, pose: torch.Tensor, stream=None):
        _dev(pose, "pose", torch.float64, (4, 4))
        self.pending.append((frame, pose.clone()))
        if len(self.pending) < self.n:
            return []
        L = self.temp.L
        _check(L.hashmap_reset(self.temp.h, _stream(stream)), "hashmap_reset")
        for f, P in self.pending:
            self.temp.allocate(f, P, stream=stream)
            self.temp.integrate(f, P, stream=stream)
        out = []
        for f, P in self.pending:
            d = self.temp.raycast(f, P, z_near=self.z_near, far_value=self.far_value, only_invalid=True,
                                  stream=stream)
            out.append((Frame(d, f.rgb, f.fx, f.fy, f.cx, f.cy, 1.0), P))
        self.pending = []
        return out


class Pipeline:
    """The per-frame method on one map with device-resident pose and mask
    (process_batch with a single session).  graph=True replays the steady-state
    step as a recorded HIP graph (GraphStep), recorded at the second frame."""

    def __init__(self, params: MapParams, tp: TrackParams, mp: MaskParams, initial_pose, dynamic=True,
                 device="cuda", graph=False):
        self.session = Session(params, initial_pose, device)
        self.tp, self.mp = tp, mp
        self.dynamic = dynamic
        self.graph = graph
        self._step = None

    @property
    def map(self):
        return self.session.map

    @property
    def pose(self):
        return self.session.pose

    @property
    def mask(self):
        return self.session.mask

    @property
    def stats(self):
        return self.session.stats

    def process(self, frame: Frame, stream=None):
        if self.graph and self.session.k > 0:
            if self._step is None:
                self._step = GraphStep([self.session], [frame], self.tp, self.mp, self.dynamic)
            self._step([frame], stream)
        else:
            process_batch([self.session], [frame], self.tp, self.mp, self.dynamic, stream)
        return self.session.pose
