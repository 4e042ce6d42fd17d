"""Seeded synthetic RGB-D sequences shaped like indoor 640x480 sensor data.

This package is the input generator shared by the CPU oracle tests, the GPU
parity tests and the benchmark.  It holds no arithmetic of the mapping method:
it builds analytic scenes and camera trajectories (numpy, seeded) and ray-casts
them with a small C++ renderer (``render.cpp``).

Workloads (sizes and parameters as named in the module-level builders):

* ``parity_room``   160x120 float32 depth, 2x2x2 m box room with one sphere,
                    fx=fy=120, cx=80, cy=60, camera moving 1 cm and 0.5 deg per
                    frame, no noise, voxel 2 cm, truncation 6 cm, 2^16 buckets,
                    2 pyramid levels x 10 Gauss-Newton iterations.
* ``static_room``   640x480 uint16 millimetre depth (0.3-5 m), 4x4x3 m room
                    with 20 textured boxes/spheres, Kinect-like axial noise
                    sigma = 0.0012 + 0.0019 (z-0.4)^2 and 2% dropout, voxel 1 cm,
                    truncation 3 cm, 2^20 buckets, 3 levels.
* ``dynamic_room``  static_room plus 1-3 rigid moving clusters (capsule
                    "people" and carried boxes, 0.5-1.5 m/s) with per-pixel
                    ground-truth dynamic labels.
* ``large_rooms``   10x10x3 m partitioned layout with 150 primitives, voxel
                    0.5 cm, 2^22 buckets.
"""
from __future__ import annotations

import ctypes
import dataclasses
import math
import os
import subprocess

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
_LIB_PATH = os.path.join(_HERE, "libsynth.so")
_lib = None

REC = 24  # floats per primitive record


def build(force: bool = True) -> str:
    """Compile the renderer with g++ (OpenMP) into synth/libsynth.so."""
    src = os.path.join(_HERE, "render.cpp")
    if force or not os.path.exists(_LIB_PATH):
        tmp = _LIB_PATH + ".tmp%d" % os.getpid()
        subprocess.check_call(["g++", "-O2", "-fopenmp", "-shared", "-fPIC", "-std=c++17",
                               src, "-o", tmp])
        os.replace(tmp, _LIB_PATH)
    return _LIB_PATH


def _load():
    global _lib
    if _lib is None:
        if not os.path.exists(_LIB_PATH):
            build(force=False)
        lib = ctypes.CDLL(_LIB_PATH)
        lib.synth_render.restype = ctypes.c_int
        lib.synth_render.argtypes = [
            ctypes.c_void_p, ctypes.c_int, ctypes.c_void_p, ctypes.c_int,
            ctypes.c_int, ctypes.c_int, ctypes.c_double, ctypes.c_double, ctypes.c_double,
            ctypes.c_double, ctypes.c_uint64, ctypes.c_int, ctypes.c_double, ctypes.c_double,
            ctypes.c_double, ctypes.c_double, ctypes.c_int, ctypes.c_int,
            ctypes.c_void_p, ctypes.c_void_p, ctypes.c_void_p, ctypes.c_void_p]
        _lib = lib
    return _lib


# ----------------------------------------------------------------------------
# primitives
# ----------------------------------------------------------------------------

def _prim(kind, label, centre, half, yaw=0.0, albedo=(0.7, 0.7, 0.7), freq=20.0,
          phase=(0.0, 0.0, 0.0), axis=(0.0, 0.0, 0.0)):
    r = np.zeros(REC, np.float32)
    r[0] = kind
    r[1] = label
    r[2:5] = centre
    r[5:8] = half
    r[8] = math.cos(yaw)
    r[9] = math.sin(yaw)
    r[10:13] = albedo
    r[13] = freq
    r[14:17] = phase
    r[17:20] = axis
    return r


def room(centre, half, rng):
    return _prim(0, 0, centre, half, albedo=rng.uniform(0.45, 0.95, 3),
                 freq=rng.uniform(2 * math.pi / 0.6, 2 * math.pi / 0.2), phase=rng.uniform(0, 6.28, 3))


def box(centre, half, yaw, rng, label=0):
    return _prim(1, label, centre, half, yaw, albedo=rng.uniform(0.25, 1.0, 3),
                 freq=rng.uniform(2 * math.pi / 0.5, 2 * math.pi / 0.12), phase=rng.uniform(0, 6.28, 3))


def sphere(centre, radius, rng, label=0):
    return _prim(2, label, centre, (radius, 0, 0), albedo=rng.uniform(0.25, 1.0, 3),
                 freq=rng.uniform(2 * math.pi / 0.4, 2 * math.pi / 0.1), phase=rng.uniform(0, 6.28, 3))


def capsule(centre, half_axis, radius, rng, label=0):
    return _prim(3, label, centre, (radius, 0, 0), albedo=rng.uniform(0.25, 1.0, 3),
                 freq=rng.uniform(2 * math.pi / 0.4, 2 * math.pi / 0.1), phase=rng.uniform(0, 6.28, 3),
                 axis=half_axis)


# ----------------------------------------------------------------------------
# camera poses (row-major 4x4, camera->world; camera x right, y down, z forward)
# ----------------------------------------------------------------------------

def look_pose(position, yaw, pitch, roll=0.0):
    f = np.array([math.cos(pitch) * math.cos(yaw), math.cos(pitch) * math.sin(yaw), math.sin(pitch)])
    r = np.cross(f, [0.0, 0.0, 1.0])
    r /= np.linalg.norm(r)
    d = np.cross(f, r)
    if roll:
        c, s = math.cos(roll), math.sin(roll)
        r, d = c * r + s * d, -s * r + c * d
    T = np.eye(4)
    T[:3, 0], T[:3, 1], T[:3, 2], T[:3, 3] = r, d, f, position
    return T


def axis_angle(axis, angle):
    a = np.asarray(axis, float)
    a = a / np.linalg.norm(a)
    K = np.array([[0, -a[2], a[1]], [a[2], 0, -a[0]], [-a[1], a[0], 0]])
    return np.eye(3) + math.sin(angle) * K + (1 - math.cos(angle)) * K @ K


@dataclasses.dataclass
class Sequence:
    """A rendered RGB-D sequence plus everything a pipeline run needs."""
    name: str
    width: int
    height: int
    fx: float
    fy: float
    cx: float
    cy: float
    poses: np.ndarray            # (n, 4, 4) float64 ground-truth camera->world
    depth: np.ndarray            # (n, H, W) float32 metres or uint16 millimetres
    rgb: np.ndarray              # (n, H, W, 3) uint8
    labels: np.ndarray           # (n, H, W) uint8, >0 where the first hit moves
    depth_scale: float           # metres per depth unit (1.0 for float32 input)
    voxel_size: float
    truncation: float
    depth_max: float
    num_buckets: int
    levels: int
    iters: int
    carve_stride: int
    seed: int
    prims: np.ndarray = None     # static primitives of the scene (records as rendered), for accuracy metrics

    @property
    def n(self):
        return self.poses.shape[0]

    @property
    def intrinsics(self):
        return (self.fx, self.fy, self.cx, self.cy)


def render(prims_per_frame, poses, W, H, fx, fy, cx, cy, seed, frame0=0, noise=False,
           dropout=0.0, float_depth=False, min_mm=300, max_mm=5000):
    lib = _load()
    prims_per_frame = np.ascontiguousarray(prims_per_frame, np.float32)
    poses = np.ascontiguousarray(poses, np.float64)
    n, n_prims = prims_per_frame.shape[0], prims_per_frame.shape[1]
    assert poses.shape == (n, 4, 4)
    rgb = np.zeros((n, H, W, 3), np.uint8)
    labels = np.zeros((n, H, W), np.uint8)
    d32 = np.zeros((n, H, W), np.float32) if float_depth else None
    d16 = None if float_depth else np.zeros((n, H, W), np.uint16)
    a, b, z0 = (0.0012, 0.0019, 0.4) if noise else (0.0, 0.0, 0.0)
    rc = lib.synth_render(prims_per_frame.ctypes.data, n_prims, poses.ctypes.data, n, W, H,
                          fx, fy, cx, cy, seed, frame0, a, b, z0, dropout, min_mm, max_mm,
                          d32.ctypes.data if d32 is not None else None,
                          d16.ctypes.data if d16 is not None else None,
                          rgb.ctypes.data, labels.ctypes.data)
    if rc != 0:
        raise RuntimeError("synth_render failed (%d)" % rc)
    return (d32 if float_depth else d16), rgb, labels


# ----------------------------------------------------------------------------
# workloads
# ----------------------------------------------------------------------------

def parity_room(n_frames=10, seed=1905020821):
    """160x120 float depth of a 2x2x2 m room holding one sphere (radius 0.3 m).

    The camera starts near the room centre looking into a corner and moves by
    exactly 1 cm along a smoothly turning heading and rotates by exactly 0.5 deg
    about a smoothly turning axis per frame.
    """
    rng = np.random.default_rng(seed)
    W, H, fx, fy, cx, cy = 160, 120, 120.0, 120.0, 80.0, 60.0
    prims = [room((0, 0, 0), (1, 1, 1), rng),
             sphere((0.35, 0.30, -0.45), 0.3, rng)]
    P = np.stack(prims)
    T0 = look_pose(np.array([-0.45, -0.45, 0.15]), yaw=math.radians(45), pitch=math.radians(-28))
    a0, b0, c0 = rng.uniform(0, 2 * math.pi, 3)
    poses = [T0]
    for k in range(1, n_frames):
        T = poses[-1].copy()
        h = np.array([math.cos(a0 + 0.15 * k), math.sin(a0 + 0.15 * k), 0.3 * math.sin(b0 + 0.2 * k)])
        T[:3, 3] += 0.01 * h / np.linalg.norm(h)
        ax = np.array([0.3 * math.cos(c0 + 0.1 * k), 0.3 * math.sin(c0 + 0.1 * k), 1.0])
        T[:3, :3] = axis_angle(ax, math.radians(0.5)) @ T[:3, :3]
        poses.append(T)
    poses = np.stack(poses)
    depth, rgb, labels = render(np.repeat(P[None], n_frames, 0), poses, W, H, fx, fy, cx, cy,
                                seed, float_depth=True)
    return Sequence("parity_room", W, H, fx, fy, cx, cy, poses, depth, rgb, labels, 1.0,
                    voxel_size=0.02, truncation=0.06, depth_max=5.0, num_buckets=1 << 16,
                    levels=2, iters=10, carve_stride=2, seed=seed)


def _furnished_room(rng, half=(2.0, 2.0, 1.5), n_objects=20, clear_radius=1.45):
    """Room of the given half size (floor at z=0) with textured boxes/spheres
    along the walls, keeping a disc of ``clear_radius`` around the centre free."""
    hx, hy, hz = half
    prims = [room((0, 0, hz), half, rng)]
    while len(prims) < n_objects + 1:
        ang = rng.uniform(0, 2 * math.pi)
        rad = rng.uniform(clear_radius + 0.25, max(hx, hy))
        x, y = rad * math.cos(ang), rad * math.sin(ang)
        if abs(x) > hx - 0.1 or abs(y) > hy - 0.1:
            continue
        if rng.uniform() < 0.6:
            h = rng.uniform([0.1, 0.1, 0.1], [0.3, 0.3, 0.6])
            z = h[2] if rng.uniform() < 0.7 else rng.uniform(0.5, 2.0)
            prims.append(box((x, y, z), h, rng.uniform(0, math.pi), rng))
        else:
            r = rng.uniform(0.1, 0.3)
            z = r if rng.uniform() < 0.5 else rng.uniform(0.5, 2.2)
            prims.append(sphere((x, y, z), r, rng))
    return prims


def _orbit_trajectory(rng, n_frames, centre_z=1.4, radius=0.35, step_cm=(0.5, 2.0), rot_deg=(0.25, 1.0)):
    """Smooth seeded camera path in the central free disc.  Translation per
    frame varies in step_cm, rotation per frame in rot_deg."""
    w = rng.uniform(0.6, 1.4, 3)
    ph = rng.uniform(0, 2 * math.pi, 6)
    yaw0 = rng.uniform(0, 2 * math.pi)
    poses = []
    s = 0.0
    yaw = yaw0
    for k in range(n_frames):
        # path parameter advances by a smoothly varying step so that the
        # translation per frame sweeps step_cm
        spd = 0.5 * (step_cm[0] + step_cm[1]) + 0.5 * (step_cm[1] - step_cm[0]) * math.sin(0.021 * k + ph[3])
        rot = 0.5 * (rot_deg[0] + rot_deg[1]) + 0.5 * (rot_deg[1] - rot_deg[0]) * math.sin(0.017 * k + ph[4])
        pos = np.array([radius * math.sin(w[0] * s + ph[0]), radius * math.sin(w[1] * s + ph[1]),
                        centre_z + 0.1 * math.sin(w[2] * s + ph[2])])
        pitch = math.radians(-22) + 0.1 * math.sin(0.013 * k + ph[5])
        poses.append(look_pose(pos, yaw, pitch))
        # advance: approximate arc length of the position curve
        dp = np.array([radius * w[0] * math.cos(w[0] * s + ph[0]), radius * w[1] * math.cos(w[1] * s + ph[1]),
                       0.1 * w[2] * math.cos(w[2] * s + ph[2])])
        s += (spd * 0.01) / max(np.linalg.norm(dp), 1e-3)
        yaw += math.radians(rot) * 0.9
    return np.stack(poses)


def _movers(rng, n_clusters, half, sweep):
    """Moving rigid clusters on circular floor paths around the room centre."""
    clusters = []
    for cid in range(1, n_clusters + 1):
        speed = rng.uniform(0.5, 1.5) / 30.0          # m per frame at 30 Hz
        radius = rng.uniform(0.95, 1.3)
        phase = rng.uniform(0, 2 * math.pi)
        if sweep:                                     # start near the end of the swing: out of view
            phase = 0.3 * (phase / (2 * math.pi) - 0.5)
        direction = 1 if rng.uniform() < 0.5 else -1
        parts = []
        if rng.uniform() < 0.6:
            tall = rng.uniform(1.2, 1.8)
            parts.append(capsule((0, 0, tall * 0.45), (0, 0, tall * 0.3), rng.uniform(0.14, 0.22), rng, cid))
            parts.append(sphere((0, 0, tall * 0.9), 0.11, rng, cid))
            parts.append(capsule((0.12, 0, tall * 0.55), (0.1, 0.0, 0.12), 0.06, rng, cid))
        else:
            tall = rng.uniform(0.2, 1.2)
            parts.append(box((0, 0, tall / 2), (rng.uniform(0.15, 0.35), rng.uniform(0.15, 0.35), tall / 2),
                             0.0, rng, cid))
            parts.append(box((0, 0, tall + 0.1), (0.12, 0.12, 0.1), 0.3, rng, cid))
        clusters.append(dict(speed=speed, radius=radius, phase=phase, dir=direction, parts=parts, sweep=sweep))
    return clusters


def _place_movers(clusters, k, cam_pose):
    """Cluster placement at frame k: each cluster walks back and forth across
    the camera's heading on a circle about the room centre at its own speed.
    "sweep" clusters swing +-1.2 rad about the heading (the view is about
    +-0.55 rad wide), so they enter and leave the view, and start outside it;
    "in_view" clusters swing +-0.55 rad from a random phase, so short
    sequences always see them."""
    f = cam_pose[:3, 2]
    yaw = math.atan2(f[1], f[0])
    out = []
    for c in clusters:
        if c["sweep"]:
            amp = 1.2
            ang = yaw + c["dir"] * amp * math.cos(c["speed"] / (c["radius"] * amp) * k + c["phase"])
        else:
            amp = 0.55
            ang = yaw + c["dir"] * amp * math.sin(c["speed"] / (c["radius"] * amp) * k + c["phase"])
        ox, oy = c["radius"] * math.cos(ang), c["radius"] * math.sin(ang)
        for p in c["parts"]:
            q = p.copy()
            q[2] += ox
            q[3] += oy
            out.append(q)
    return out


def static_room(n_frames=300, seed=1905020822, width=640, height=480):
    rng = np.random.default_rng(seed)
    prims = _furnished_room(rng)
    fx = fy = 525.0 * width / 640.0
    cx, cy = (width - 1) / 2.0, (height - 1) / 2.0
    poses = _orbit_trajectory(rng, n_frames)
    P = np.stack(prims)
    depth, rgb, labels = render(np.repeat(P[None], n_frames, 0), poses, width, height, fx, fy, cx, cy,
                                seed, noise=True, dropout=0.02)
    return Sequence("static_room", width, height, fx, fy, cx, cy, poses, depth, rgb, labels, 0.001,
                    voxel_size=0.01, truncation=0.03, depth_max=5.0, num_buckets=1 << 20,
                    levels=3, iters=10, carve_stride=4, seed=seed, prims=P)


def dynamic_room(n_frames=400, seed=1905020823, width=640, height=480, n_clusters=None, movers="sweep"):
    """Furnished room with 1-3 moving clusters (people-sized capsules or
    boxes).  movers="sweep": clusters walk into and out of the view and are
    outside it at frame 0 (the long-sequence workload); movers="in_view":
    clusters stay near the view centre from frame 0 (short parity cases)."""
    if movers not in ("sweep", "in_view"):
        raise ValueError("movers must be 'sweep' or 'in_view'")
    rng = np.random.default_rng(seed)
    prims = _furnished_room(rng)
    fx = fy = 525.0 * width / 640.0
    cx, cy = (width - 1) / 2.0, (height - 1) / 2.0
    poses = _orbit_trajectory(rng, n_frames)
    clusters = _movers(rng, int(n_clusters or rng.integers(1, 4)), (2.0, 2.0, 1.5), movers == "sweep")
    frames = [np.stack(prims + _place_movers(clusters, k, poses[k])) for k in range(n_frames)]
    depth, rgb, labels = render(np.stack(frames), poses, width, height, fx, fy, cx, cy,
                                seed, noise=True, dropout=0.02)
    return Sequence("dynamic_room", width, height, fx, fy, cx, cy, poses, depth, rgb, labels, 0.001,
                    voxel_size=0.01, truncation=0.03, depth_max=5.0, num_buckets=1 << 20,
                    levels=3, iters=10, carve_stride=4, seed=seed)


def large_rooms(n_frames=1000, seed=1905020824, width=640, height=480, n_objects=150):
    """10x10x3 m floor split by partition walls with doorways; 150 primitives
    outside the camera's loop corridor."""
    rng = np.random.default_rng(seed)
    prims = [room((0, 0, 1.5), (5.0, 5.0, 1.5), rng)]
    # partition walls (thin boxes) leaving doorways where the loop passes
    loop_r = 2.6
    for x in (-3.3, 3.3):
        prims.append(box((x, 2.6, 1.5), (0.05, 2.4, 1.5), 0.0, rng))
        prims.append(box((x, -2.6, 1.5), (0.05, 2.4, 1.5), 0.0, rng))
    while len(prims) < n_objects:
        x, y = rng.uniform(-4.8, 4.8, 2)
        if abs(math.hypot(x, y) - loop_r) < 0.9:
            continue
        if rng.uniform() < 0.6:
            h = rng.uniform([0.1, 0.1, 0.1], [0.4, 0.4, 0.7])
            prims.append(box((x, y, h[2]), h, rng.uniform(0, math.pi), rng))
        else:
            r = rng.uniform(0.1, 0.35)
            prims.append(sphere((x, y, r if rng.uniform() < 0.5 else rng.uniform(0.5, 2.2)), r, rng))
    fx = fy = 525.0 * width / 640.0
    cx, cy = (width - 1) / 2.0, (height - 1) / 2.0
    poses = []
    ang = rng.uniform(0, 2 * math.pi)
    for k in range(n_frames):
        spd = 0.0125 + 0.0075 * math.sin(0.02 * k)
        pos = np.array([loop_r * math.cos(ang), loop_r * math.sin(ang), 1.4 + 0.1 * math.sin(0.03 * k)])
        yaw = ang + math.pi / 2 + 0.6 * math.sin(0.011 * k)
        poses.append(look_pose(pos, yaw, math.radians(-20)))
        ang += spd / loop_r
    poses = np.stack(poses)
    P = np.stack(prims)
    depth, rgb, labels = render(np.repeat(P[None], n_frames, 0), poses, width, height, fx, fy, cx, cy,
                                seed, noise=True, dropout=0.02)
    # depth_max 3.5 m: beyond it the axial noise (sigma 2 cm at 3.5 m, 3.8 cm at 4.8 m) exceeds the
    # 3 cm truncation and biases registration (about 1 cm per frame at 5 m in this layout)
    return Sequence("large_rooms", width, height, fx, fy, cx, cy, poses, depth, rgb, labels, 0.001,
                    voxel_size=0.005, truncation=0.03, depth_max=3.5, num_buckets=1 << 22,
                    levels=3, iters=10, carve_stride=2, seed=seed, prims=P)


def depth_metres(seq: Sequence, k: int) -> np.ndarray:
    """Frame k's depth as float32 metres (raw * scale in float32)."""
    d = seq.depth[k]
    if d.dtype == np.float32:
        return d
    return d.astype(np.float32) * np.float32(seq.depth_scale)
