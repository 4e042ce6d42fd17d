"""Closed-form inputs for pins and parity cases.

* ``fill_map``: a voxel-block map (sorted int32 keys, sdf, weight, RGB8) whose
  voxel values are a given analytic field sampled at the voxel centres v*s.
* ``ray_depth``: depth images of analytic planes/spheres from a pinhole camera.
* ``scene_distance``: distance of points to the surface of a rendered scene's
  static primitives (the ground truth of the synthetic model-accuracy metric).

These are input generators only; they hold none of the mapping method's
arithmetic (no interpolation, projection rules, averaging or tracking).
"""
from __future__ import annotations

import numpy as np


def block_voxel_centres(keys, voxel_size):
    """(n,512,3) float64 centres of the voxels of the given blocks; the local
    index is lx + 8 ly + 64 lz."""
    keys = np.asarray(keys, np.int64)
    l = np.arange(512)
    local = np.stack([l & 7, (l >> 3) & 7, l >> 6], -1)
    v = keys[:, None, :] * 8 + local[None]
    return v.astype(np.float64) * float(np.float32(voxel_size))


def blocks_near(points, voxel_size, pad_blocks=1):
    """Sorted unique block keys within pad_blocks of the given world points."""
    B = 8 * float(np.float32(voxel_size))
    b = np.floor(np.asarray(points) / B).astype(np.int64)
    offs = np.stack(np.meshgrid(*[np.arange(-pad_blocks, pad_blocks + 1)] * 3, indexing="ij"), -1).reshape(-1, 3)
    allk = (b[:, None, :] + offs[None]).reshape(-1, 3)
    return np.unique(allk, axis=0).astype(np.int32)


def fill_map(keys, voxel_size, sdf_fn, rgb_fn=None, weight=1.0):
    keys = np.asarray(keys, np.int32)
    c = block_voxel_centres(keys, voxel_size)
    sdf = np.asarray(sdf_fn(c), np.float64).reshape(len(keys), 512)
    w = np.full((len(keys), 512), weight, np.float64)
    if rgb_fn is None:
        rgb = np.full((len(keys), 512, 3), 128, np.uint8)
    else:
        rgb = np.clip(np.rint(rgb_fn(c)), 0, 255).astype(np.uint8).reshape(len(keys), 512, 3)
    return keys, sdf, w, rgb


def camera_rays(W, H, fx, fy, cx, cy):
    u, v = np.meshgrid(np.arange(W, dtype=np.float64), np.arange(H, dtype=np.float64))
    return np.stack([(u - cx) / fx, (v - cy) / fy, np.ones_like(u)], -1)  # camera z = 1


def ray_depth_planes(pose, W, H, fx, fy, cx, cy, planes):
    """Depth (float64, camera z) of the first hit among planes n.p = d
    (each plane given as (n, d)); also returns the world hit points and the
    index of the plane hit (-1: none)."""
    dc = camera_rays(W, H, fx, fy, cx, cy)
    R, o = pose[:3, :3], pose[:3, 3]
    d = dc @ R.T
    best = np.full((H, W), np.inf)
    idx = np.full((H, W), -1)
    for k, (n, off) in enumerate(planes):
        n = np.asarray(n, np.float64)
        den = d @ n
        with np.errstate(divide="ignore", invalid="ignore"):
            t = (off - o @ n) / den
        ok = (den != 0) & (t > 1e-9) & (t < best)
        best = np.where(ok, t, best)
        idx = np.where(ok, k, idx)
    pts = o + best[..., None] * d
    return best, pts, idx


def ray_depth_sphere(pose, W, H, fx, fy, cx, cy, centre, radius, background=None):
    dc = camera_rays(W, H, fx, fy, cx, cy)
    R, o = pose[:3, :3], pose[:3, 3]
    d = dc @ R.T
    oc = o - np.asarray(centre, np.float64)
    a = np.einsum("hwi,hwi->hw", d, d)
    b = d @ oc
    c = oc @ oc - radius * radius
    disc = b * b - a * c
    t = np.where(disc >= 0, (-b - np.sqrt(np.maximum(disc, 0))) / a, np.inf)
    t = np.where(t > 1e-9, t, np.inf)
    if background is not None:
        t = np.minimum(t, background)
    return t


def scene_distance(prims, points):
    """Unsigned distance (float64) of each point to the nearest surface of the
    primitives (records as synth renders them: room interior, boxes with yaw
    about world z, spheres, capsules)."""
    pts = np.asarray(points, np.float64).reshape(-1, 3)
    best = np.full(len(pts), np.inf)
    for r in np.asarray(prims, np.float64):
        kind, c, h = int(r[0]), r[2:5], r[5:8]
        d = pts - c
        if kind in (0, 1):
            co, si = (r[8], r[9]) if kind == 1 else (1.0, 0.0)
            local = np.stack([co * d[:, 0] + si * d[:, 1], -si * d[:, 0] + co * d[:, 1], d[:, 2]], 1)
            q = np.abs(local) - h
            sd = np.linalg.norm(np.maximum(q, 0.0), axis=1) + np.minimum(q.max(axis=1), 0.0)
            dist = np.abs(sd)
        elif kind == 2:
            dist = np.abs(np.linalg.norm(d, axis=1) - h[0])
        else:
            a = r[17:20]
            p0 = c - a
            ba = 2.0 * a
            t = np.clip(((pts - p0) @ ba) / max(float(ba @ ba), 1e-300), 0.0, 1.0)
            dist = np.abs(np.linalg.norm(pts - (p0 + t[:, None] * ba), axis=1) - h[0])
        best = np.minimum(best, dist)
    return best
