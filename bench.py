#!/usr/bin/env python3
"""Throughput of the ReFusion per-frame hot path on one MI355X.

Headline workload (default): the large rooms -- a 10x10x3 m multi-room
layout with 150 textured primitives, 1000 frames of 640x480 uint16
millimetre depth (0.3-5 m) + RGB8 with Kinect-like axial noise and 2%
dropout; voxel 0.5 cm, truncation 3 cm, 8^3 blocks, 2^22 buckets, clipping
plane 3.5 m (measurements beyond it carve free space up to it), 3-level
pyramid x 10 Gauss-Newton iterations, Table I weights (w_c 0.025, theta
0.007, gamma 0.5), FP32 storage.

One step = one frame through the whole method: registration without mask,
residual mask with flood fill, registration with the mask, block allocation
with carve rays, integration with free-space carving.  The whole sequence is
fused: frame 0 initialises the map, the frames up to the last K + W build it
untimed, W warmup frames follow, and the last K frames are timed.  All
inputs are on the device before the timed region (the host-to-device upload
of a frame is measured apart, "h2d").

Prints ONE JSON line.  Kernel durations are measured with HIP events on the
stream the kernels run on.  "roofline" is the dominant kernel (the tracking
sweep): its algorithmic bytes come from the host footprint of sampled frames
(distinct voxel records and buckets a sweep reads, plus image bytes).
"roofline_integrate" is the integration kernel, whose algorithmic bytes come
from device counters of voxel updates.  Extra measurements after the
headline: the same sequence in FP16+u8 storage ("fp16", with its final pose
against FP32's), with compact free space ("compact": blocks carved whole,
free blocks without voxels; its final pose against the per-voxel map's and
its voxel memory), with the clipping plane at 5 m ("depth_max_5m"), the
640x480 static room of 300 frames at 1 cm voxels ("static_room"), and the
640x480 dynamic room of 400 frames with moving clusters ("dynamic_room", with
the dynamic mask's IoU against the generator's mover labels).  The CPU oracle
is timed on a bounded sample of the headline sequence, single-thread and with
all host cores, per stage too ("cpu_baseline").
"""
from __future__ import annotations

import argparse
import ctypes
import json
import math
import os
import sys
import time

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

METRIC = "640x480 frames/sec tracked+fused (HBM GB/s % peak); p50/p99 frame latency"
HBM_PEAK_GBS = 8000.0
ACC_MAX_TRIANGLES = 4_000_000     # larger meshes: accuracy on a sample of their triangles
ACC_SAMPLE_TRIANGLES = 300_000


def log(*a):
    print(*a, file=sys.stderr, flush=True)


def profile_key(seq_name, n, storage, depth_max, K):
    """The measurement a PMC summary applies to."""
    return "%s:%d frames:%s:depth_max %.3g:last %d timed" % (seq_name, n, storage, depth_max, K)


def traffic_from_profile(kernel, key):
    """(HBM bytes per launch, L2 hit rate) of `kernel` from the committed
    rocprofv3 PMC summary of the same measurement (FETCH_SIZE + WRITE_SIZE,
    calibrated; TCC_HIT / (TCC_HIT + TCC_MISS)), if it was taken on the same
    workload key (sequence, length, storage, depth_max, timed frames) and on
    the current kernel source; else (None, None)."""
    wl, _, st = key.split(":")[:3]
    path = os.path.join(ROOT, "profiles", "%s_%s_%s_pmc.json" % (kernel.replace("_kernel", ""), wl, st))
    if not os.path.exists(path):
        return None, None
    with open(path) as fh:
        d = json.load(fh)
    from paper_1905_02082_amd.profiling import kernel_source_hash
    if d.get("kernel_source_hash") != kernel_source_hash(kernel) or d.get("workload") != key:
        return None, None
    return d.get("hbm_bytes_per_launch"), d.get("l2_hit_rate")


def track_footprint(seq, block_keys, frame_ids, storage):
    """Algorithmic bytes of one tracking sweep (one track_kernel launch) per
    pyramid level, averaged over frame_ids: every distinct voxel record a
    trilinear lookup reads (corners inside allocated blocks), one hash bucket
    per distinct corner block, the depth and colour of every pixel of the
    level (and its mask byte in the masked pass), and the 29 FP64 sums
    written.  Host arithmetic on the ground-truth pose of each frame."""
    import numpy as np
    rec = {"fp32": 12, "fp16": 8}[storage]
    bkeys = np.asarray(block_keys, dtype=np.int64)
    enc = lambda b: ((b[:, 0] + (1 << 20)) << 42) | ((b[:, 1] + (1 << 20)) << 21) | (b[:, 2] + (1 << 20))
    have = np.sort(enc(bkeys)) if len(bkeys) else np.zeros(0, np.int64)
    fx, fy, cx, cy = seq.intrinsics
    corners = np.array([[i & 1, (i >> 1) & 1, i >> 2] for i in range(8)], dtype=np.int64)
    out = np.zeros(seq.levels)
    pix = np.zeros(seq.levels)
    for k in frame_ids:
        D = seq.depth[k].astype(np.float64) * (seq.depth_scale if seq.depth[k].dtype == np.uint16 else 1.0)
        T = seq.poses[k]
        for lv in range(seq.levels):
            st = 1 << lv
            d = D[::st, ::st]
            v, u = np.mgrid[0:seq.height:st, 0:seq.width:st]
            ok = (d > 0) & (d <= seq.depth_max)
            x = np.stack([(u[ok] - cx) / fx * d[ok], (v[ok] - cy) / fy * d[ok], d[ok]], 1)
            y = x @ T[:3, :3].T + T[:3, 3]
            g = np.floor(y / seq.voxel_size).astype(np.int64)
            vox = (g[:, None, :] + corners[None]).reshape(-1, 3)
            blk = np.floor_divide(vox, 8)
            bid = enc(blk)
            ub = np.unique(bid)
            alloc = np.isin(bid, have, assume_unique=False)
            voxel_ids = np.unique(enc(vox[alloc] + (1 << 19)))  # any injective code of the voxel
            out[lv] += voxel_ids.size * rec + ub.size * 16 + d.size * (2 + 3) + 29 * 8
            pix[lv] += d.size
    return out / max(len(frame_ids), 1), pix / max(len(frame_ids), 1)


def mesh_measurement(m, seq, storage, reps=5):
    """Marching-tetrahedra mesh of the fused map, after the timed region: the
    extraction time (HIP events around extract_mesh on its stream), its HBM
    roofline (algorithmic bytes = every live voxel record read once plus the
    triangles written) and the model accuracy: distance of the unique mesh
    vertices to the scene's analytic surfaces."""
    import numpy as np
    import torch
    from synth.analytic import scene_distance
    tris = m.mesh()
    n = int(tris.shape[0])
    cap = max(n, 1)
    buf = torch.empty((cap, 3, 3), dtype=torch.float32, device=m.device)
    cnt = torch.zeros(1, dtype=torch.int32, device=m.device)
    stream = torch.cuda.current_stream()
    ms = []
    for _ in range(reps):
        e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
        e0.record(stream)
        m.L.extract_mesh(m.h, ctypes.c_void_p(buf.data_ptr()), cap, ctypes.c_void_p(cnt.data_ptr()),
                         ctypes.c_void_p(stream.cuda_stream))
        e1.record(stream)
        torch.cuda.synchronize()
        ms.append(e0.elapsed_time(e1))
    t = float(np.median(ms))
    _, nb = m.status()
    rec = {"fp32": 8, "fp16": 4}[storage]
    alg = nb * 512 * rec + n * 36
    achieved = alg / (t * 1e-3) / 1e9
    out = {"triangles": n, "blocks": nb, "extract_ms": round(t, 4), "triangles_per_s": round(n / (t * 1e-3), 1),
           "roofline": {"kernels": "mesh_count_kernel + mesh_scan_kernel + mesh_write_kernel", "bound": "hbm",
                        "achieved": round(achieved, 2), "peak": HBM_PEAK_GBS, "unit": "GB/s",
                        "frac": round(achieved / HBM_PEAK_GBS, 4), "alg_bytes": int(alg), "traffic": None}}
    log("mesh: %d triangles from %d blocks, %.2f ms per extraction" % (n, nb, t))
    if seq.prims is not None and n:
        # the accuracy of a large mesh is taken on a seeded sample of its
        # triangles (the host distance evaluation is the slow part)
        T = tris.cpu().numpy()
        sampled = n > ACC_MAX_TRIANGLES
        if sampled:
            T = T[np.random.default_rng(1905020826).choice(n, ACC_SAMPLE_TRIANGLES, replace=False)]
        t0 = time.perf_counter()
        V = np.unique(T.reshape(-1, 3).astype(np.float64), axis=0)
        d = scene_distance(seq.prims, V)
        log("mesh: accuracy on %d vertices in %.1f s" % (len(V), time.perf_counter() - t0))
        out["accuracy"] = {"vertices": int(len(V)),
                           "sample": ("the vertices of %d of the %d triangles (seeded)" % (ACC_SAMPLE_TRIANGLES, n)
                                      if sampled else "every vertex"),
                           "mean_mm": round(1e3 * float(d.mean()), 3),
                           "median_mm": round(1e3 * float(np.median(d)), 3),
                           "p90_mm": round(1e3 * float(np.percentile(d, 90)), 3),
                           "within_mm": {str(x): round(float((d <= x * 1e-3).mean()), 4) for x in (1, 2, 5, 10, 20)}}
    return out


def virtual_depth_measurement(m, seq, frame, pose, reps=5):
    """Ray casting the fused map from the last frame's registered pose
    (Sec. III-E): every pixel (the virtual depth image) and the fill of the
    frame's zero depths; HIP-event time per call and, for the fill, the
    fraction of zeros that the model explains."""
    import numpy as np
    import torch
    stream = torch.cuda.current_stream()
    res = {}
    for name, only in (("all_pixels", False), ("fill_zeros", True)):
        out = m.raycast(frame, pose, only_invalid=only)
        ms = []
        for _ in range(reps):
            e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
            e0.record(stream)
            m.raycast(frame, pose, only_invalid=only, out=out)
            e1.record(stream)
            torch.cuda.synchronize()
            ms.append(e0.elapsed_time(e1))
        res[name + "_ms"] = round(float(np.median(ms)), 4)
        if only:
            z = out.cpu().numpy()
            zeros = frame.depth.cpu().numpy() == 0
            res["zero_pixels"] = int(zeros.sum())
            res["zeros_explained"] = round(float((z[zeros] != m.params.depth_max).mean()) if zeros.any() else 0.0, 4)
        else:
            res["pixels_with_surface"] = round(float((out > 0).float().mean().item()), 4)
    return res


WORKLOAD_FRAMES = {"large_rooms": 1000, "static_room": 300, "dynamic_room": 400}
WORKLOAD_BLOCKS = {"large_rooms": 3 << 20, "static_room": 1 << 18, "dynamic_room": 1 << 18}


def make_sequence(workload, n):
    import synth
    if workload == "static_room":
        return synth.static_room(n_frames=n)
    if workload == "dynamic_room":
        return synth.dynamic_room(n_frames=n)
    if workload == "large_rooms":
        return synth.large_rooms(n_frames=n)
    raise SystemExit("unknown workload %s" % workload)


def cpu_baseline(seq, budget_s=30.0, threads=1):
    """The oracle as it stands: frame 0 fusion, then full frames until the
    time budget is spent; returns frames/s of the full frames, the sample
    description and the threads used.  threads > 1 runs the oracle's OpenMP
    build (the same source, loops over pixels and blocks shared out) with
    that many threads."""
    import oracle as O
    lib = O.load_variant("omp" if threads > 1 else "serial")
    if threads > 1:
        lib.orc_set_threads(threads)
    a = O.OracleMap(seq.voxel_size, seq.truncation, seq.depth_max, 255, seq.carve_stride, real_bits=64, lib=lib)
    b = O.OracleMap(seq.voxel_size, seq.truncation, seq.depth_max, 255, seq.carve_stride, real_bits=32, lib=lib)
    T = seq.poses[0]
    fr = O.Frame(seq.depth[0], seq.rgb[0], *seq.intrinsics, depth_scale=seq.depth_scale)
    T, _ = O.process_frame(a, fr, T, 0, seq.levels, seq.iters, mask_map=b)
    done, spent = 0, 0.0
    times = {}
    k = 1
    while k < seq.n and (done == 0 or spent < budget_s):
        fr = O.Frame(seq.depth[k], seq.rgb[k], *seq.intrinsics, depth_scale=seq.depth_scale)
        t0 = time.perf_counter()
        T, _ = O.process_frame(a, fr, T, k, seq.levels, seq.iters, mask_map=b, times=times)
        spent += time.perf_counter() - t0
        done += 1
        k += 1
        log("cpu oracle (%d threads) frame %d: %.2f s" % (threads, k - 1, spent / done))
    used = lib.orc_get_threads() if threads > 1 else 1
    stages = {k2: round(1000.0 * v / done, 2) for k2, v in times.items()}
    return done / spent, ("frames 1-%d of the headline sequence (full method per frame after frame-0 fusion), "
                          "FP64 oracle + FP32 mask mirror, %s" % (done, "%d OpenMP threads" % used if threads > 1
                                                                  else "single thread")), used, stages


def host_cpu():
    """(logical CPUs usable by this process, CPU model name)."""
    n = len(os.sched_getaffinity(0)) if hasattr(os, "sched_getaffinity") else os.cpu_count()
    model = None
    try:
        with open("/proc/cpuinfo") as fh:
            for line in fh:
                if line.startswith("model name"):
                    model = line.split(":", 1)[1].strip()
                    break
    except OSError:
        pass
    return n, model


def upload_frames(seq, dev):
    """Every frame of the sequence on the device (before any timed region)."""
    import paper_1905_02082_amd as rf
    return [rf.Frame.from_numpy(seq.depth[k], seq.rgb[k], *seq.intrinsics, depth_scale=seq.depth_scale,
                                device=dev) for k in range(seq.n)]


def h2d_measurement(seq, frames, ks, dev):
    """Host-to-device upload of the frames ks from pinned host memory on the
    stream the kernels use (HIP events): the PCIe share of a frame when the
    frames start in host memory.  Never part of `value`."""
    import numpy as np
    import torch
    stream = torch.cuda.current_stream()
    ms = []
    for k in ks:
        d = seq.depth[k]
        dh = torch.from_numpy(np.ascontiguousarray(d).view(np.int16) if d.dtype == np.uint16
                              else np.ascontiguousarray(d, np.float32)).pin_memory()
        ch = torch.from_numpy(np.ascontiguousarray(seq.rgb[k])).pin_memory()
        e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
        e0.record(stream)
        frames[k].depth.copy_(dh, non_blocking=True)
        frames[k].rgb.copy_(ch, non_blocking=True)
        e1.record(stream)
        torch.cuda.synchronize()
        ms.append(e0.elapsed_time(e1))
    return float(np.median(ms)), int(dh.numel() * dh.element_size() + ch.numel())


def mask_iou_measurement(seq, frames, dev, first=10):
    """Quality of the dynamic mask against the generator's labels (pixels
    whose first hit is a mover): the method runs over the whole sequence
    (untimed, FP32), and from frame `first` on each frame's final mask is
    compared pixel by pixel with the labels.  Reports the IoU of the frames
    with movers in view (mean, median) and over all their pixels."""
    import numpy as np
    import torch

    import paper_1905_02082_amd as rf
    mp = rf.MapParams(seq.voxel_size, seq.truncation, seq.depth_max, seq.num_buckets, WORKLOAD_BLOCKS[seq.name], 255,
                      seq.carve_stride, "fp32", seq.width * seq.height)
    tp = rf.TrackParams(seq.levels, seq.iters, 0.025, 64, 0.0)
    mk = rf.MaskParams(0.5, 0.007)
    s = rf.Session(mp, seq.poses[0], dev)
    inter, union = [], []
    for k in range(seq.n):
        rf.process_batch([s], [frames[k]], tp, mk, True)
        if k < first:
            continue
        gt = torch.from_numpy(seq.labels[k] > 0).to(dev)
        m = s.mask > 0
        inter.append(torch.logical_and(m, gt).sum())
        union.append(torch.logical_or(m, gt).sum())
    torch.cuda.synchronize()
    inter = np.array([int(x) for x in inter], np.int64)
    union = np.array([int(x) for x in union], np.int64)
    movers = union > 0
    iou = inter[movers] / union[movers]
    del s
    return {"frames": int(len(inter)), "frames_with_movers": int(movers.sum()),
            "mean_iou": round(float(iou.mean()), 4) if len(iou) else None,
            "median_iou": round(float(np.median(iou)), 4) if len(iou) else None,
            "pixel_iou": round(float(inter.sum() / max(union.sum(), 1)), 4),
            "note": "final mask of every frame from frame %d on against the pixels whose first hit is a mover" % first}


def run_workload(seq, frames, storage, W, K, B, dev, name, depth_max=None, free_blocks=False):
    """Fuses the sequence with the full method per frame; frames 0 .. n-K-W-1
    build the map untimed, the next W are warmup, the last K are timed.
    Returns the measurement dict (frames/s, latencies, stages, rooflines)."""
    import numpy as np
    import torch

    import paper_1905_02082_amd as rf
    n = seq.n
    offset = 25  # batched sessions: session i starts i * offset frames later in the same sequence
    n_run = n - offset * (B - 1)
    if K + W > n_run - 1:
        raise SystemExit("%s: --steps + --warmup must leave frame 0 before them (%d frames)" % (name, n_run))
    dmax = seq.depth_max if depth_max is None else depth_max
    mp = rf.MapParams(seq.voxel_size, seq.truncation, dmax, seq.num_buckets, WORKLOAD_BLOCKS[seq.name], 255,
                      seq.carve_stride, storage, seq.width * seq.height, free_blocks)
    tp = rf.TrackParams(seq.levels, seq.iters, 0.025, 64, 0.0)
    mk = rf.MaskParams(0.5, 0.007)
    sessions = [rf.Session(mp, seq.poses[offset * i], dev) for i in range(B)]
    stream = torch.cuda.current_stream()
    torch.cuda.synchronize()
    stage_names = ["track1", "mask", "track2", "allocate", "integrate"]

    def step(k, ev=None):
        rf.process_batch(sessions, [frames[offset * i + k] for i in range(B)], tp, mk, True, stream, ev)

    first_timed = n_run - K
    t0 = time.perf_counter()
    for k in range(first_timed):
        step(k)
    torch.cuda.synchronize()
    log("%s: fused %d frames untimed (%d map-building + %d warmup) in %.1f s" %
        (name, first_timed, first_timed - W, W, time.perf_counter() - t0))
    c0 = np.sum([s.map.cumulative_counts() for s in sessions], axis=0)
    events = [[torch.cuda.Event(enable_timing=True) for _ in range(6)] for _ in range(K)]
    torch.cuda.synchronize()
    t_start = time.perf_counter()
    for i in range(K):
        step(first_timed + i, events[i])
    torch.cuda.synchronize()
    t_end = time.perf_counter()
    c1 = np.sum([s.map.cumulative_counts() for s in sessions], axis=0)
    status = [s.map.status() for s in sessions]
    flags = int(np.bitwise_or.reduce([f for f, _ in status]))
    nblocks = int(status[0][1])
    wall = t_end - t_start
    per_stage = np.array([[events[i][j].elapsed_time(events[i][j + 1]) for j in range(5)] for i in range(K)])
    frame_ms = np.array([events[i][0].elapsed_time(events[i][5]) for i in range(K)])
    fps = B * K / wall
    T_final = sessions[0].pose.cpu().numpy()
    log("%s: timed %d frames, %.1f frames/s; measuring footprints" % (name, K, fps))

    # tracking roofline: algorithmic bytes per sweep from the host footprint of
    # sampled timed frames; duration = tracking stage time / launches (each
    # pass is levels x iterations track_kernel launches plus one reset and one
    # finalize launch of a few microseconds, counted in)
    keys = sessions[0].map.export()[0].cpu().numpy()
    sample = list(range(first_timed, n_run, max(1, K // 4)))[:4]
    t_fp = time.perf_counter()
    fp1, pix = track_footprint(seq, keys, sample, storage)
    log("%s: tracking footprint of %d frames in %.1f s" % (name, len(sample), time.perf_counter() - t_fp))
    sweeps = seq.levels * seq.iters
    track_alg = B * seq.iters * (2 * fp1.sum() + pix.sum()) / (2 * sweeps)
    track_ms = float((per_stage[:, 0] + per_stage[:, 2]).mean()) / (2 * sweeps)
    track_achieved = track_alg / (track_ms * 1e-3) / 1e9

    # integration roofline: algorithmic bytes per launch from the voxel-update counters
    band = c1[0] - c0[0]
    free = c1[1] - c0[1]
    blocks = c1[2] - c0[2]
    map_frames = c1[3] - c0[3]                               # maps x frames integrated
    rec = {"fp32": (8, 4), "fp16": (4, 4)}[storage]         # (sdf+weight, colour) bytes per voxel
    img = seq.width * seq.height * (2 + 1 + 3)              # depth u16 + mask u8 + RGB8
    alg_bytes = (band * 2 * (rec[0] + rec[1]) + free * 2 * rec[0] + blocks * (4 + 16) + map_frames * img)
    alg_per_launch = alg_bytes / K                          # one integration launch per step
    integ_ms = float(per_stage[:, 4].mean())
    achieved = alg_per_launch / (integ_ms * 1e-3) / 1e9
    key = profile_key(seq.name, n_run, storage, dmax, K) if B == 1 and not free_blocks else None
    traffic, l2_hit = traffic_from_profile("integrate_kernel", key) if key else (None, None)
    track_traffic, track_l2_hit = traffic_from_profile("track_kernel", key) if key else (None, None)

    E = np.linalg.inv(seq.poses[n_run - 1]) @ T_final       # session 0, against the generator's ground truth
    out = {
        "frames_per_s": round(fps, 3),
        "ms_per_step": round(1000.0 * wall / K, 4),
        "frames": n_run, "timed_frames": K, "warmup_frames": W, "map_building_frames": first_timed - W,
        "storage": storage, "depth_max_m": dmax, "sessions": B,
        "latency_ms": {"p50": round(float(np.percentile(frame_ms, 50)), 4),
                       "p99": round(float(np.percentile(frame_ms, 99)), 4)},
        "stages_ms": {nm: round(float(per_stage[:, j].mean()), 4) for j, nm in enumerate(stage_names)},
        "roofline": {"kernel": "track_kernel", "bound": "hbm", "achieved": round(track_achieved, 2),
                     "peak": HBM_PEAK_GBS, "unit": "GB/s", "frac": round(track_achieved / HBM_PEAK_GBS, 4),
                     "traffic": track_traffic, "l2_hit_rate": track_l2_hit,
                     "alg_bytes_per_launch": int(track_alg), "avg_launch_ms": round(track_ms, 5),
                     "launches_per_step": 2 * sweeps, "alg_bytes_per_level": [int(x) for x in fp1]},
        "roofline_integrate": {"kernel": "integrate_kernel", "bound": "hbm", "achieved": round(achieved, 2),
                               "peak": HBM_PEAK_GBS, "unit": "GB/s", "frac": round(achieved / HBM_PEAK_GBS, 4),
                               "traffic": traffic, "l2_hit_rate": l2_hit,
                               "alg_bytes_per_launch": int(alg_per_launch), "avg_launch_ms": round(integ_ms, 5),
                               "band_updates_per_launch": int(band / K), "free_updates_per_launch": int(free / K),
                               "blocks_per_launch": int(blocks / K)},
        "map": {"blocks": nblocks, "flags": flags, "final_position_error_m": round(float(np.linalg.norm(E[:3, 3])), 5)},
        "profile_key": key,
    }
    out["roofline_integrate"]["blocks_carved_whole_per_launch"] = int((c1[4] - c0[4]) / K)
    if free_blocks:
        keys_total = sessions[0].map.num_keys()
        out["map"].update({"blocks_with_voxels": nblocks, "free_blocks": keys_total - nblocks,
                           "voxel_bytes": int(nblocks) * 512 * ({"fp32": 12, "fp16": 8}[storage])})
    return out, sessions


def workload_text(seq, r):
    return ("%s %dx%d, %d frames (last %d timed), voxel %.3g m, truncation %.3g m, depth_max %.3g m, 8^3 blocks, "
            "2^%d buckets, %d levels x %d GN iterations, %s storage, full dynamic pipeline per frame%s"
            % (seq.name, seq.width, seq.height, r["frames"], r["timed_frames"], seq.voxel_size, seq.truncation,
               r["depth_max_m"], int(round(math.log2(seq.num_buckets))), seq.levels, seq.iters, r["storage"],
               "" if r["sessions"] == 1 else ", %d sessions per launch set" % r["sessions"]))


def serving_bench(args):
    """64 concurrent sessions over the dynamic-room generator, mixed
    resolutions, Poisson arrivals at 30 fps, FP16+u8 storage, HBM-budget
    admission; continuous batching (paper_1905_02082_amd.serving)."""
    import numpy as np
    import torch

    import paper_1905_02082_amd as rf
    import synth
    from paper_1905_02082_amd import serving

    dev = torch.device("cuda:0")
    rng = np.random.default_rng(1905020825)
    res = [(320, 240), (640, 480), (1280, 720)]
    probs = [0.3, 0.5, 0.2]
    n_sess = args.sessions
    t0 = time.perf_counter()
    seqs = {}
    for (w, h) in res:
        seqs[(w, h)] = [synth.dynamic_room(n_frames=args.serve_src_frames, width=w, height=h,
                                           seed=1905020825 + 17 * i + w) for i in range(2)]
    log("rendered serving sources in %.1f s" % (time.perf_counter() - t0))
    specs = []
    for sid in range(n_sess):
        w, h = res[rng.choice(3, p=probs)]
        seq = seqs[(w, h)][rng.integers(2)]
        n = int(rng.integers(300, 2001) * args.serve_scale)
        n = max(n, 2)
        start = 0.0 if args.unpaced else float(rng.uniform(0.0, 2.0))
        arr = (np.full(n, start) if args.unpaced else serving.poisson_arrivals(n, start, 30.0, rng))
        params = rf.MapParams(seq.voxel_size, seq.truncation, seq.depth_max, 1 << 20, 1 << 17, 255,
                              seq.carve_stride, args.storage if args.storage else "fp16", w * h)
        specs.append(serving.SessionSpec(sid, seq, serving.ping_pong(seq.n, n), arr, params))
    tp = rf.TrackParams(3, 10, 0.025, 64, 0.0)
    mp = rf.MaskParams(0.5, 0.007)
    budget = int(args.hbm_budget_gib * 2**30)
    r = serving.serve(specs, tp, mp, budget, max_batch=args.max_batch, depth=2, device=dev,
                      progress=lambda st, c, t: log("serving: step %d, %d/%d frames" % (st, c, t)),
                      batch_window_ms=args.batch_window_ms)
    summ = r.summary()
    out = {"metric": "aggregate frames/s of %d concurrent mixed-resolution sessions; p50/p99 frame latency"
                     % n_sess,
           "value": summ["frames_per_s"], "unit": "frames/s", "n_gpus": 1, "steps": summ["steps"],
           "warmup": 0, "ms_per_step": round(1000.0 * summ["wall_s"] / max(summ["steps"], 1), 3),
           "higher_is_better": True, "scaling": "weak", "vs_baseline": None, "dtype": "f32",
           "data": "synthetic",
           "config": {"workload": "serving: %d sessions, 30%% 320x240 / 50%% 640x480 / 20%% 1280x720, "
                                  "%s arrivals, lengths U[300,2000] x %.3g frames, %s storage, HBM budget %.1f GiB, "
                                  "max batch %d, batch window %.3g ms"
                                  % (n_sess, "unpaced" if args.unpaced else "Poisson 30 fps",
                                     args.serve_scale, args.storage or "fp16",
                                     args.hbm_budget_gib, args.max_batch, args.batch_window_ms)},
           "latency_ms": summ["latency_ms"], "serving": summ}
    print(json.dumps(out), flush=True)


def main():
    ap = argparse.ArgumentParser(description=__doc__, formatter_class=argparse.RawDescriptionHelpFormatter)
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=100, help="timed frames (the last frames of the sequence)")
    ap.add_argument("--warmup", type=int, default=10, help="untimed frames just before the timed ones")
    ap.add_argument("--workload", default="large_rooms",
                    choices=["large_rooms", "static_room", "dynamic_room", "serving"])
    ap.add_argument("--frames", type=int, default=None,
                    help="sequence length (default: 1000 large rooms, 300 static room, 400 dynamic room)")
    ap.add_argument("--storage", default=None, choices=["fp32", "fp16"],
                    help="voxel storage (default fp32; serving default fp16)")
    ap.add_argument("--depth-max", type=float, default=None, help="clipping plane (default: the workload's)")
    ap.add_argument("--extras", default="fp16,compact,depth_max_5m,static_room,dynamic_room",
                    help="comma list of extra measurements after the headline: fp16 (same sequence, FP16+u8 "
                         "storage), compact (same sequence, compact free space), depth_max_5m (same sequence, "
                         "clipping plane 5 m), static_room (300 frames), or none")
    ap.add_argument("--sessions", type=int, default=64, help="serving: concurrent sessions")
    ap.add_argument("--serve-scale", type=float, default=1.0, help="serving: scale of session lengths")
    ap.add_argument("--serve-src-frames", type=int, default=40, help="serving: rendered frames per source")
    ap.add_argument("--hbm-budget-gib", type=float, default=16.0, help="serving: admission budget")
    ap.add_argument("--max-batch", type=int, default=64, help="serving: sessions per step")
    ap.add_argument("--unpaced", action="store_true", help="serving: all frames available at once")
    ap.add_argument("--batch-window-ms", type=float, default=0.0,
                    help="serving: while a step runs, the next waits up to this long for more ready frames")
    ap.add_argument("--batch", type=int, default=1,
                    help="sessions processed together per step (1..8; the same scene at staggered frames)")
    ap.add_argument("--no-mesh", action="store_true", help="skip the mesh extraction measurement after the timed region")
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--cpu-budget", type=float, default=15.0, help="seconds of oracle time per cpu_baseline leg")
    args = ap.parse_args()

    world = int(os.environ.get("WORLD_SIZE", "1"))
    if args.gpus != 1 or world != 1:
        print("bench.py runs on one GPU only: the library has no multi-GPU path (sessions would shard "
              "across GPUs with no exchange); run with --gpus 1", file=sys.stderr)
        sys.exit(2)

    import numpy as np
    import torch

    import paper_1905_02082_amd as rf

    if not torch.cuda.is_available():
        raise SystemExit("bench.py needs a GPU")
    if args.workload == "serving":
        serving_bench(args)
        return
    storage = args.storage or "fp32"
    dev = torch.device("cuda:0")
    torch.cuda.set_device(dev)
    W, K, B = args.warmup, args.steps, args.batch
    if W < 0 or K < 1:
        raise SystemExit("--steps must be >= 1 and --warmup >= 0")
    if not 1 <= B <= 8:
        raise SystemExit("--batch must be in [1, 8]")
    extras = [] if args.extras in ("", "none") else args.extras.split(",")
    order = ("fp16", "compact", "depth_max_5m", "static_room", "dynamic_room")  # the rooms last: they replace the frames
    for e in extras:
        if e not in order:
            raise SystemExit("unknown extra %s" % e)
    extras = [e for e in order if e in extras]
    n = (args.frames or WORKLOAD_FRAMES[args.workload]) + 25 * (B - 1)
    t0 = time.perf_counter()
    seq = make_sequence(args.workload, n)
    log("rendered %d frames %dx%d in %.1f s" % (seq.n, seq.width, seq.height, time.perf_counter() - t0))
    frames = upload_frames(seq, dev)
    torch.cuda.synchronize()

    head, sessions = run_workload(seq, frames, storage, W, K, B, dev, "headline", args.depth_max)
    out = {
        "metric": METRIC,
        "value": head["frames_per_s"],
        "unit": "frames/s",
        "n_gpus": 1,
        "steps": K,
        "warmup": W,
        "ms_per_step": head["ms_per_step"],     # one step = one frame of every session
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "f32",
        "data": "synthetic",
        "config": {"workload": workload_text(seq, head), "frames": head["frames"],
                   "map_building_frames": head["map_building_frames"], "width": seq.width,
                   "height": seq.height, "storage": storage, "depth_max_m": head["depth_max_m"], "sessions": B},
    }
    for k in ("latency_ms", "stages_ms", "roofline", "roofline_integrate", "map"):
        out[k] = head[k]
    out["profile_key"] = head["profile_key"]
    h2d_ms, h2d_bytes = h2d_measurement(seq, frames, range(seq.n - min(K, 20), seq.n), dev)
    out["h2d"] = {"ms_per_frame": round(h2d_ms, 4), "bytes_per_frame": h2d_bytes,
                  "frames_per_s_incl_h2d": round(B * 1000.0 / (head["ms_per_step"] + B * h2d_ms), 3),
                  "note": "pinned host -> device upload of a frame on the kernels' stream, timed apart and "
                          "added serially (no copy/compute overlap); not part of value"}
    if not args.no_mesh and B == 1:
        out["mesh"] = mesh_measurement(sessions[0].map, seq, storage)
        out["virtual_depth"] = virtual_depth_measurement(sessions[0].map, seq, frames[seq.n - 1], sessions[0].pose)
    pose_head = sessions[0].pose.cpu().numpy()
    del sessions
    torch.cuda.empty_cache()
    if B == 1:
        for e in extras:
            if e == "fp16" and storage != "fp16":
                r, ss = run_workload(seq, frames, "fp16", W, K, 1, dev, "fp16", args.depth_max)
                Tf = ss[0].pose.cpu().numpy()
                dT = np.linalg.inv(pose_head) @ Tf
                r["final_pose_vs_fp32"] = {"dt_m": round(float(np.linalg.norm(dT[:3, 3])), 7),
                                           "dr_rad": round(float(np.arccos(np.clip((np.trace(dT[:3, :3]) - 1) / 2,
                                                                                   -1, 1))), 8)}
                out["fp16"] = r
            elif e == "compact":
                r, ss = run_workload(seq, frames, storage, W, K, 1, dev, "compact", args.depth_max, free_blocks=True)
                Tc = ss[0].pose.cpu().numpy()
                dT = np.linalg.inv(pose_head) @ Tc
                r["final_pose_vs_per_voxel"] = {"dt_m": round(float(np.linalg.norm(dT[:3, 3])), 7),
                                                "dr_rad": round(float(np.arccos(np.clip((np.trace(dT[:3, :3]) - 1) / 2,
                                                                                        -1, 1))), 8)}
                out["compact"] = r
            elif e == "depth_max_5m" and (args.depth_max or seq.depth_max) != 5.0:
                r, ss = run_workload(seq, frames, storage, W, K, 1, dev, "depth_max_5m", 5.0)
                out["depth_max_5m"] = r
            elif e in ("static_room", "dynamic_room") and args.workload != e:
                if frames is not None:
                    del frames
                    frames = None
                torch.cuda.empty_cache()
                sq = make_sequence(e, WORKLOAD_FRAMES[e])
                fr2 = upload_frames(sq, dev)
                r, ss = run_workload(sq, fr2, "fp32", W, K, 1, dev, e)
                r["workload"] = workload_text(sq, r)
                if e == "dynamic_room":
                    del ss
                    ss = []
                    torch.cuda.empty_cache()
                    r["mask_iou"] = mask_iou_measurement(sq, fr2, dev)
                    log("dynamic_room: mask IoU %s" % r["mask_iou"]["mean_iou"])
                out[e] = r
                del fr2
            else:
                continue
            del ss
            torch.cuda.empty_cache()
    if not args.no_cpu_baseline and B == 1:
        ncpu, model = host_cpu()
        # all the host cores this process may use: the affinity set, capped by
        # OMP_NUM_THREADS where the host assigns a share of its cores
        share = int(os.environ.get("OMP_NUM_THREADS") or ncpu)
        v1, sample1, _, st1 = cpu_baseline(seq, args.cpu_budget, threads=1)
        vn, samplen, used, stn = cpu_baseline(seq, args.cpu_budget, threads=max(2, min(ncpu, share)))
        out["cpu_baseline"] = {"value": round(vn, 5), "unit": "frames/s", "cores": used, "kind": "oracle",
                               "sample": samplen, "cpu_model": model, "nproc": ncpu, "stages_ms": stn,
                               "single_thread": {"value": round(v1, 5), "cores": 1, "sample": sample1,
                                                 "stages_ms": st1}}
    print(json.dumps(out), flush=True)
    # release every map (and its arena) and drain the stream before the
    # interpreter shuts down, so no destructor runs against a torn-down runtime
    frames = None
    import gc
    gc.collect()
    torch.cuda.synchronize()


if __name__ == "__main__":
    main()
