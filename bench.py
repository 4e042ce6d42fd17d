#!/usr/bin/env python3
"""Throughput of the ReFusion per-frame hot path on one MI355X.

Workload (default): the 640x480 static indoor room -- 300 frames of uint16
millimetre depth (0.3-5 m) + RGB8, ray-cast from a seeded 4x4x3 m room with
20 textured boxes/spheres, Kinect-like axial noise and 2% dropout; voxel 1 cm,
truncation 3 cm, 8^3 blocks, 2^20 buckets, 3-level pyramid x 10 Gauss-Newton
iterations, Table I weights (w_c 0.025, theta 0.007, gamma 0.5).

One step = one frame through the whole method: registration without mask,
residual mask with flood fill, registration with the mask, block allocation
with carve rays, integration with free-space carving.  Frame 0 initialises
the map; the first W frames are warmup; K frames are timed.  All inputs are
on the device before the timed region.

Prints ONE JSON line.  Kernel durations are measured with HIP events on the
stream the kernels run on.  "roofline" is the dominant kernel (the tracking
sweep): its algorithmic bytes come from the host footprint of sampled frames
(distinct voxel records and buckets a sweep reads, plus image bytes).
"roofline_integrate" is the integration kernel, whose algorithmic bytes come
from device counters of voxel updates.
"""
from __future__ import annotations

import argparse
import ctypes
import json
import os
import sys
import time

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

METRIC = "640x480 frames/sec tracked+fused (HBM GB/s % peak); p50/p99 frame latency"
HBM_PEAK_GBS = 8000.0


def log(*a):
    print(*a, file=sys.stderr, flush=True)


def traffic_from_profile(kernel, workload, storage):
    """(HBM bytes per launch, L2 hit rate) of `kernel` from the committed
    rocprofv3 PMC summary (FETCH_SIZE + WRITE_SIZE, calibrated; TCC_HIT /
    (TCC_HIT + TCC_MISS)), if it was taken on the current kernel source
    (else None, None)."""
    path = os.path.join(ROOT, "profiles", "%s_%s_%s_pmc.json" % (kernel.replace("_kernel", ""), workload, storage))
    if not os.path.exists(path):
        return None, None
    with open(path) as fh:
        d = json.load(fh)
    from paper_1905_02082_amd.profiling import kernel_source_hash
    if d.get("kernel_source_hash") != kernel_source_hash(kernel):
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
    if seq.prims is not None and n:
        V = np.unique(tris.reshape(-1, 3).cpu().numpy().astype(np.float64), axis=0)
        d = scene_distance(seq.prims, V)
        out["accuracy"] = {"vertices": int(len(V)), "mean_mm": round(1e3 * float(d.mean()), 3),
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


def make_sequence(workload, n):
    import synth
    if workload == "static_room":
        return synth.static_room(n_frames=n)
    if workload == "dynamic_room":
        return synth.dynamic_room(n_frames=n)
    if workload == "large_rooms":
        return synth.large_rooms(n_frames=n)
    raise SystemExit("unknown workload %s" % workload)


def cpu_baseline(seq, budget_s=30.0):
    """The oracle as it stands (single thread): frame 0 fusion, then full
    frames until the time budget is spent; returns frames/s of the full
    frames and the sample description."""
    import oracle as O
    a = O.OracleMap(seq.voxel_size, seq.truncation, seq.depth_max, 255, seq.carve_stride, real_bits=64)
    b = O.OracleMap(seq.voxel_size, seq.truncation, seq.depth_max, 255, seq.carve_stride, real_bits=32)
    T = seq.poses[0]
    fr = O.Frame(seq.depth[0], seq.rgb[0], *seq.intrinsics, depth_scale=seq.depth_scale)
    T, _ = O.process_frame(a, fr, T, 0, seq.levels, seq.iters, mask_map=b)
    done, spent = 0, 0.0
    k = 1
    while k < seq.n and (done == 0 or spent < budget_s):
        fr = O.Frame(seq.depth[k], seq.rgb[k], *seq.intrinsics, depth_scale=seq.depth_scale)
        t0 = time.perf_counter()
        T, _ = O.process_frame(a, fr, T, k, seq.levels, seq.iters, mask_map=b)
        spent += time.perf_counter() - t0
        done += 1
        k += 1
        log("cpu oracle frame %d: %.2f s" % (k - 1, spent / done))
    return done / spent, "frames 1-%d of the same sequence (full method per frame after frame-0 fusion), " \
                          "FP64 oracle + FP32 mask mirror, single thread" % done


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
                      progress=lambda st, c, t: log("serving: step %d, %d/%d frames" % (st, c, t)))
    summ = r.summary()
    out = {"metric": "aggregate frames/s of %d concurrent mixed-resolution sessions; p50/p99 frame latency"
                     % n_sess,
           "value": summ["frames_per_s"], "unit": "frames/s", "n_gpus": 1, "steps": summ["steps"],
           "warmup": 0, "ms_per_step": round(1000.0 * summ["wall_s"] / max(summ["steps"], 1), 3),
           "higher_is_better": True, "scaling": "weak", "vs_baseline": None, "dtype": "f32",
           "data": "synthetic",
           "config": {"workload": "serving: %d sessions, 30%% 320x240 / 50%% 640x480 / 20%% 1280x720, "
                                  "%s arrivals, lengths U[300,2000] x %.3g frames, %s storage, HBM budget %.1f GiB, "
                                  "max batch %d" % (n_sess, "unpaced" if args.unpaced else "Poisson 30 fps",
                                                    args.serve_scale, args.storage or "fp16",
                                                    args.hbm_budget_gib, args.max_batch)},
           "latency_ms": summ["latency_ms"], "serving": summ}
    print(json.dumps(out), flush=True)


def main():
    ap = argparse.ArgumentParser(description=__doc__, formatter_class=argparse.RawDescriptionHelpFormatter)
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=280, help="timed frames")
    ap.add_argument("--warmup", type=int, default=20, help="untimed frames before the timed region")
    ap.add_argument("--workload", default="static_room",
                    choices=["static_room", "dynamic_room", "large_rooms", "serving"])
    ap.add_argument("--storage", default=None, choices=["fp32", "fp16"],
                    help="voxel storage (default fp32; serving default fp16)")
    ap.add_argument("--sessions", type=int, default=64, help="serving: concurrent sessions")
    ap.add_argument("--serve-scale", type=float, default=1.0, help="serving: scale of session lengths")
    ap.add_argument("--serve-src-frames", type=int, default=40, help="serving: rendered frames per source")
    ap.add_argument("--hbm-budget-gib", type=float, default=16.0, help="serving: admission budget")
    ap.add_argument("--max-batch", type=int, default=64, help="serving: sessions per step")
    ap.add_argument("--unpaced", action="store_true", help="serving: all frames available at once")
    ap.add_argument("--batch", type=int, default=1,
                    help="sessions processed together per step (1..8; the same scene at staggered frames)")
    ap.add_argument("--no-mesh", action="store_true", help="skip the mesh extraction measurement after the timed region")
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--cpu-budget", type=float, default=20.0, help="seconds of oracle time for cpu_baseline")
    args = ap.parse_args()

    world = int(os.environ.get("WORLD_SIZE", "1"))
    if args.gpus != 1 or world != 1:
        print("bench.py runs on one GPU only: this build has no multi-GPU path (sessions would shard "
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
    if args.storage is None:
        args.storage = "fp32"
    dev = torch.device("cuda:0")
    torch.cuda.set_device(dev)
    W, K, B = args.warmup, args.steps, args.batch
    n = W + K
    if W < 1:
        raise SystemExit("--warmup must be >= 1 (frame 0 initialises the map)")
    if not 1 <= B <= 8:
        raise SystemExit("--batch must be in [1, 8]")
    offset = 25  # session i starts at frame i * offset of the same rendered sequence
    t0 = time.perf_counter()
    seq = make_sequence(args.workload, n + offset * (B - 1))
    log("rendered %d frames %dx%d in %.1f s" % (seq.n, seq.width, seq.height, time.perf_counter() - t0))

    max_blocks = {"static_room": 1 << 18, "dynamic_room": 1 << 18, "large_rooms": 3 << 20}[args.workload]
    mp = rf.MapParams(seq.voxel_size, seq.truncation, seq.depth_max, seq.num_buckets, max_blocks, 255,
                      seq.carve_stride, args.storage, seq.width * seq.height)
    tp = rf.TrackParams(seq.levels, seq.iters, 0.025, 64, 0.0)
    mk = rf.MaskParams(0.5, 0.007)
    frames = [rf.Frame.from_numpy(seq.depth[k], seq.rgb[k], *seq.intrinsics, depth_scale=seq.depth_scale,
                                  device=dev) for k in range(seq.n)]
    sessions = [rf.Session(mp, seq.poses[offset * i], dev) for i in range(B)]
    stream = torch.cuda.current_stream()
    torch.cuda.synchronize()

    stage_names = ["track1", "mask", "track2", "allocate", "integrate"]

    def step(k, ev=None):
        rf.process_batch(sessions, [frames[offset * i + k] for i in range(B)], tp, mk, True, stream, ev)

    # frame 0 initialises each map at its given pose; frames 1..W-1 warm up
    for k in range(W):
        step(k)
    torch.cuda.synchronize()
    c0 = np.sum([s.map.cumulative_counts() for s in sessions], axis=0)

    events = [[torch.cuda.Event(enable_timing=True) for _ in range(6)] for _ in range(K)]
    torch.cuda.synchronize()
    t_start = time.perf_counter()
    for i in range(K):
        step(W + i, events[i])
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

    # tracking roofline (the dominant kernel): algorithmic bytes per sweep from
    # the host footprint of sampled frames; duration = tracking stage time /
    # sweeps (each pass is levels x iterations track_kernel launches plus one
    # reset and one finalize launch of a few microseconds, counted in)
    keys = sessions[0].map.export()[0].cpu().numpy()
    sample = list(range(W, n, max(1, K // 4)))[:4]
    fp1, pix = track_footprint(seq, keys, sample, args.storage)
    sweeps = seq.levels * seq.iters
    track_alg = B * seq.iters * (2 * fp1.sum() + pix.sum()) / (2 * sweeps)
    track_ms = float((per_stage[:, 0] + per_stage[:, 2]).mean()) / (2 * sweeps)
    track_achieved = track_alg / (track_ms * 1e-3) / 1e9

    # integration roofline: algorithmic bytes per launch from the voxel-update counters
    band = c1[0] - c0[0]
    free = c1[1] - c0[1]
    blocks = c1[2] - c0[2]
    map_frames = c1[3] - c0[3]                               # maps x frames integrated
    rec = {"fp32": (8, 4), "fp16": (4, 4)}[args.storage]   # (sdf+weight, colour) bytes per voxel
    img = seq.width * seq.height * (2 + 1 + 3)              # depth u16 + mask u8 + RGB8
    alg_bytes = (band * 2 * (rec[0] + rec[1]) + free * 2 * rec[0] + blocks * (4 + 16) + map_frames * img)
    launches = K                                            # one integration launch per step
    alg_per_launch = alg_bytes / max(launches, 1)
    integ_ms = float(per_stage[:, 4].mean())
    achieved = alg_per_launch / (integ_ms * 1e-3) / 1e9
    traffic, l2_hit = traffic_from_profile("integrate_kernel", args.workload, args.storage) if B == 1 else (None, None)
    track_traffic, track_l2_hit = (traffic_from_profile("track_kernel", args.workload, args.storage) if B == 1
                                   else (None, None))

    # trajectory error against the generator's ground truth (context only)
    E = np.linalg.inv(seq.poses[n - 1]) @ T_final       # session 0
    ate_last = float(np.linalg.norm(E[:3, 3]))

    out = {
        "metric": METRIC,
        "value": round(fps, 3),
        "unit": "frames/s",
        "n_gpus": 1,
        "steps": K,
        "warmup": W,
        "ms_per_step": round(1000.0 * wall / K, 4),     # one step = one frame of every session
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "f32",
        "data": "synthetic",
        "config": {"workload": "%s %dx%d, %d frames, voxel %.3g m, truncation %.3g m, 8^3 blocks, 2^%d buckets, "
                               "%d levels x %d GN iterations, %s storage, full dynamic pipeline per frame%s"
                               % (args.workload, seq.width, seq.height, n, seq.voxel_size, seq.truncation,
                                  int(np.log2(seq.num_buckets)), seq.levels, seq.iters, args.storage,
                                  "" if B == 1 else ", %d sessions per launch set" % B),
                   "frames": n, "width": seq.width, "height": seq.height, "storage": args.storage,
                   "sessions": B},
        "latency_ms": {"p50": round(float(np.percentile(frame_ms, 50)), 4),
                       "p99": round(float(np.percentile(frame_ms, 99)), 4)},
        "stages_ms": {nm: round(float(per_stage[:, j].mean()), 4) for j, nm in enumerate(stage_names)},
        "roofline": {"kernel": "track_kernel", "bound": "hbm", "achieved": round(track_achieved, 2),
                     "peak": HBM_PEAK_GBS, "unit": "GB/s", "frac": round(track_achieved / HBM_PEAK_GBS, 4),
                     "traffic": track_traffic,
                     "l2_hit_rate": track_l2_hit,
                     "alg_bytes_per_launch": int(track_alg),
                     "avg_launch_ms": round(track_ms, 5),
                     "launches_per_step": 2 * sweeps,
                     "alg_bytes_per_level": [int(x) for x in fp1]},
        "roofline_integrate": {"kernel": "integrate_kernel", "bound": "hbm", "achieved": round(achieved, 2),
                     "peak": HBM_PEAK_GBS, "unit": "GB/s", "frac": round(achieved / HBM_PEAK_GBS, 4),
                     "traffic": traffic,
                     "l2_hit_rate": l2_hit,
                     "alg_bytes_per_launch": int(alg_per_launch),
                     "avg_launch_ms": round(integ_ms, 5),
                     "band_updates_per_launch": int(band / max(launches, 1)),
                     "free_updates_per_launch": int(free / max(launches, 1)),
                     "blocks_per_launch": int(blocks / max(launches, 1))},
        "map": {"blocks": nblocks, "flags": flags, "final_position_error_m": round(ate_last, 5)},
    }
    if not args.no_mesh and B == 1:
        out["mesh"] = mesh_measurement(sessions[0].map, seq, args.storage)
        out["virtual_depth"] = virtual_depth_measurement(sessions[0].map, seq, frames[n - 1], sessions[0].pose)
    if not args.no_cpu_baseline and B == 1:
        v, sample = cpu_baseline(seq, args.cpu_budget)
        out["cpu_baseline"] = {"value": round(v, 5), "unit": "frames/s", "cores": 1, "kind": "oracle",
                               "sample": sample}
    print(json.dumps(out), flush=True)


if __name__ == "__main__":
    main()
