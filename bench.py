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

Prints ONE JSON line.  The dominant kernel's duration is measured with HIP
events on the stream it runs on; its algorithmic bytes come from device
counters of voxel updates (see the design doc for the per-unit figures).
"""
from __future__ import annotations

import argparse
import hashlib
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


def kernel_source_hash():
    h = hashlib.sha256()
    for f in ("rf_fusion.hip", "rf_device.h"):
        with open(os.path.join(ROOT, "paper_1905_02082_amd", "csrc", f), "rb") as fh:
            h.update(fh.read())
    return h.hexdigest()[:16]


def traffic_from_profile(workload, storage):
    """HBM bytes per integration launch from the committed rocprofv3 PMC
    summary, if it was taken on the current kernel source (else None)."""
    path = os.path.join(ROOT, "profiles", "integrate_%s_%s_pmc.json" % (workload, storage))
    if not os.path.exists(path):
        return None
    with open(path) as fh:
        d = json.load(fh)
    if d.get("kernel_source_hash") != kernel_source_hash():
        return None
    return d.get("hbm_bytes_per_launch")


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
    W, K = args.warmup, args.steps
    n = W + K
    if W < 1:
        raise SystemExit("--warmup must be >= 1 (frame 0 initialises the map)")
    t0 = time.perf_counter()
    seq = make_sequence(args.workload, n)
    log("rendered %d frames %dx%d in %.1f s" % (n, seq.width, seq.height, time.perf_counter() - t0))

    max_blocks = {"static_room": 1 << 18, "dynamic_room": 1 << 18, "large_rooms": 1 << 22}[args.workload]
    mp = rf.MapParams(seq.voxel_size, seq.truncation, seq.depth_max, seq.num_buckets, max_blocks, 255,
                      seq.carve_stride, args.storage, seq.width * seq.height)
    tp = rf.TrackParams(seq.levels, seq.iters, 0.025, 64, 0.0)
    mk = rf.MaskParams(0.5, 0.007)
    frames = [rf.Frame.from_numpy(seq.depth[k], seq.rgb[k], *seq.intrinsics, depth_scale=seq.depth_scale,
                                  device=dev) for k in range(n)]
    m = rf.Map(mp, dev)
    pose = torch.as_tensor(seq.poses[0]).to(dev).contiguous()
    mask = torch.zeros((seq.height, seq.width), dtype=torch.uint8, device=dev)
    stats = torch.zeros(16, dtype=torch.float64, device=dev)
    stream = torch.cuda.current_stream()
    torch.cuda.synchronize()

    stage_names = ["track1", "mask", "track2", "allocate", "integrate"]

    def step(fr, ev=None):
        if ev is not None:
            ev[0].record(stream)
        m.track(fr, pose, tp, None, stats)
        if ev is not None:
            ev[1].record(stream)
        m.dynamic_mask(fr, pose, mk, out=mask)
        if ev is not None:
            ev[2].record(stream)
        m.track(fr, pose, tp, mask, stats)
        if ev is not None:
            ev[3].record(stream)
        m.allocate(fr, pose, mask)
        if ev is not None:
            ev[4].record(stream)
        m.integrate(fr, pose, mask)
        if ev is not None:
            ev[5].record(stream)

    # frame 0 initialises the map at its given pose; frames 1..W-1 warm up
    m.allocate(frames[0], pose)
    m.integrate(frames[0], pose)
    for k in range(1, W):
        step(frames[k])
    torch.cuda.synchronize()
    c0 = m.cumulative_counts()

    events = [[torch.cuda.Event(enable_timing=True) for _ in range(6)] for _ in range(K)]
    torch.cuda.synchronize()
    t_start = time.perf_counter()
    for i in range(K):
        step(frames[W + i], events[i])
    torch.cuda.synchronize()
    t_end = time.perf_counter()
    c1 = m.cumulative_counts()
    flags, nblocks = m.status()

    wall = t_end - t_start
    per_stage = np.array([[events[i][j].elapsed_time(events[i][j + 1]) for j in range(5)] for i in range(K)])
    frame_ms = np.array([events[i][0].elapsed_time(events[i][5]) for i in range(K)])
    fps = K / wall
    T_final = pose.cpu().numpy()

    # integration roofline: algorithmic bytes per launch from the voxel-update counters
    band = c1[0] - c0[0]
    free = c1[1] - c0[1]
    blocks = c1[2] - c0[2]
    launches = c1[3] - c0[3]
    rec = {"fp32": (8, 4), "fp16": (4, 4)}[args.storage]   # (sdf+weight, colour) bytes per voxel
    img = seq.width * seq.height * (2 + 1 + 3)              # depth u16 + mask u8 + RGB8
    alg_bytes = (band * 2 * (rec[0] + rec[1]) + free * 2 * rec[0] + blocks * (4 + 16) + launches * img)
    alg_per_launch = alg_bytes / max(launches, 1)
    integ_ms = float(per_stage[:, 4].mean())
    achieved = alg_per_launch / (integ_ms * 1e-3) / 1e9
    traffic = traffic_from_profile(args.workload, args.storage)

    # trajectory error against the generator's ground truth (context only)
    E = np.linalg.inv(seq.poses[n - 1]) @ T_final
    ate_last = float(np.linalg.norm(E[:3, 3]))

    out = {
        "metric": METRIC,
        "value": round(fps, 3),
        "unit": "frames/s",
        "n_gpus": 1,
        "steps": K,
        "warmup": W,
        "ms_per_step": round(1000.0 * wall / K, 4),
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "f32",
        "data": "synthetic",
        "config": {"workload": "%s %dx%d, %d frames, voxel %.3g m, truncation %.3g m, 8^3 blocks, 2^%d buckets, "
                               "%d levels x %d GN iterations, %s storage, full dynamic pipeline per frame"
                               % (args.workload, seq.width, seq.height, n, seq.voxel_size, seq.truncation,
                                  int(np.log2(seq.num_buckets)), seq.levels, seq.iters, args.storage),
                   "frames": n, "width": seq.width, "height": seq.height, "storage": args.storage},
        "latency_ms": {"p50": round(float(np.percentile(frame_ms, 50)), 4),
                       "p99": round(float(np.percentile(frame_ms, 99)), 4)},
        "stages_ms": {nm: round(float(per_stage[:, j].mean()), 4) for j, nm in enumerate(stage_names)},
        "roofline": {"kernel": "integrate_kernel", "bound": "hbm", "achieved": round(achieved, 2),
                     "peak": HBM_PEAK_GBS, "unit": "GB/s", "frac": round(achieved / HBM_PEAK_GBS, 4),
                     "traffic": traffic,
                     "alg_bytes_per_launch": int(alg_per_launch),
                     "avg_launch_ms": round(integ_ms, 5),
                     "band_updates_per_launch": int(band / max(launches, 1)),
                     "free_updates_per_launch": int(free / max(launches, 1)),
                     "blocks_per_launch": int(blocks / max(launches, 1))},
        "map": {"blocks": nblocks, "flags": flags, "final_position_error_m": round(ate_last, 5)},
    }
    if not args.no_cpu_baseline:
        v, sample = cpu_baseline(seq, args.cpu_budget)
        out["cpu_baseline"] = {"value": round(v, 5), "unit": "frames/s", "cores": 1, "kind": "oracle",
                               "sample": sample}
    print(json.dumps(out), flush=True)


if __name__ == "__main__":
    main()
