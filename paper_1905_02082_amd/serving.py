"""Continuous batching of many reconstruction sessions on one GPU.

Each session owns a device-resident map, pose and mask (paper_1905_02082_amd.
Session).  Frames arrive over time (per session: its own start time and
arrival process).  The server loop:

  * admits waiting sessions while the HBM budget allows (a session's arena
    size is known exactly from hashmap_bytes) and frees a session's map when
    its last frame completes, so later sessions take its place; a session
    that had to wait starts streaming when it is admitted (its frames'
    arrival times move by the wait, which is reported separately);
  * forms each step from every admitted session that has an arrived frame
    (oldest frames first, up to max_batch) and runs the step as one launch set
    per stage over all of them (process_batch), uploading the frames from
    pinned host memory on the same stream;
  * keeps up to `depth` steps in flight, so the host prepares step n+1 while
    the GPU runs step n; a session's consecutive frames stay ordered on the
    stream;
  * records a completion event per step and measures each frame's latency
    from its arrival time to that event.

Results do not depend on how frames were batched (every job's arithmetic is
independent of its neighbours), which tests/test_gpu_batch.py checks.
"""
from __future__ import annotations

import dataclasses
import heapq
import math
import time
from typing import List

import numpy as np
import torch

from . import Frame, MapParams, MaskParams, Session, TrackParams, hashmap_bytes, process_batch


@dataclasses.dataclass
class SessionSpec:
    """One client: frames `order[k]` of a host sequence, arriving at
    `arrivals[k]` seconds after the server starts."""
    sid: int
    seq: object                  # synth.Sequence (host arrays)
    order: np.ndarray            # frame index into seq for each streamed frame
    arrivals: np.ndarray         # seconds, non-decreasing
    params: MapParams


def poisson_arrivals(n, start, fps, rng):
    """n arrival times of a Poisson process of rate fps starting at start."""
    gaps = rng.exponential(1.0 / fps, size=n)
    gaps[0] = 0.0
    return start + np.cumsum(gaps)


def ping_pong(n_src, n):
    """Frame order that plays a sequence forward and backward (continuous motion)."""
    period = max(2 * n_src - 2, 1)
    k = np.arange(n) % period
    return np.where(k < n_src, k, period - k)


@dataclasses.dataclass
class ServeResult:
    frames: int
    wall_s: float
    latencies_ms: np.ndarray
    admission_waits_ms: np.ndarray   # per session: admission time - first scheduled arrival
    steps: int
    mean_batch: float
    peak_sessions: int
    peak_bytes: int
    admitted_late: int           # sessions that waited for memory
    per_resolution: dict

    @property
    def fps(self):
        return self.frames / self.wall_s

    def summary(self):
        lat, adm = self.latencies_ms, self.admission_waits_ms
        return {"frames": self.frames, "wall_s": round(self.wall_s, 3), "frames_per_s": round(self.fps, 2),
                "latency_ms": {"p50": round(float(np.percentile(lat, 50)), 3),
                               "p99": round(float(np.percentile(lat, 99)), 3),
                               "max": round(float(lat.max()), 3)},
                "admission_wait_ms": {"p50": round(float(np.percentile(adm, 50)), 3),
                                      "p99": round(float(np.percentile(adm, 99)), 3),
                                      "max": round(float(adm.max()), 3)},
                "steps": self.steps, "mean_batch": round(self.mean_batch, 2),
                "peak_sessions": self.peak_sessions, "peak_hbm_gib": round(self.peak_bytes / 2**30, 3),
                "sessions_that_waited_for_memory": self.admitted_late,
                "per_resolution": self.per_resolution}


class _Live:
    def __init__(self, spec: SessionSpec, session: Session, nbytes: int, shift: float):
        self.spec = spec
        self.session = session
        self.nbytes = nbytes
        self.shift = shift      # admission wait: the session's arrivals move by it
        self.next = 0           # next frame to submit
        self.done = 0           # frames completed

    def arrival(self, k):
        return float(self.spec.arrivals[k]) + self.shift


def serve(specs: List[SessionSpec], tp: TrackParams, mp: MaskParams, hbm_budget: int, max_batch=64, depth=2,
          dynamic=True, device="cuda", pinned_frames=None, progress=None, on_finish=None,
          batch_window_ms=0.0) -> ServeResult:
    """Runs all sessions to completion; returns latency and throughput.

    batch_window_ms: while a step is already running on the GPU, a further
    step waits until max_batch frames are ready or its oldest frame has
    waited this long (0: it is issued as soon as one frame is ready).  An
    idle GPU always takes the ready frames at once.

    on_finish(spec, session), if given, is called once per session after its
    last frame has completed and before its map is released (the session's
    pose and map are final then).  A session whose map alone exceeds
    hbm_budget could never be admitted: it raises ValueError up front."""
    for spec in specs:
        nb = hashmap_bytes(spec.params)
        if nb > hbm_budget:
            raise ValueError("session %r needs %d bytes of map arena, more than the whole HBM budget (%d)"
                             % (spec.sid, nb, hbm_budget))
        if len(spec.arrivals) == 0 or len(spec.order) != len(spec.arrivals):
            raise ValueError("session %r: order and arrivals must be non-empty and of equal length" % spec.sid)
    dev = torch.device(device)
    stream = torch.cuda.current_stream(dev)
    if pinned_frames is None:
        pinned_frames = {}

    def host_frame(seq, k):
        key = (id(seq), int(k))
        if key not in pinned_frames:
            d = seq.depth[k]
            dt = torch.from_numpy(np.ascontiguousarray(d).view(np.int16) if d.dtype == np.uint16
                                  else np.ascontiguousarray(d, np.float32)).pin_memory()
            ct = torch.from_numpy(np.ascontiguousarray(seq.rgb[k])).pin_memory()
            pinned_frames[key] = (dt, ct)
        return pinned_frames[key]

    waiting = sorted(specs, key=lambda s: s.arrivals[0])
    live: List[_Live] = []
    used = 0
    peak_bytes = 0
    peak_sessions = 0
    late = 0
    inflight = []            # (event, [(live, arrival_s, pixels)], frame tensors)
    latencies = []
    waits = []
    per_res = {}
    n_steps = 0
    batch_sizes = []
    total = sum(len(s.arrivals) for s in specs)
    completed = 0

    t_origin = torch.cuda.Event(enable_timing=True)
    t_origin.record(stream)
    torch.cuda.synchronize(dev)
    t0 = time.perf_counter()

    def now():
        return time.perf_counter() - t0

    def retire(block):
        nonlocal completed
        while inflight and (block or inflight[0][0].query()):
            ev, members, _ = inflight.pop(0)
            ev.synchronize()
            t_done = t_origin.elapsed_time(ev) / 1000.0
            for lv, arr, key in members:
                ms = (t_done - arr) * 1000.0
                latencies.append(ms)
                per_res.setdefault(key, []).append(ms)
                lv.done += 1
                completed += 1
            block = False

    while completed < total:
        t = now()
        # admission: in arrival order, while the budget allows
        while waiting and waiting[0].arrivals[0] <= t:
            spec = waiting[0]
            nb = hashmap_bytes(spec.params)
            if used + nb > hbm_budget:
                break
            waiting.pop(0)
            shift = max(0.0, t - float(spec.arrivals[0]))
            if shift > 1.0 / 30.0:
                late += 1
            waits.append(shift * 1000.0)
            s = Session(spec.params, spec.seq.poses[spec.order[0]], dev)
            live.append(_Live(spec, s, nb, shift))
            used += nb
            peak_bytes = max(peak_bytes, used)
        peak_sessions = max(peak_sessions, len(live))
        # step: admitted sessions with an arrived, unsubmitted frame, oldest first
        ready = [lv for lv in live if lv.next < len(lv.spec.arrivals) and lv.arrival(lv.next) <= t]
        ready.sort(key=lambda lv: lv.arrival(lv.next))
        ready = ready[:max_batch]
        hold = (batch_window_ms > 0.0 and inflight and len(ready) < max_batch and ready and
                (t - ready[0].arrival(ready[0].next)) * 1000.0 < batch_window_ms)
        if ready and len(inflight) < depth and not hold:
            frames, members, keep = [], [], []
            for lv in ready:
                seq = lv.spec.seq
                k = int(lv.spec.order[lv.next])
                dh, ch = host_frame(seq, k)
                dd = dh.to(dev, non_blocking=True)
                cd = ch.to(dev, non_blocking=True)
                keep += [dd, cd]
                frames.append(Frame(dd, cd, *seq.intrinsics, depth_scale=seq.depth_scale))
                members.append((lv, lv.arrival(lv.next), "%dx%d" % (seq.width, seq.height)))
                lv.next += 1
            process_batch([lv.session for lv in ready], frames, tp, mp, dynamic, stream)
            ev = torch.cuda.Event(enable_timing=True)
            ev.record(stream)
            inflight.append((ev, members, keep))
            n_steps += 1
            batch_sizes.append(len(ready))
        else:
            if inflight:
                retire(block=len(inflight) >= depth or not ready)
                if hold:
                    time.sleep(0.0002)
            elif not ready:
                # idle until the next arrival (or admission retry)
                nxt = [lv.arrival(lv.next) for lv in live if lv.next < len(lv.spec.arrivals)]
                if waiting:
                    nxt.append(waiting[0].arrivals[0])
                if nxt:
                    time.sleep(max(0.0, min(min(nxt) - now(), 0.002)))
        retire(block=False)
        # release finished sessions
        for lv in [lv for lv in live if lv.done == len(lv.spec.arrivals)]:
            if on_finish is not None:
                on_finish(lv.spec, lv.session)
            live.remove(lv)
            used -= lv.nbytes
            del lv.session
        if progress is not None and n_steps % 200 == 0 and n_steps:
            progress(n_steps, completed, total)
    torch.cuda.synchronize(dev)
    wall = now()
    lat = np.asarray(latencies)
    pr = {k: {"frames": len(v), "p50_ms": round(float(np.percentile(v, 50)), 3),
              "p99_ms": round(float(np.percentile(v, 99)), 3)} for k, v in sorted(per_res.items())}
    return ServeResult(total, wall, lat, np.asarray(waits), n_steps, float(np.mean(batch_sizes)) if batch_sizes else 0.0,
                       peak_sessions, peak_bytes, late, pr)
