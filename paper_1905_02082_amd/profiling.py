"""Helpers for rocprofv3 measurements of the library's kernels.

  python paper_1905_02082_amd/profiling.py copy --mib 1024
      runs a plain device-to-device copy of a known size (the calibration
      kernel for the FETCH_SIZE / WRITE_SIZE counters: it reads and writes
      exactly mib MiB per copy).
  python -m paper_1905_02082_amd.profiling summary DIR [--kernel REGEX] [--by-grid]
      prints per-kernel call counts and durations (optionally split by grid
      size, e.g. per pyramid level) from the rocprofv3 database under DIR.
  python -m paper_1905_02082_amd.profiling pmc --fetch DIR --write DIR
         --copy-fetch DIR --copy-write DIR --kernel REGEX --skip N
         [--l2 DIR] [--copy-mib 1024] [--json OUT --name KERNEL --workload W --storage S]
      HBM bytes per dispatch of the kernels matching REGEX: FETCH_SIZE and
      WRITE_SIZE (KiB per dispatch, each from its own rocprofv3 --pmc run)
      scaled by the factor that makes the same counter read the known size of
      the calibration copy; the first N matching dispatches are skipped
      (warmup).  With --l2, also the L2 hit rate TCC_HIT / (TCC_HIT +
      TCC_MISS) over the same dispatches, from a run with
      --pmc TCC_HIT_sum TCC_MISS_sum.  With --json, writes the figures with the
      hash of the kernel's sources, so a later edit of the kernel invalidates
      them.
"""
from __future__ import annotations

import argparse
import glob
import hashlib
import json
import os
import re
import sqlite3
import statistics
import sys

HERE = os.path.dirname(os.path.abspath(__file__))

# sources whose text determines each measured kernel
KERNEL_SOURCES = {"integrate_kernel": ("rf_fusion.hip", "rf_device.h", "rf_internal.h"),
                  "track_kernel": ("rf_track.hip", "rf_device.h", "rf_internal.h")}


def kernel_source_hash(kernel):
    h = hashlib.sha256()
    for f in KERNEL_SOURCES[kernel]:
        with open(os.path.join(HERE, "csrc", f), "rb") as fh:
            h.update(fh.read())
    return h.hexdigest()[:16]


def copy_kernel(mib: int, reps: int = 5):
    import torch
    dev = torch.device("cuda:0")
    n = mib * 2**20
    a = torch.ones(n, dtype=torch.uint8, device=dev)
    b = torch.empty_like(a)
    torch.cuda.synchronize()
    for _ in range(reps):
        b.copy_(a)
    torch.cuda.synchronize()
    print("copied %d MiB x %d" % (mib, reps), flush=True)


def _db(path):
    dbs = sorted(glob.glob(os.path.join(path, "**", "*.db"), recursive=True))
    if not dbs:
        raise SystemExit("no rocprofv3 database under %s" % path)
    return sqlite3.connect(dbs[-1])


def summary(path, kernel=None, by_grid=False, out=sys.stdout):
    c = _db(path)
    rows = list(c.execute("select name, duration, grid_x, workgroup_x from kernels order by start"))
    by = {}
    for name, dur, gx, wx in rows:
        if kernel and not re.search(kernel, name):
            continue
        key = (name, gx // max(wx, 1)) if by_grid else (name, None)
        by.setdefault(key, []).append(dur)
    print("%-64s %8s %7s %12s %10s %10s" % ("kernel", "groups", "calls", "total_us", "avg_us", "median_us"),
          file=out)
    for (name, g), d in sorted(by.items(), key=lambda kv: -sum(kv[1])):
        print("%-64s %8s %7d %12.1f %10.2f %10.2f" % (name[:64], "" if g is None else g, len(d), sum(d) / 1e3,
                                                       sum(d) / len(d) / 1e3, statistics.median(d) / 1e3),
              file=out)


def last_frames(path, n, out=sys.stdout):
    """Per-kernel time over the last n frames of a kernel trace (a frame ends
    with the integration's fold launch), and the idle time between one
    kernel's end and the next one's start."""
    c = _db(path)
    rows = list(c.execute("select name, start, duration from kernels order by start"))
    ends = [i for i, r in enumerate(rows) if "integ_fold_kernel" in r[0]]
    if len(ends) < n + 1:
        raise SystemExit("fewer than %d frames in the trace" % (n + 1))
    sel = rows[ends[-n - 1] + 1:ends[-1] + 1]
    by = {}
    for name, _, d in sel:
        by.setdefault(re.sub(r"\(.*", "", name), []).append(d / 1e3)
    span = (sel[-1][1] + sel[-1][2] - sel[0][1]) / 1e3
    busy = sum(r[2] for r in sel) / 1e3
    print("last %d frames: %d dispatches, %.1f us per frame, kernel time %.1f us per frame, idle %.1f us per "
          "frame (%.2f us per dispatch)" % (n, len(sel), span / n, busy / n, (span - busy) / n, (span - busy) / len(sel)),
          file=out)
    for k, v in sorted(by.items(), key=lambda kv: -sum(kv[1])):
        print("  %-60s n %5d  avg %8.2f us  per frame %8.1f us" % (k[:60], len(v), sum(v) / len(v), sum(v) / n),
              file=out)


def _counter(path, counter, kernel):
    """Per-dispatch values (dispatch order) of one counter for kernels matching the regex."""
    c = _db(path)
    rows = list(c.execute("select dispatch_id, kernel_name, counter_name, value from counters_collection"))
    vals = {}
    for did, name, ctr, v in rows:
        if ctr == counter and re.search(kernel, str(name)):
            vals[did] = vals.get(did, 0.0) + float(v)
    return [vals[k] for k in sorted(vals)]


def calibration(path, counter, mib):
    """Factor that makes `counter` read the known bytes of the calibration copy."""
    v = _counter(path, counter, r"copyBuffer|copy_kernel|direct_copy")
    if not v:
        raise SystemExit("no copy dispatch under %s" % path)
    kib = statistics.median(v)
    return (mib * 1024.0) / kib, kib


def pmc(args):
    f_fetch, k_fetch = calibration(args.copy_fetch, "FETCH_SIZE", args.copy_mib)
    f_write, k_write = calibration(args.copy_write, "WRITE_SIZE", args.copy_mib)
    fe = _counter(args.fetch, "FETCH_SIZE", args.kernel)[args.skip:]
    wr = _counter(args.write, "WRITE_SIZE", args.kernel)[args.skip:]
    if not fe or not wr:
        raise SystemExit("no matching dispatches after skipping %d" % args.skip)
    fetch_b = statistics.mean(fe) * 1024.0 * f_fetch
    write_b = statistics.mean(wr) * 1024.0 * f_write
    res = {"kernel": args.name or args.kernel, "dispatches": [len(fe), len(wr)],
           "fetch_bytes_per_launch": round(fetch_b), "write_bytes_per_launch": round(write_b),
           "hbm_bytes_per_launch": round(fetch_b + write_b),
           "calibration": {"copy_mib": args.copy_mib, "fetch_kib_read": k_fetch, "fetch_factor": round(f_fetch, 4),
                           "write_kib_read": k_write, "write_factor": round(f_write, 4)}}
    if args.l2:
        hit = _counter(args.l2, "TCC_HIT_sum", args.kernel)[args.skip:]
        miss = _counter(args.l2, "TCC_MISS_sum", args.kernel)[args.skip:]
        if not hit or len(hit) != len(miss):
            raise SystemExit("no matching TCC_HIT_sum / TCC_MISS_sum dispatches under %s" % args.l2)
        res["l2_hit_rate"] = round(sum(hit) / max(sum(hit) + sum(miss), 1.0), 4)
        res["l2_dispatches"] = len(hit)
    if args.json:
        res.update({"workload": args.workload, "storage": args.storage,
                    "kernel_source_hash": kernel_source_hash(args.name)})
        with open(args.json, "w") as fh:
            json.dump(res, fh, indent=1)
    print(json.dumps(res))


def main():
    ap = argparse.ArgumentParser()
    sub = ap.add_subparsers(dest="cmd", required=True)
    a = sub.add_parser("copy")
    a.add_argument("--mib", type=int, default=1024)
    a.add_argument("--reps", type=int, default=5)
    s = sub.add_parser("summary")
    s.add_argument("dir")
    s.add_argument("--kernel", default=None)
    s.add_argument("--by-grid", action="store_true")
    f = sub.add_parser("frames")
    f.add_argument("dir")
    f.add_argument("--last", type=int, default=20)
    p = sub.add_parser("pmc")
    for k in ("fetch", "write", "copy_fetch", "copy_write"):
        p.add_argument("--" + k.replace("_", "-"), dest=k, required=True)
    p.add_argument("--kernel", required=True)
    p.add_argument("--skip", type=int, default=0)
    p.add_argument("--l2", default=None)
    p.add_argument("--copy-mib", type=int, default=1024)
    p.add_argument("--json", default=None)
    p.add_argument("--name", default=None, choices=sorted(KERNEL_SOURCES))
    p.add_argument("--workload", default=None)
    p.add_argument("--storage", default=None)
    args = ap.parse_args()
    if args.cmd == "copy":
        copy_kernel(args.mib, args.reps)
    elif args.cmd == "summary":
        summary(args.dir, args.kernel, args.by_grid)
    elif args.cmd == "frames":
        last_frames(args.dir, args.last)
    else:
        pmc(args)


if __name__ == "__main__":
    main()
