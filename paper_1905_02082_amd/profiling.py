"""Helpers for rocprofv3 measurements of the library's kernels.

  python -m paper_1905_02082_amd.profiling copy --mib 1024
      runs a plain device-to-device copy of a known size (the calibration
      kernel for the FETCH_SIZE / WRITE_SIZE counters: it must read and write
      exactly mib MiB).
  python -m paper_1905_02082_amd.profiling summary DIR [--kernel REGEX]
      prints per-kernel call counts and durations (and per-dispatch PMC
      values, when the run collected counters) from the rocprofv3 database
      found under DIR.
"""
from __future__ import annotations

import argparse
import glob
import os
import re
import sqlite3
import statistics
import sys


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


def summary(path, kernel=None, out=sys.stdout):
    c = _db(path)
    rows = list(c.execute("select name, duration, grid_x, workgroup_x, id from kernels"))
    by = {}
    for name, dur, gx, wx, kid in rows:
        if kernel and not re.search(kernel, name):
            continue
        by.setdefault(name, []).append(dur)
    print("%-72s %7s %12s %10s %10s" % ("kernel", "calls", "total_us", "avg_us", "median_us"), file=out)
    for name, d in sorted(by.items(), key=lambda kv: -sum(kv[1])):
        print("%-72s %7d %12.1f %10.2f %10.2f" % (name[:72], len(d), sum(d) / 1e3, sum(d) / len(d) / 1e3,
                                                    statistics.median(d) / 1e3), file=out)
    # per-dispatch counters, if the run collected any
    try:
        rows = list(c.execute("select kernel_name, counter_name, value from counters_collection"))
    except sqlite3.Error:
        rows = []
    if rows:
        vals = {}
        for name, ctr, v in rows:
            if kernel and not re.search(kernel, str(name)):
                continue
            vals.setdefault((str(name)[:60], ctr), []).append(float(v))
        print("\nper-dispatch counters (mean over dispatches):", file=out)
        for (name, ctr), v in sorted(vals.items()):
            print("  %-60s %-12s n=%-5d mean=%.1f" % (name, ctr, len(v), sum(v) / len(v)), file=out)


def main():
    ap = argparse.ArgumentParser()
    sub = ap.add_subparsers(dest="cmd", required=True)
    a = sub.add_parser("copy")
    a.add_argument("--mib", type=int, default=1024)
    a.add_argument("--reps", type=int, default=5)
    s = sub.add_parser("summary")
    s.add_argument("dir")
    s.add_argument("--kernel", default=None)
    args = ap.parse_args()
    if args.cmd == "copy":
        copy_kernel(args.mib, args.reps)
    else:
        summary(args.dir, args.kernel)


if __name__ == "__main__":
    main()
