"""Summaries of rocprofv3 output for the rollout kernels.

  python -m paper_1503_00330_amd.profiling stats <kernel_stats.csv> [--top N]
      per-kernel call count and mean/min/max duration (``--kernel-trace --stats``)
  python -m paper_1503_00330_amd.profiling counters <pmc_dir> [<pmc_dir> ...] --kernel NAME
      mean per dispatch of every counter collected for one kernel (``--pmc``,
      csv output), over one or more runs
  python -m paper_1503_00330_amd.profiling traffic <fetch_dir> <write_dir>
          --kernel NAME --copy-bytes B
      HBM bytes per launch of one kernel from a FETCH_SIZE run and a WRITE_SIZE
      run (``--pmc``, csv output), each counter scaled by what it reads for the
      largest ``copyBuffer`` dispatch of the same run, a plain copy of B bytes

``stats`` and ``counters`` print markdown tables, ``traffic`` ``key: value`` lines.  The traffic
summary records a digest of the rollout kernel sources, so a reader can tell
whether the counters still describe the current kernel.
"""
from __future__ import annotations

import argparse
import csv
import glob
import hashlib
import os
from collections import defaultdict
from typing import Dict, List, Optional

HERE = os.path.dirname(os.path.abspath(__file__))
KERNEL_SOURCES = ("csrc/mfma.hip", "csrc/common.hpp", "csrc/internal.hpp", "build.py")


def source_digest() -> str:
    """sha256 over the sources the matrix-core rollout kernels are built from
    and the build script that holds their compiler flags."""
    h = hashlib.sha256()
    for rel in KERNEL_SOURCES:
        with open(os.path.join(HERE, rel), "rb") as f:
            h.update(rel.encode() + b"\0" + f.read())
    return h.hexdigest()


def _csv(path: str, suffix: str) -> str:
    if os.path.isdir(path):
        hits = sorted(glob.glob(os.path.join(path, "**", "*" + suffix), recursive=True))
        if not hits:
            raise FileNotFoundError("no *%s under %s" % (suffix, path))
        return hits[0]
    return path


def kernel_stats(path: str, top: int = 12) -> List[dict]:
    rows = list(csv.DictReader(open(_csv(path, "kernel_stats.csv"))))
    out = []
    for r in rows[:top]:
        out.append({"name": r["Name"], "calls": int(r["Calls"]), "avg_us": float(r["AverageNs"]) / 1e3,
                    "min_us": float(r["MinNs"]) / 1e3, "max_us": float(r["MaxNs"]) / 1e3,
                    "pct": float(r["Percentage"])})
    return out


def _counter(path: str, counter: str) -> Dict[str, List[float]]:
    vals: Dict[str, List[float]] = defaultdict(list)
    for r in csv.DictReader(open(_csv(path, "counter_collection.csv"))):
        if r["Counter_Name"] == counter:
            vals[r["Kernel_Name"]].append(float(r["Counter_Value"]))
    return vals


def counters(dirs: List[str], kernel: str) -> Dict[str, float]:
    """Mean per dispatch of each counter of `kernel` over the runs in `dirs`."""
    vals: Dict[str, List[float]] = defaultdict(list)
    for d in dirs:
        for r in csv.DictReader(open(_csv(d, "counter_collection.csv"))):
            if kernel in r["Kernel_Name"]:
                vals[r["Counter_Name"]].append(float(r["Counter_Value"]))
    if not vals:
        raise ValueError("no dispatches of %r" % kernel)
    return {k: sum(v) / len(v) for k, v in sorted(vals.items())}


def traffic(fetch_dir: str, write_dir: str, kernel: str, copy_bytes: int) -> dict:
    """Bytes per launch of `kernel`: FETCH_SIZE and WRITE_SIZE (KiB per
    dispatch) averaged over its dispatches, each scaled by copy_bytes over what
    the counter read for the largest copyBuffer dispatch of its run."""
    res = {}
    for key, path, counter in (("fetch", fetch_dir, "FETCH_SIZE"), ("write", write_dir, "WRITE_SIZE")):
        vals = _counter(path, counter)
        kern = [v for name, vs in vals.items() if kernel in name for v in vs]
        copy = [v for name, vs in vals.items() if "copyBuffer" in name for v in vs]
        if not kern or not copy:
            raise ValueError("%s: no dispatches of %r or of a copy kernel" % (counter, kernel))
        scale = copy_bytes / (max(copy) * 1024.0)
        res[key + "_kib_per_dispatch"] = sum(kern) / len(kern)
        res[key + "_dispatches"] = len(kern)
        res[key + "_copy_scale"] = scale
        res[key + "_bytes_per_launch"] = sum(kern) / len(kern) * 1024.0 * scale
    res["traffic_bytes_per_launch"] = res["fetch_bytes_per_launch"] + res["write_bytes_per_launch"]
    return res


def read_summary(path: str) -> Dict[str, str]:
    """The key: value lines of a summary written by this module."""
    out = {}
    with open(path) as f:
        for line in f:
            if ":" in line and not line.startswith((" ", "|", "#")):
                k, v = line.split(":", 1)
                out[k.strip()] = v.strip()
    return out


def launch_tag(plan: dict) -> str:
    """variant/samples/waves/split of a rollout_describe() result."""
    return "%s/%d/%d/%d" % (plan["variant"], plan["tile_samples"], plan["tile_waves"], plan["tile_split"])


def traffic_from_summary(path: str, launch: Optional[str] = None) -> Optional[float]:
    """Bytes per launch recorded in a traffic summary, or None when the file is
    missing, the kernel sources changed since the counters were taken, or
    (given `launch`, see launch_tag) the summary records another launch."""
    if not os.path.exists(path):
        return None
    s = read_summary(path)
    if s.get("source_sha256") != source_digest():
        return None
    if launch is not None and s.get("launch", launch) != launch:
        return None
    try:
        return float(s["traffic_bytes_per_launch"])
    except (KeyError, ValueError):
        return None


def main(argv=None):
    ap = argparse.ArgumentParser()
    sub = ap.add_subparsers(dest="cmd", required=True)
    a = sub.add_parser("stats")
    a.add_argument("csv")
    a.add_argument("--top", type=int, default=12)
    c = sub.add_parser("counters")
    c.add_argument("dirs", nargs="+")
    c.add_argument("--kernel", required=True)
    b = sub.add_parser("traffic")
    b.add_argument("fetch_dir")
    b.add_argument("write_dir")
    b.add_argument("--kernel", required=True)
    b.add_argument("--copy-bytes", type=int, required=True)
    b.add_argument("--launch", help="the launch profiled, variant/samples/waves/split")
    args = ap.parse_args(argv)
    if args.cmd == "stats":
        print("| kernel | calls | avg us | min us | max us | % |")
        print("|---|---|---|---|---|---|")
        for r in kernel_stats(args.csv, args.top):
            print("| %s | %d | %.1f | %.1f | %.1f | %.2f |" % (r["name"][:110], r["calls"], r["avg_us"],
                                                             r["min_us"], r["max_us"], r["pct"]))
    elif args.cmd == "counters":
        print("| counter | mean per dispatch |")
        print("|---|---|")
        for k, v in counters(args.dirs, args.kernel).items():
            print("| %s | %.4g |" % (k, v))
    else:
        r = traffic(args.fetch_dir, args.write_dir, args.kernel, args.copy_bytes)
        print("kernel: %s" % args.kernel)
        if args.launch:
            print("launch: %s" % args.launch)
        print("source_sha256: %s" % source_digest())
        for k in sorted(r):
            print("%s: %.6g" % (k, r[k]))


if __name__ == "__main__":
    main()
