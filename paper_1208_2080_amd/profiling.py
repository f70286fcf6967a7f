"""Summaries of rocprofv3 output for the committed profiles.

    python -m paper_1208_2080_amd.profiling stats DIR --cmd "..."
        per-kernel call counts and average durations from a
        ``rocprofv3 --kernel-trace --stats --output-format csv`` run;
    python -m paper_1208_2080_amd.profiling pmc FETCH_DIR WRITE_DIR --kernel K --cmd-fetch "..." --cmd-write "..."
        HBM bytes per dispatch of kernel K from two ``--pmc FETCH_SIZE`` /
        ``--pmc WRITE_SIZE`` runs of a command that also makes a 1 GiB device
        copy (bench.py --copy-calibration): the counters read KiB, and the
        copy's readings give the bytes each KiB stands for.

Each summary records the command that produced the data and a digest of the
kernel sources it was taken on (bench.py reports traffic only when that
digest matches the current sources).
"""
from __future__ import annotations

import argparse
import csv
import glob
import hashlib
import os
import sys
from collections import defaultdict

HERE = os.path.dirname(os.path.abspath(__file__))
COPY_BYTES = 1 << 30


def kernel_source_digest() -> str:
    h = hashlib.sha256()
    for name in ("sw_kernels.hip", "sw_device.hpp", "sw_layout.hpp"):
        with open(os.path.join(HERE, "csrc", name), "rb") as f:
            h.update(f.read())
    return h.hexdigest()[:16]


def _short(name: str) -> str:
    base = name.split("(")[0].replace("void ", "").replace("swmi::", "")
    return base


def _find(d: str, suffix: str) -> str:
    hits = glob.glob(os.path.join(d, "**", "*" + suffix), recursive=True)
    if not hits:
        raise SystemExit(f"no *{suffix} under {d}")
    return sorted(hits)[0]


def stats(d: str, cmd: str) -> str:
    rows = list(csv.DictReader(open(_find(d, "kernel_stats.csv"))))
    out = ["# rocprofv3 kernel-trace summary", f"# command: {cmd}",
           f"# kernel_source_sha256_16: {kernel_source_digest()}",
           f"{'kernel':60s} {'calls':>7s} {'avg_us':>10s} {'total_ms':>10s} {'pct':>6s}"]
    for r in rows:
        out.append(f"{_short(r['Name'])[:60]:60s} {int(r['Calls']):7d} {float(r['AverageNs']) / 1e3:10.2f} "
                   f"{float(r['TotalDurationNs']) / 1e6:10.3f} {float(r['Percentage']):6.2f}")
    return "\n".join(out) + "\n"


def _counter_means(d: str, counter: str):
    """Average value of `counter` per dispatch, by kernel (summed over the
    counter's instances within a dispatch)."""
    per_dispatch = defaultdict(float)
    names = {}
    for r in csv.DictReader(open(_find(d, "counter_collection.csv"))):
        if r["Counter_Name"] != counter:
            continue
        key = r["Dispatch_Id"]
        per_dispatch[key] += float(r["Counter_Value"])
        names[key] = r["Kernel_Name"]
    by_kernel = defaultdict(list)
    for key, v in per_dispatch.items():
        by_kernel[names[key]].append(v)
    return by_kernel


def pmc(fetch_dir: str, write_dir: str, kernel: str, cmd_fetch: str, cmd_write: str) -> str:
    fetch = _counter_means(fetch_dir, "FETCH_SIZE")
    write = _counter_means(write_dir, "WRITE_SIZE")

    def pick(table):
        vals = [v for name, vs in table.items() if _short(name).startswith(kernel + "<") or _short(name) == kernel
                for v in vs]
        if not vals:
            raise SystemExit(f"kernel {kernel} not in the counters")
        return vals

    def copy_reading(table):
        # the largest blit copy of the run is the 1 GiB calibration copy
        vals = [v for name, vs in table.items() if "copyBuffer" in name for v in vs]
        if not vals:
            raise SystemExit("no device copy in the counters (run with --copy-calibration)")
        return max(vals)

    fk, wk = pick(fetch), pick(write)
    cf, cw = copy_reading(fetch), copy_reading(write)
    f_avg, w_avg = sum(fk) / len(fk), sum(wk) / len(wk)
    fs, ws = COPY_BYTES / cf, COPY_BYTES / cw
    lines = ["# rocprofv3 --pmc FETCH_SIZE / WRITE_SIZE (KiB per dispatch)",
             f"# command (fetch): {cmd_fetch}", f"# command (write): {cmd_write}",
             f"kernel: {kernel}", f"dispatches: {len(fk)}",
             f"kernel_source_sha256_16: {kernel_source_digest()}",
             f"fetch_kib_per_dispatch: {f_avg:.1f}", f"write_kib_per_dispatch: {w_avg:.1f}",
             f"copy_fetch_kib: {cf:.1f}", f"copy_write_kib: {cw:.1f}",
             f"fetch_scale_bytes_per_kib: {fs:.3f}", f"write_scale_bytes_per_kib: {ws:.3f}",
             f"traffic_bytes_per_dispatch: {f_avg * fs + w_avg * ws:.0f}"]
    return "\n".join(lines) + "\n"


def main(argv=None):
    ap = argparse.ArgumentParser(description=__doc__, formatter_class=argparse.RawDescriptionHelpFormatter)
    sub = ap.add_subparsers(dest="what", required=True)
    a = sub.add_parser("stats")
    a.add_argument("dir")
    a.add_argument("--cmd", required=True)
    b = sub.add_parser("pmc")
    b.add_argument("fetch_dir")
    b.add_argument("write_dir")
    b.add_argument("--kernel", required=True)
    b.add_argument("--cmd-fetch", required=True)
    b.add_argument("--cmd-write", required=True)
    args = ap.parse_args(argv)
    if args.what == "stats":
        sys.stdout.write(stats(args.dir, args.cmd))
    else:
        sys.stdout.write(pmc(args.fetch_dir, args.write_dir, args.kernel, args.cmd_fetch, args.cmd_write))


if __name__ == "__main__":
    main()
