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
    for name in ("sw_kernels.hip", "sw_xy.hip", "sw_whole.hip", "sw_tile.hpp", "sw_device.hpp", "sw_layout.hpp"):
        with open(os.path.join(HERE, "csrc", name), "rb") as f:
            h.update(f.read())
    return h.hexdigest()[:16]


def _short(name: str) -> str:
    base = name.replace("(anonymous namespace)::", "").split("(")[0]
    return base.replace("void ", "").replace("swmi::", "")


def _find(d: str, suffix: str) -> str:
    hits = glob.glob(os.path.join(d, "**", "*" + suffix), recursive=True)
    if not hits:
        raise SystemExit(f"no *{suffix} under {d}")
    return sorted(hits)[0]


def _grid(r) -> int:
    for key in ("Grid_Size", "Grid_Size_X"):
        if key in r and r[key] not in ("", None):
            return int(float(r[key]))
    return 0


def stats(d: str, cmd: str) -> str:
    """Per-kernel dispatch counts and average durations from the kernel trace;
    each kernel counts only its dispatches of the largest grid in the run (the
    workload the run was made for, not smaller side runs of the same kernel)."""
    by_name = defaultdict(list)
    for r in csv.DictReader(open(_find(d, "kernel_trace.csv"))):
        by_name[_short(r["Kernel_Name"])].append((_grid(r), int(r["End_Timestamp"]) - int(r["Start_Timestamp"])))
    rows = []
    for name, v in by_name.items():
        g = max(x[0] for x in v)
        durs = [x[1] for x in v if x[0] == g]
        rows.append((name, g, len(durs), sum(durs) / len(durs), sum(durs)))
    total = sum(r[4] for r in rows)
    rows.sort(key=lambda r: -r[4])
    out = ["# rocprofv3 kernel-trace summary (per kernel: its dispatches of the largest grid)",
           f"# command: {cmd}", f"# kernel_source_sha256_16: {kernel_source_digest()}",
           f"{'kernel':44s} {'grid':>10s} {'calls':>7s} {'avg_us':>10s} {'total_ms':>10s} {'pct':>6s}"]
    for name, g, n, avg, tot in rows:
        out.append(f"{name[:44]:44s} {g:10d} {n:7d} {avg / 1e3:10.2f} {tot / 1e6:10.3f} {100 * tot / total:6.2f}")
    return "\n".join(out) + "\n"


def _counter_means(d: str, counter: str):
    """Average value of `counter` per dispatch, by kernel (summed over the
    counter's instances within a dispatch)."""
    per_dispatch = defaultdict(float)
    names, grids = {}, {}
    for r in csv.DictReader(open(_find(d, "counter_collection.csv"))):
        if r["Counter_Name"] != counter:
            continue
        key = r["Dispatch_Id"]
        per_dispatch[key] += float(r["Counter_Value"])
        names[key] = r["Kernel_Name"]
        grids[key] = _grid(r)
    by_kernel = defaultdict(list)
    for key, v in per_dispatch.items():
        by_kernel[names[key]].append((grids[key], v))
    return by_kernel


def pmc(fetch_dir: str, write_dir: str, kernel: str, cmd_fetch: str, cmd_write: str) -> str:
    fetch = _counter_means(fetch_dir, "FETCH_SIZE")
    write = _counter_means(write_dir, "WRITE_SIZE")

    def pick(table):
        # the kernel's instantiation named exactly, its dispatches of the largest grid
        vs = [gv for name, gvs in table.items() if _short(name) == kernel for gv in gvs]
        if not vs:
            raise SystemExit(f"kernel {kernel} not in the counters")
        g = max(x[0] for x in vs)
        return [x[1] for x in vs if x[0] == g]

    def copy_reading(table):
        # the largest blit copy of the run is the 1 GiB calibration copy
        vals = [v for name, gvs in table.items() if "copyBuffer" in name for _, v in gvs]
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
