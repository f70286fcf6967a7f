"""Summaries of rocprofv3 output for the committed profiles.

    python -m paper_1208_2080_amd.profiling stats DIR --cmd "..."
        per-kernel call counts and average durations from a
        ``rocprofv3 --kernel-trace --stats --output-format csv`` run;
    python -m paper_1208_2080_amd.profiling pmc FETCH_DIR WRITE_DIR --kernel K --cmd-fetch "..." --cmd-write "..."
        HBM bytes per dispatch of kernel K from two ``--pmc FETCH_SIZE`` /
        ``--pmc WRITE_SIZE`` runs of a command that also makes a 1 GiB device
        copy (bench.py --copy-calibration): the counters read KiB, and the
        copy's readings give the bytes each KiB stands for;
    python -m paper_1208_2080_amd.profiling counters DIR... --kernels K... --cmd "..."
        averages per dispatch of the counters of ``--pmc`` runs (one run per
        counter pass), and instructions per wave;
    python -m paper_1208_2080_amd.profiling phases [--L 16384 --q 2 --xy]
        per-phase shader-clock ticks of the sweep kernels' waves, from the
        profiling library (``python -m paper_1208_2080_amd.build --phase-clocks``
        builds it; a GPU runs it).

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


def counters(dirs, kernels, cmds, sites=None, rows_per_wave=0) -> str:
    """Average per dispatch of every counter in the runs under `dirs` (one run
    per counter pass), for each named kernel at its largest grid; per wave (the
    counters divided by SQ_WAVES), per wave-row (given the rows a wave covers)
    and, given sites per dispatch, per site."""
    tables = []
    for d in dirs:
        names = sorted({r["Counter_Name"] for r in csv.DictReader(open(_find(d, "counter_collection.csv")))})
        tables += [(c, _counter_means(d, c)) for c in names]
    waves = dict(tables).get("SQ_WAVES")
    lines = ["# rocprofv3 --pmc counter summary (per dispatch of the kernel's largest grid)"]
    lines += [f"# command: {c}" for c in cmds]
    lines.append(f"# kernel_source_sha256_16: {kernel_source_digest()}")
    for k in kernels:
        lines.append(f"kernel: {k}")
        w_avg = None
        for cname, table in tables:
            vs = [gv for name, gvs in table.items() if _short(name) == k for gv in gvs]
            if not vs:
                continue
            g = max(x[0] for x in vs)
            vals = [x[1] for x in vs if x[0] == g]
            avg = sum(vals) / len(vals)
            if cname == "SQ_WAVES":
                w_avg = avg
            lines.append(f"  {cname}: {avg:.1f} per dispatch ({len(vals)} dispatches, grid {g})")
        if w_avg:
            for cname, table in tables:
                if cname == "SQ_WAVES" or not cname.startswith("SQ_INSTS"):
                    continue
                vs = [gv for name, gvs in table.items() if _short(name) == k for gv in gvs]
                if vs:
                    g = max(x[0] for x in vs)
                    vals = [x[1] for x in vs if x[0] == g]
                    per = sum(vals) / len(vals) / w_avg
                    extra = f", {sum(vals) / len(vals) * 64 / sites[k]:.1f} lane-instructions per site" \
                        if sites and k in sites else ""
                    if rows_per_wave:
                        extra = f", per wave-row {per / rows_per_wave:.1f}" + extra
                    lines.append(f"  {cname} per wave: {per:.1f}{extra}")
    return "\n".join(lines) + "\n"


# The marks of the kernels' phase clocks (SW_PHASE in the kernel sources), by
# the table each kernel adds to: (kernel, [phase names in mark order]).
PHASE_NAMES = [
    ("k_bond_label", ["staging (spins into LDS)", "rows: draws, ballots, row labels, queue drains, counting",
                      "measurement sums of the strip", "barrier", "seams and the last drain",
                      "bond words out, edge record, barrier", "edge roots, node claims, barrier",
                      "tile labels out", "slots, ring sums"]),
    ("k_merge", ["edge record and slots", "node words, walks to the roots", "hooks"]),
    ("k_flip", ["labels in", "roots inside the tile listed", "node roots found", "states drawn", "barrier",
                "walks", "spins out"]),
    ("k_bond_label (preset bonds, XY)", ["staging", "rows: row labels, queue drains", "measurement sums", "barrier",
                                         "seams and the last drain", "bond words out, edge record, barrier",
                                         "edge roots, node claims, barrier", "tile labels out", "slots, ring sums"]),
    ("k_flip (XY)", ["labels in", "roots inside the tile listed", "node roots found", "states drawn", "barrier",
                     "walks", "reflections"]),
]
PHASES = 10   # phase counters per kernel in the profiling build (PHASES in sw_tile.hpp)


def phases(L: int, q: int, xy: bool, sweeps: int, warmup: int, cmd: str) -> str:
    """Per-phase ticks per wave of the sweep kernels, from `sweeps` sweeps of an
    L x L lattice (Potts q at K_c, or XY near the Kosterlitz-Thouless point)
    swept with the profiling library, after `warmup` sweeps."""
    import ctypes
    import math
    import torch
    from paper_1208_2080_amd import binding, build
    binding.LIB_PATH = build.PHASE_LIB
    lib = binding.lib()
    fn = lib.sw_phase_clocks
    fn.argtypes = [ctypes.POINTER(ctypes.c_ulonglong), ctypes.c_int]
    buf = (ctypes.c_ulonglong * (len(PHASE_NAMES) * (PHASES + 1)))()
    if xy:
        from paper_1208_2080_amd import workloads
        lat = binding.XYLattice(L, workloads.K_KT_XY, seed=1, obs_capacity=64, tile_rows=64)
    else:
        lat = binding.Lattice(L, q, math.log(1 + math.sqrt(q)), seed=1, obs_capacity=64, tile_rows=64)
    lat.sweep(warmup)
    torch.cuda.synchronize()
    if fn(buf, 1):
        raise SystemExit("sw_phase_clocks failed")
    lat.sweep(sweeps)
    torch.cuda.synchronize()
    if fn(buf, 1):
        raise SystemExit("sw_phase_clocks failed")
    lat.close()
    v = list(buf)
    what = f"XY L={L}" if xy else f"Potts q={q} L={L} at K_c"
    lines = ["# per-phase shader-clock ticks per wave (profiling build, -DSW_PHASE_CLOCKS)",
             f"# command: {cmd}",
             f"# kernel_source_sha256_16: {kernel_source_digest()}",
             f"# workload: {what}, tile_rows 64, {sweeps} sweeps after {warmup}; each wave sums the ticks it",
             "# spends between consecutive marks, so a phase's share is of the waves' lifetime (waiting",
             "# included), not of any one issue unit; the marks themselves perturb the timing a little"]
    for k, (name, names) in enumerate(PHASE_NAMES):
        row = v[k * (PHASES + 1):(k + 1) * (PHASES + 1)]
        waves = row[PHASES]
        if not waves:
            continue
        tot = sum(row[:PHASES])
        lines.append(f"kernel: {name}: {waves // sweeps} waves per sweep, {tot / waves:.0f} ticks per wave")
        for i, nm in enumerate(names):
            lines.append(f"  {i}  {nm:58s} {row[i] / waves:8.0f}  {100.0 * row[i] / tot:5.1f} %")
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
    c = sub.add_parser("counters")
    c.add_argument("dirs", nargs="+")
    c.add_argument("--kernels", nargs="+", required=True)
    c.add_argument("--cmd", action="append", required=True)
    c.add_argument("--sites", nargs="*", default=[], help="kernel=sites pairs (sites per dispatch)")
    c.add_argument("--rows-per-wave", type=int, default=0)
    e = sub.add_parser("phases")
    e.add_argument("--L", type=int, default=16384)
    e.add_argument("--q", type=int, default=2)
    e.add_argument("--xy", action="store_true")
    e.add_argument("--sweeps", type=int, default=20)
    e.add_argument("--warmup", type=int, default=20)
    args = ap.parse_args(argv)
    if args.what == "phases":
        cmd = "python -m paper_1208_2080_amd.profiling " + " ".join(argv if argv is not None else sys.argv[1:])
        sys.stdout.write(phases(args.L, args.q, args.xy, args.sweeps, args.warmup, cmd))
        return
    if args.what == "counters":
        sites = {kv.rsplit("=", 1)[0]: float(kv.rsplit("=", 1)[1]) for kv in args.sites}
        sys.stdout.write(counters(args.dirs, args.kernels, args.cmd, sites, args.rows_per_wave))
        return
    if args.what == "stats":
        sys.stdout.write(stats(args.dir, args.cmd))
    else:
        sys.stdout.write(pmc(args.fetch_dir, args.write_dir, args.kernel, args.cmd_fetch, args.cmd_write))


if __name__ == "__main__":
    main()
