#!/usr/bin/env python3
"""Benchmark of the Swendsen-Wang sweep on one MI355X.

One step = one full SW sweep (bonds, cluster labels, flip) of the 2D q-state
Potts model including the measurement of energy and state counts ("update +
measurement" of the paper's Table 1).  Default workload: q = 2 at the critical
coupling K_c = ln(1 + sqrt 2), L = 16384 (2^28 sites), random start, synthetic.

Prints one JSON line: spin flips per ns (L^2 x sweeps / time), the roofline of
the dominant kernel (HIP-event time per launch against its algorithmic bytes),
and the CPU oracle timed on a bounded sample of the same workload.
"""
from __future__ import annotations

import argparse
import json
import os
import sys
import time

ROOT = os.path.dirname(os.path.abspath(__file__))
if ROOT not in sys.path:
    sys.path.insert(0, ROOT)

HBM_PEAK_GBS = 8000.0            # MI355X HBM3E, vendor figure
FP64_PEAK_TFLOPS = 78.6          # MI355X dense FP64 vector, vendor figure
# FP64 arithmetic of the XY bond kernel per site, a neighbour's values counted
# once: sin and cos of the angle (37), the projection (3), the two bond tests
# (7: the FP32 estimates not counted), the measurement terms (30)
XY_BOND_FLOPS_PER_SITE = 77
# Algorithmic bytes per site of one launch: the byte model of the method's
# stated layout (uint8 spins, uint32 labels, 2-bit bond masks).  The kernels
# store 16-bit tile labels, so they move 2 B/site less each than this model
# counts (3.25 and 3.0 B/site); the measured bytes are the roofline's
# `traffic`.
KERNEL_BYTES_PER_SITE = {
    "k_bond_label": 1.0 + 0.25 + 4.0,   # read spins, write bond planes, write labels
    "k_flip": 4.0 + 1.0,                # read labels, write spins
}
SWEEP_BYTES_PER_SITE = 10.25
PHASE_KERNELS = ["k_bond_label", "k_merge", "k_flip", "k_measure+k_bump"]


def workloads():
    from paper_1208_2080_amd import workloads as wl
    return {
        "L16384": dict(wl.PLAIN_16384),
        "L4096": dict(wl.PLAIN_4096),
        "L65536q2": dict(wl.HUGE_Q2),
        "L65536q3": dict(wl.HUGE_Q3),
        "L64": dict(wl.SMALL),
    }


def kernel_source_digest() -> str:
    from paper_1208_2080_amd.profiling import kernel_source_digest as digest
    return digest()


def measured_traffic(kernel: str, workload: str, tile_rows: int):
    """HBM bytes per launch from committed rocprofv3 PMC summaries, if they were
    taken on the current kernel source (else None)."""
    path = os.path.join(ROOT, "profiles", f"{kernel}_{workload}_ty{tile_rows}_pmc.txt")
    if not os.path.exists(path):
        return None
    vals = {}
    with open(path) as f:
        for line in f:
            if ":" in line and not line.startswith("#"):
                k, v = line.split(":", 1)
                vals[k.strip()] = v.strip()
    try:
        if vals.get("kernel_source_sha256_16") != kernel_source_digest():
            return None
        return (float(vals["fetch_kib_per_dispatch"]) * float(vals["fetch_scale_bytes_per_kib"])
                + float(vals["write_kib_per_dispatch"]) * float(vals["write_scale_bytes_per_kib"]))
    except (KeyError, ValueError):
        return None


def cpu_baseline(cfg: dict) -> dict:
    """The CPU oracle, single-threaded, on one sweep of the same lattice."""
    import oracle
    L = cfg["L"]
    lat = oracle.OracleLattice(L, cfg["q"], cfg["K"], cfg["seed"], random_start=cfg["random_start"])
    t0 = time.perf_counter()
    lat.run(1)
    dt = time.perf_counter() - t0
    cpu = host_cpu()
    return {"value": L * L / (dt * 1e9), "unit": "spin flips/ns", "cores": 1, "kind": "oracle",
            "sample": f"1 sweep of the same L={L} q={cfg['q']} lattice from its start (sweep 0), "
                      f"{dt:.1f} s on 1 host core ({cpu['nproc']} available)",
            "cpu_model": cpu["cpu_model"], "nproc": cpu["nproc"]}


def host_cpu() -> dict:
    """The host's CPU model and the cores this process may use."""
    model = "unknown"
    try:
        with open("/proc/cpuinfo") as f:
            for line in f:
                if line.startswith("model name"):
                    model = line.split(":", 1)[1].strip()
                    break
    except OSError:
        pass
    try:
        cores = len(os.sched_getaffinity(0))
    except AttributeError:
        cores = os.cpu_count() or 1
    return {"cpu_model": model, "nproc": cores}


def copy_calibration(nbytes: int = 1 << 30):
    """A plain device copy of known size, for scaling HBM byte counters."""
    import torch
    a = torch.empty(nbytes, dtype=torch.uint8, device="cuda")
    b = torch.empty_like(a)
    a.fill_(1)
    torch.cuda.synchronize()
    b.copy_(a)
    torch.cuda.synchronize()
    del a, b


def copy_ceiling(nbytes: int = 1 << 30, reps: int = 10) -> dict:
    """The HBM rate a plain device-to-device copy reaches (read + write bytes
    per second), timed with HIP events: the practical ceiling next to the 8 TB/s
    peak."""
    import torch
    a = torch.empty(nbytes, dtype=torch.uint8, device="cuda")
    b = torch.empty_like(a)
    a.fill_(1)
    b.copy_(a)
    e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
    torch.cuda.synchronize()
    e0.record()
    for _ in range(reps):
        b.copy_(a)
    e1.record()
    e1.synchronize()
    ms = e0.elapsed_time(e1) / reps
    del a, b
    torch.cuda.empty_cache()
    return {"bytes_per_copy": 2 * nbytes, "ms": ms, "GB_per_s": 2 * nbytes / (ms * 1e-3) / 1e9}


def huge_lattices(warmup: int, steps: int) -> dict:
    """L = 65536 (2^32 sites, one lattice of ~23 GiB) from the cold start, q = 2
    and q = 3 at K_c: flips/ns over `steps` sweeps after `warmup`, with the
    per-kernel HIP-event times and the roofline fraction of the labelling kernel."""
    import torch
    from paper_1208_2080_amd import binding
    out = {}
    for name in ("L65536q2", "L65536q3"):
        cfg = workloads()[name]
        L, q = cfg["L"], cfg["q"]
        N = L * L
        print(f"# {name}: L={L} q={q} cold start, {warmup} + {steps} sweeps", file=sys.stderr, flush=True)
        lat = binding.Lattice(L, q, cfg["K"], seed=cfg["seed"], random_start=cfg["random_start"], obs_capacity=64)
        lat.sweep(warmup)
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        ph = lat.sweep_profiled(steps)
        wall = time.perf_counter() - t0
        obs = lat.measure(lat.sweeps_done - 1, 1)[0]
        assert obs[2:].sum() == N, "observable counts do not sum to N"
        lat.close()
        del lat
        torch.cuda.empty_cache()
        per = {PHASE_KERNELS[i]: ph[i] / steps for i in range(3)}
        bl = KERNEL_BYTES_PER_SITE["k_bond_label"] * N / (per["k_bond_label"] * 1e-3) / 1e9
        value = N * steps / (wall * 1e9)
        out[name] = {"L": L, "q": q, "K": cfg["K"], "start": "cold", "warmup": warmup, "steps": steps,
                     "flips_per_ns": value, "phase_ms_per_sweep": per,
                     "k_bond_label_GB_per_s": bl, "k_bond_label_frac": bl / HBM_PEAK_GBS,
                     "k_bond_label_traffic": measured_traffic("k_bond_label", name, 64),
                     "sweep_roofline_frac": value * SWEEP_BYTES_PER_SITE / HBM_PEAK_GBS}
    return out


def small_lattice(sweeps: int) -> dict:
    """The small correctness configuration (L = 64, q = 2, K_c, random start,
    measurement every sweep) timed on its own: launch-bound at this size, so
    the sweeps replay captured HIP graphs."""
    import torch
    from paper_1208_2080_amd import binding
    cfg = workloads()["L64"]
    L = cfg["L"]
    lat = binding.Lattice(L, cfg["q"], cfg["K"], seed=cfg["seed"], random_start=cfg["random_start"],
                          obs_capacity=sweeps + 1)
    lat.sweep(20)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    lat.sweep(sweeps)
    torch.cuda.synchronize()
    wall = time.perf_counter() - t0
    lat.close()
    return {"L": L, "q": cfg["q"], "sweeps": sweeps, "flips_per_ns": L * L * sweeps / (wall * 1e9),
            "us_per_sweep": wall * 1e6 / sweeps}


def xy_lattice(warmup: int, steps: int, with_cpu: bool) -> dict:
    """The XY model (Wolff's embedded clusters) on the same machinery: an
    L = 16384 lattice near the KT coupling, random start, measurement every
    sweep; per-phase device times from HIP events (bonds + labels, merge,
    reflections, final measurement), and the XY oracle on one L = 4096 sweep."""
    import torch
    from paper_1208_2080_amd import binding
    from paper_1208_2080_amd import workloads as wl
    cfg = dict(wl.XY_16384)
    L, K = cfg["L"], cfg["K"]
    lat = binding.XYLattice(L, K, seed=cfg["seed"], random_start=True, obs_capacity=steps + 1)
    print(f"# XY L={L} K={K}: {warmup} + {steps} sweeps", file=sys.stderr, flush=True)
    lat.sweep(warmup)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    ph = lat.sweep_profiled(steps)
    torch.cuda.synchronize()
    wall = time.perf_counter() - t0
    row = lat.measure(lat.sweeps_done - 1, 1)[0]
    d = binding.xy_derived(row, L, K)
    lat.close()
    del lat
    torch.cuda.empty_cache()
    out = {"workload": f"SW sweep with embedded clusters, 2D XY L={L} K={K} periodic, random start, "
                       f"update + measurement", "L": L, "K": K, "sweeps": steps,
           "flips_per_ns": L * L * steps / (wall * 1e9), "ms_per_sweep": wall * 1e3 / steps,
           "phase_ms_per_sweep": {"k_xy_bonds+k_bond_label": ph[0] / steps, "k_merge": ph[1] / steps,
                                  "k_flip(reflect)": ph[2] / steps, "final measure": ph[3]},
           "energy_per_site_last": d["e"]}
    bond_ms = ph[4] / steps
    achieved = XY_BOND_FLOPS_PER_SITE * L * L / (bond_ms * 1e-3) / 1e12
    out["roofline"] = {"bound": "alu", "kernel": "k_xy_bonds", "achieved": achieved, "peak": FP64_PEAK_TFLOPS,
                       "unit": "TFLOP/s", "frac": achieved / FP64_PEAK_TFLOPS,
                       "traffic": measured_traffic("k_xy_bonds", "xyL16384", 64),
                       "alg_flops_per_launch": XY_BOND_FLOPS_PER_SITE * L * L, "avg_launch_ms": bond_ms}
    if with_cpu:
        import oracle
        Lc = cfg["cpu_L"]
        ref = oracle.XYOracleLattice(Lc, K, cfg["seed"])
        t0 = time.perf_counter()
        ref.sweep()
        dt = time.perf_counter() - t0
        out["cpu_oracle"] = {"value": Lc * Lc / (dt * 1e9), "unit": "spin flips/ns", "cores": 1, "kind": "oracle",
                             "sample": f"one XY sweep (with measurement) of L = {Lc}"}
    return out


def _oracle_replica(args):
    import oracle
    r, sweeps = args
    lat = oracle.OracleLattice(r["L"], r["q"], r["K"], r["seed"], random_start=r.get("random_start", True))
    t0 = time.perf_counter()
    lat.run(sweeps)
    return r["L"] ** 2 * sweeps, time.perf_counter() - t0


def cpu_baseline_batched(n_replicas: int, sweeps: int) -> dict:
    """The oracle on the batched mix over all host cores, one replica per
    process: aggregate flips/ns over the wall time of the pool."""
    import multiprocessing as mp
    from paper_1208_2080_amd import workloads as wl
    reps = wl.batched_replicas(n=n_replicas, sweeps=sweeps)
    cores = min(host_cpu()["nproc"], 16)
    t0 = time.perf_counter()
    with mp.get_context("spawn").Pool(cores) as pool:
        res = pool.map(_oracle_replica, [(r, sweeps) for r in reps], chunksize=1)
    wall = time.perf_counter() - t0
    flips = sum(f for f, _ in res)
    return {"value": flips / (wall * 1e9), "unit": "spin flips/ns", "cores": cores, "kind": "oracle",
            "sample": f"{sweeps} sweep(s) of each of the {n_replicas} batched replicas (one per process), "
                      f"{wall:.1f} s wall"}


def batched_vs_plain(n_replicas: int, sweeps: int, tile_rows: int) -> dict:
    """Aggregate flips/ns of independent replicas of uneven L, q, K swept as one
    batch (one launch per phase, HIP graph) versus one lattice after another.
    Without an explicit tile height the library's autotuner picks it (outside
    the timed region), and the plain loop uses the same height."""
    import numpy as np
    import torch
    from paper_1208_2080_amd import binding
    from paper_1208_2080_amd import workloads as wl

    reps = wl.batched_replicas(n=n_replicas, sweeps=sweeps)
    flips = sum(r["L"] ** 2 for r in reps) * sweeps
    b = binding.Batch(reps, obs_capacity=2, tile_rows=tile_rows or "auto")
    tile_rows = b.tile_rows
    b.sweep_all(2)                                   # warm-up (and graph capture)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    done = 0
    while done < sweeps:
        n = min(100, sweeps - done)
        b.sweep_all(n)
        done += n
    torch.cuda.synchronize()
    t_batch = time.perf_counter() - t0
    lats = [binding.Lattice(r["L"], r["q"], r["K"], seed=r["seed"], obs_capacity=2, tile_rows=tile_rows)
            for r in reps]
    for lat in lats:
        lat.sweep(2)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    for lat in lats:
        lat.sweep(sweeps)
    torch.cuda.synchronize()
    t_plain = time.perf_counter() - t0
    same = all(np.array_equal(b.spins(i), lat.spins()) for i, lat in enumerate(lats))
    for lat in lats:
        lat.close()
    b_tuned = b.tuned_ms
    b.close()
    return {"replicas": n_replicas, "sweeps": sweeps, "sites": flips // sweeps, "tile_rows": tile_rows,
            "autotune_ms_per_sweep": b_tuned,
            "batched_flips_per_ns": flips / (t_batch * 1e9), "plain_flips_per_ns": flips / (t_plain * 1e9),
            "speedup": t_plain / t_batch, "identical_results": bool(same)}


def small_mixes(sweeps: int) -> list:
    """Batches of many small lattices (q = 2 at K_c, random start): 1024 of
    L = 64, 256 of L = 128, 64 of L = 256 -- the same number of sites each,
    swept as one batch (one launch per phase, HIP graph): flips/ns and
    microseconds per batch sweep."""
    import torch
    from paper_1208_2080_amd import binding
    from paper_1208_2080_amd import workloads as wl
    out = []
    for n, L in ((1024, 64), (256, 128), (64, 256)):
        reps = [{"L": L, "q": 2, "K": wl.critical_coupling(2), "seed": 5000 + r, "random_start": True}
                for r in range(n)]
        # the default (whole lattice in LDS where L <= 128) and 64-row tiles
        for ty in ((0, 64) if L <= binding.WHOLE_LMAX else (0,)):
            b = binding.Batch(reps, obs_capacity=2, tile_rows=ty)
            b.sweep_all(2)
            torch.cuda.synchronize()
            t0 = time.perf_counter()
            done = 0
            while done < sweeps:
                k = min(100, sweeps - done)
                b.sweep_all(k)
                done += k
            torch.cuda.synchronize()
            wall = time.perf_counter() - t0
            b.close()
            path = "whole" if (ty == 0 and L <= binding.WHOLE_LMAX) else "tiles64"
            out.append({"replicas": n, "L": L, "path": path, "sweeps": sweeps,
                        "flips_per_ns": n * L * L * sweeps / (wall * 1e9), "us_per_batch_sweep": wall * 1e6 / sweeps})
    return out


def label_equivalence(lat, sweeps: int, per_launch_ms: dict) -> dict:
    """The paper's labelling (iterated label equivalence: scan + analysis under
    a host loop) on the bonds of `sweeps` further sweeps of the bench lattice,
    against this library's tile union-find + merge on the same lattice."""
    import numpy as np

    passes, ms, same = [], [], True
    for _ in range(sweeps):
        lat.sweep(1)
        le, n, t = lat.label_equivalence()
        passes.append(n)
        ms.append(t)
        same = same and bool(np.array_equal(le, lat.labels()))
        del le
    return {"sweeps": sweeps, "mean_passes": float(np.mean(passes)), "passes": passes,
            "ms_per_labelling": float(np.mean(ms)), "ms_per_pass": float(np.sum(ms) / np.sum(passes)),
            "tile_union_find_ms": per_launch_ms["k_bond_label"] + per_launch_ms["k_merge"],
            "identical_labels": same}


def serving(n_jobs: int, capacity_flips_per_ns: float, tile_rows: int, loads=(0.5, 0.9, 1.2)) -> list:
    """The continuous-batching server on Poisson job streams offered at fractions
    of the measured single-lattice capacity (jobs/s = load x flips/s / mean flips
    per job), under a 64 GiB HBM budget."""
    import numpy as np
    from paper_1208_2080_amd import serve
    from paper_1208_2080_amd import workloads as wl

    probe = wl.serving_jobs(n=4000)
    mean_flips = float(np.mean([j["L"] ** 2 * j["sweeps"] for j in probe]))
    out = []
    for load in loads:
        rate = load * capacity_flips_per_ns * 1e9 / mean_flips
        raw = wl.serving_jobs(n=n_jobs, rate_per_s=rate)
        jobs = [serve.Job(id=j["id"], L=j["L"], q=j["q"], K=j["K"], seed=j["seed"], sweeps=j["sweeps"],
                          arrival=j["arrival"]) for j in raw]
        backend = serve.GpuBackend(max_jobs=128, max_tiles=1 << 20, tile_rows=tile_rows)
        srv = serve.SwServer(backend, hbm_budget=64 << 30, max_jobs=128, max_tiles=1 << 20, step_sweeps=20)
        print(f"# serving {n_jobs} jobs at {load:.1f} x capacity ({rate:.2f} jobs/s)", file=sys.stderr, flush=True)
        _, stats = srv.run(jobs, realtime=True)
        backend.close()
        out.append(dict(stats, load=load, offered_jobs_per_s=rate))
    # the same jobs one after another, each as a plain lattice, all at once
    # (no arrivals): the per-job loop the server is measured against
    import torch
    from paper_1208_2080_amd import binding
    raw = wl.serving_jobs(n=n_jobs, rate_per_s=1.0)
    print(f"# the {n_jobs} jobs one after another", file=sys.stderr, flush=True)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    for j in raw:
        lat = binding.Lattice(j["L"], j["q"], j["K"], seed=j["seed"], obs_capacity=j["sweeps"] + 1,
                              tile_rows=tile_rows)
        lat.sweep(j["sweeps"])
        lat.measure(0, j["sweeps"])
        lat.spins()
        lat.close()
    wall = time.perf_counter() - t0
    flips = sum(j["L"] ** 2 * j["sweeps"] for j in raw)
    out.append({"plain_per_job_loop": True, "jobs": n_jobs, "wall_s": wall, "flips_per_ns": flips / (wall * 1e9)})
    return out


def main():
    ap = argparse.ArgumentParser(description=__doc__, formatter_class=argparse.RawDescriptionHelpFormatter)
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=2000, help="timed sweeps")
    ap.add_argument("--warmup", type=int, default=50, help="untimed sweeps first")
    ap.add_argument("--workload", default="L16384", choices=sorted(workloads()))
    ap.add_argument("--tile-rows", type=int, default=0)
    ap.add_argument("--update-only", action="store_true", help="no measurement (Table 1 'update only')")
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--copy-calibration", action="store_true",
                    help="also run a 1 GiB device copy (reference for HBM byte counters)")
    ap.add_argument("--batched", type=int, default=20, metavar="SWEEPS",
                    help="time 256 uneven replicas batched vs one after another for SWEEPS sweeps (0: skip)")
    ap.add_argument("--huge", type=int, default=10, metavar="SWEEPS",
                    help="time SWEEPS sweeps of the L = 65536 lattices, q = 2 and 3 (0: skip)")
    ap.add_argument("--small", type=int, default=1000, metavar="SWEEPS",
                    help="time SWEEPS sweeps of the L = 64 lattice (0: skip)")
    ap.add_argument("--xy", type=int, default=50, metavar="SWEEPS",
                    help="time SWEEPS sweeps of the L = 16384 XY lattice (0: skip)")
    ap.add_argument("--serve", type=int, default=0, metavar="JOBS",
                    help="also run the server on JOBS Poisson jobs at 0.5, 0.9 and 1.2 x capacity")
    ap.add_argument("--label-equivalence", type=int, default=0, metavar="SWEEPS",
                    help="also label the bonds of SWEEPS further sweeps with the paper's iterated label "
                         "equivalence (a comparison) and report its passes and time")
    args = ap.parse_args()

    if args.gpus != 1 or int(os.environ.get("WORLD_SIZE", "1")) != 1:
        print("bench.py measures one GPU only: this build has no multi-GPU path "
              "(the sweep of one lattice runs on one MI355X); use --gpus 1", file=sys.stderr)
        sys.exit(2)

    import torch
    from paper_1208_2080_amd import binding

    cfg = workloads()[args.workload]
    L, q, K = cfg["L"], cfg["q"], cfg["K"]
    N = L * L
    torch.cuda.set_device(0)
    if args.copy_calibration:
        copy_calibration()
    lat = binding.Lattice(L, q, K, seed=cfg["seed"], random_start=cfg["random_start"],
                          obs_capacity=0 if args.update_only else 1024, tile_rows=args.tile_rows)
    print(f"# {args.workload}: L={L} q={q} K={K:.12f} ({N} sites), warmup {args.warmup}", file=sys.stderr,
          flush=True)
    lat.sweep(args.warmup)
    torch.cuda.synchronize()

    # timed region: exactly `steps` sweeps, HIP events around every kernel
    phases = [0.0, 0.0, 0.0, 0.0]
    chunk = 5000
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    done = 0
    while done < args.steps:
        n = min(chunk, args.steps - done)
        ph = lat.sweep_profiled(n)
        phases = [a + b for a, b in zip(phases, ph)]
        done += n
    torch.cuda.synchronize()
    wall = time.perf_counter() - t0
    print(f"# timed {args.steps} sweeps in {wall:.3f} s", file=sys.stderr, flush=True)

    if not args.update_only:
        obs = lat.measure(lat.sweeps_done - 1, 1)[0]
        assert obs[2:].sum() == N, "observable counts do not sum to N"

    value = N * args.steps / (wall * 1e9)
    per_launch_ms = {PHASE_KERNELS[i]: phases[i] / args.steps for i in range(3)}
    dominant = max(("k_bond_label", "k_flip"), key=lambda k: per_launch_ms[k])
    ty = args.tile_rows or 64
    alg_bytes = KERNEL_BYTES_PER_SITE[dominant] * N
    achieved = alg_bytes / (per_launch_ms[dominant] * 1e-3) / 1e9
    traffic = measured_traffic(dominant, args.workload, ty)
    out = {
        "metric": "spin flips/ns on 1 MI355X, q=2 at K_c, L=16384/65536; batched vs plain",
        "value": value,
        "unit": "spin flips/ns",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": wall * 1e3 / args.steps,
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "u32",   # 32-bit integer arithmetic (draws, thresholds, labels); spins stored as u8
        "data": "synthetic",
        "config": {"workload": f"SW sweep, 2D Potts L={L} q={q} K={K:.9f} periodic, "
                               f"{'random' if cfg['random_start'] else 'cold'} start, "
                               f"{'update only' if args.update_only else 'update + measurement'}",
                   "L": L, "q": q, "K": K, "seed": cfg["seed"], "tile_rows": ty},
        "roofline": {"bound": "hbm", "kernel": dominant, "achieved": achieved, "peak": HBM_PEAK_GBS,
                     "unit": "GB/s", "frac": achieved / HBM_PEAK_GBS,
                     "traffic": traffic,
                     "alg_bytes_per_launch": alg_bytes,
                     "avg_launch_ms": per_launch_ms[dominant]},
        "phase_ms_per_sweep": {k: v for k, v in per_launch_ms.items()},
        "sweep_roofline_frac": value * SWEEP_BYTES_PER_SITE / HBM_PEAK_GBS,
    }
    if args.label_equivalence:
        print("# iterated label equivalence on the same bonds", file=sys.stderr, flush=True)
        out["label_equivalence"] = label_equivalence(lat, args.label_equivalence, per_launch_ms)
    lat.close()
    del lat
    torch.cuda.empty_cache()
    if not args.update_only:
        # Table 1's other column: the same sweeps with the measurement off
        lat = binding.Lattice(L, q, K, seed=cfg["seed"], random_start=cfg["random_start"], obs_capacity=0,
                              tile_rows=args.tile_rows)
        lat.sweep(args.warmup)
        torch.cuda.synchronize()
        n_uo = min(args.steps, 1000)
        t0 = time.perf_counter()
        lat.sweep(n_uo)
        torch.cuda.synchronize()
        out["update_only_flips_per_ns"] = N * n_uo / ((time.perf_counter() - t0) * 1e9)
        lat.close()
        del lat
        torch.cuda.empty_cache()
    if args.huge:
        out["L65536"] = huge_lattices(2, args.huge)
    if args.small:
        out["L64"] = small_lattice(args.small)
        out["small_lattice_batches"] = small_mixes(1000)
    if args.xy:
        out["xy_L16384"] = xy_lattice(5, args.xy, not args.no_cpu_baseline)
    if args.serve:
        out["serving"] = serving(args.serve, value, args.tile_rows)
    if args.batched:
        print("# batched vs plain", file=sys.stderr, flush=True)
        out["batched_vs_plain"] = batched_vs_plain(256, args.batched, args.tile_rows)
    out["copy_ceiling"] = copy_ceiling()
    if not args.no_cpu_baseline:
        print("# timing the CPU oracle on one sweep", file=sys.stderr, flush=True)
        out["cpu_baseline"] = cpu_baseline(cfg)
        if args.batched:
            print("# timing the CPU oracle on the batched mix, all cores", file=sys.stderr, flush=True)
            out["cpu_baseline_batched"] = cpu_baseline_batched(256, 1)
    else:
        out["cpu_baseline"] = None
    print(json.dumps(out), flush=True)


if __name__ == "__main__":
    main()
