"""Moment ratio of the magnetisation: the check of Sec. 4, where the code is
validated by the temperature dependence of the moment ratio of the
magnetisation, whose curves for different L cross at the critical point.

The order parameter of the q-state Potts model is taken as the vector
magnetisation M = sum_i e(s_i), with e(0..q-1) the q unit vectors pointing to
the corners of a regular simplex in q - 1 dimensions (e(a).e(b) = 1 for a = b,
-1/(q-1) otherwise); for q = 2 this is the Ising magnetisation.  Its square per
site follows exactly from the state counts n_c that every sweep measures:

    m^2 = |M|^2 / N^2 = (q sum_c n_c^2 - N^2) / ((q - 1) N^2)
        = sum_{c < c'} ((n_c - n_c') / N)^2 / (q - 1),

and the second form is a sum of non-negative terms (no cancellation in FP64
even at N = 2^32).  The moment ratio is U = <m^4> / <m^2>^2: 1 in the ordered
phase, 1 + 2/(q-1) for a disordered (Gaussian) order parameter, and
L-independent at K_c up to corrections, so curves U_L(K) for two sizes cross
near K_c.

``run`` sweeps one replica per (L, K) in one batch on the GPU; the analysis
functions are plain host arithmetic on the int64 observable rows.
"""
from __future__ import annotations

import argparse
import json
import sys
import time

import numpy as np


def m2_from_counts(counts: np.ndarray, q: int) -> np.ndarray:
    """m^2 per row from the state counts (rows of n_0..n_{q-1}), in FP64."""
    c = np.asarray(counts, dtype=np.int64).reshape(-1, q)
    N = c.sum(axis=1).astype(np.float64)
    acc = np.zeros(c.shape[0], dtype=np.float64)
    for a in range(q):
        for b in range(a + 1, q):
            d = (c[:, a] - c[:, b]).astype(np.float64) / N   # exact integer difference, one rounding
            acc += d * d
    return acc / (q - 1)


def improved_from_cluster_sums(cs_rows, N: int, q: int):
    """Improved estimators of m^2 and m^4 per sweep from the cluster-size sums
    [S2, S4] (exact integers) of the sweep's clusters: the means of |M|^2 / N^2
    and |M|^4 / N^4 over the clusters' independent uniform states,

        E|M|^2 = S2,   E|M|^4 = ((q + 1) S2^2 - 2 S4) / (q - 1),

    (simplex-vector magnetisation: e(a).e(b) = 1 if a = b, -1/(q-1) else, so
    cross terms of different clusters vanish on average and E (e(a).e(b))^2 =
    1/(q-1)).  The numerators are exact integers; each ratio is rounded once."""
    m2 = np.empty(len(cs_rows), dtype=np.float64)
    m4 = np.empty(len(cs_rows), dtype=np.float64)
    N2, N4 = N * N, N ** 4
    for i, (s2, s4) in enumerate(cs_rows):
        s2, s4 = int(s2), int(s4)
        m2[i] = s2 / N2
        m4[i] = ((q + 1) * s2 * s2 - 2 * s4) / ((q - 1) * N4)
    return m2, m4


def _jackknife(blocks_num: np.ndarray, blocks_den: np.ndarray):
    """Ratio <a> / <b>^2 and its jackknife error over equal blocks."""
    n = len(blocks_num)
    a, b = blocks_num.mean(), blocks_den.mean()
    value = a / (b * b)
    if n < 2:
        return value, float("nan")
    sa, sb = blocks_num.sum(), blocks_den.sum()
    loo = np.array([((sa - blocks_num[i]) / (n - 1)) / ((sb - blocks_den[i]) / (n - 1)) ** 2 for i in range(n)])
    err = float(np.sqrt((n - 1) / n * np.sum((loo - loo.mean()) ** 2)))
    return float(value), err


def moments(rows: np.ndarray, q: int, n_blocks: int = 20) -> dict:
    """<m^2>, <m^4> (standard errors of block means) and U = <m^4>/<m^2>^2
    (jackknife error), over n_blocks blocks of consecutive sweeps, from
    observable rows [n_unsat, n_active, n_0, ..., n_{q-1}]."""
    rows = np.asarray(rows, dtype=np.int64)
    m2 = m2_from_counts(rows[:, 2:2 + q], q)
    return _block_moments(m2, m2 * m2, n_blocks)


def improved_moments(cs_rows, N: int, q: int, n_blocks: int = 20) -> dict:
    """As ``moments`` with the cluster-size improved estimators (cs_rows: the
    [S2, S4] of each sweep)."""
    m2, m4 = improved_from_cluster_sums(cs_rows, N, q)
    return _block_moments(m2, m4, n_blocks)


def _block_moments(m2: np.ndarray, m4: np.ndarray, n_blocks: int) -> dict:
    nb = max(1, min(n_blocks, len(m2)))
    per = len(m2) // nb
    b2 = m2[:nb * per].reshape(nb, per).mean(axis=1)
    b4 = m4[:nb * per].reshape(nb, per).mean(axis=1)
    U, U_err = _jackknife(b4, b2)
    se = (lambda b: float(b.std(ddof=1) / np.sqrt(nb)) if nb > 1 else float("nan"))
    return {"m2": float(m2.mean()), "m2_err": se(b2), "m4": float(m4.mean()), "m4_err": se(b4),
            "U": U, "U_err": U_err, "samples": int(len(m2))}


def crossing(Ks, U_small, U_large):
    """Coupling where U of the larger lattice crosses U of the smaller one
    (linear interpolation between neighbouring grid points; None if the
    difference does not change sign).  Below K_c the larger lattice is more
    disordered (larger U), above it more ordered (smaller U)."""
    Ks = np.asarray(Ks, dtype=np.float64)
    d = np.asarray(U_large, dtype=np.float64) - np.asarray(U_small, dtype=np.float64)
    for i in range(len(Ks) - 1):
        if d[i] > 0 >= d[i + 1]:
            return float(Ks[i] + (Ks[i + 1] - Ks[i]) * d[i] / (d[i] - d[i + 1]))
    return None


def run(q: int, Ls, K_factors, sweeps: int, therm: int, chunk: int = 1000, seed0: int = 7000,
        tile_rows=0, device=None, improved: bool = True) -> dict:
    """Sweep one replica per (L, K = K_c(q) * factor) in one batch on the GPU
    (random start; `therm` sweeps discarded, then `sweeps` measured) and return
    U per replica and the crossings of successive sizes, from the state counts
    and (improved=True) also from the cluster-size improved estimators."""
    import torch
    from . import binding
    from . import workloads as wl

    Kc = wl.critical_coupling(q)
    grid = [(int(L), float(f)) for L in Ls for f in K_factors]
    reps = [{"L": L, "q": q, "K": Kc * f, "seed": seed0 + i, "random_start": True, "cluster_sums": improved}
            for i, (L, f) in enumerate(grid)]
    chunk = max(1, min(chunk, sweeps))
    b = binding.Batch(reps, obs_capacity=chunk + 1, tile_rows=tile_rows, device=device)
    if therm:
        b.sweep_all(therm)
    rows = [[] for _ in reps]
    cs = [[] for _ in reps]
    t0 = time.perf_counter()
    done = 0
    while done < sweeps:
        n = min(chunk, sweeps - done)
        b.sweep_all(n)
        for r in range(len(reps)):
            rows[r].append(b.measure(r, therm + done, n))
            if improved:
                cs[r].append(b.cluster_sums(r, therm + done, n))
        done += n
    torch.cuda.synchronize(b.device)
    wall = time.perf_counter() - t0
    flips = sum(L * L for L, _ in grid) * sweeps
    out = {"q": q, "K_c": Kc, "sweeps": sweeps, "therm": therm, "tile_rows": b.tile_rows,
           "wall_s": wall, "flips_per_ns": flips / (wall * 1e9), "points": []}
    b.close()
    U = {}
    for (L, f), rr, cc in zip(grid, rows, cs):
        mo = moments(np.concatenate(rr), q)
        if improved:
            imp = improved_moments(np.concatenate(cc), L * L, q)
            mo.update({k + "_impr": v for k, v in imp.items() if k != "samples"})
        U[(L, f)] = mo
        out["points"].append({"L": L, "K_over_Kc": f, **mo})
    Ls_sorted = sorted(set(L for L, _ in grid))
    fs = sorted(set(f for _, f in grid))
    out["crossings"] = []
    for La, Lb in zip(Ls_sorted, Ls_sorted[1:]):
        k = crossing(fs, [U[(La, f)]["U"] for f in fs], [U[(Lb, f)]["U"] for f in fs])
        c = {"L": [La, Lb], "K_over_Kc": k}
        if improved:
            c["K_over_Kc_impr"] = crossing(fs, [U[(La, f)]["U_impr"] for f in fs], [U[(Lb, f)]["U_impr"] for f in fs])
        out["crossings"].append(c)
    return out


def main(argv=None):
    ap = argparse.ArgumentParser(description="moment-ratio crossing of the q-state Potts model on the GPU")
    ap.add_argument("--q", type=int, nargs="+", default=[2, 3])
    ap.add_argument("--L", type=int, nargs="+", default=[32, 64, 128, 256])
    ap.add_argument("--k-factors", type=float, nargs="+",
                    default=[0.98, 0.985, 0.99, 0.995, 1.0, 1.005, 1.01, 1.015, 1.02])
    ap.add_argument("--sweeps", type=int, default=100000)
    ap.add_argument("--therm", type=int, default=2000)
    args = ap.parse_args(argv)
    for q in args.q:
        print(f"# q={q}: {len(args.L)} sizes x {len(args.k_factors)} couplings, {args.sweeps} sweeps",
              file=sys.stderr, flush=True)
        res = run(q, args.L, args.k_factors, args.sweeps, args.therm)
        print(json.dumps(res), flush=True)


if __name__ == "__main__":
    main()
