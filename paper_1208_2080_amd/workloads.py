"""Seeded synthetic inputs shared by the tests, the smoke check and the benchmark.

This module holds no arithmetic of the method itself (no bonds, labels, random
draws of the sweep or observables): only parameter sets and seeded inputs with
the shapes and distributions of the paper's workloads (q = 2 at the critical
temperature on L x L periodic lattices, Sec. 4) and of the batched and served
forms.  Both the oracle side and the GPU side read their inputs from here.
"""
from __future__ import annotations

import math

import numpy as np


def critical_coupling(q: int) -> float:
    """Critical coupling K_c(q) = J / k_B T_c = ln(1 + sqrt(q)) of the square-lattice
    Potts model; for q = 2 this is T_c / J = 1.1346 as quoted in Sec. 4."""
    return math.log1p(math.sqrt(q))


# Correctness workload: 64 x 64, q = 2 at K_c, random start, 1000 sweeps.
SMALL = {"L": 64, "q": 2, "K": critical_coupling(2), "seed": 1, "random_start": True, "sweeps": 1000}
# Single-lattice throughput workloads (q = 2 at K_c, random start).
PLAIN_4096 = {"L": 4096, "q": 2, "K": critical_coupling(2), "seed": 1, "random_start": True, "sweeps": 10000}
PLAIN_16384 = {"L": 16384, "q": 2, "K": critical_coupling(2), "seed": 1, "random_start": True, "sweeps": 10000}
# One lattice of 2^32 sites, cold start, q = 2 and q = 3 at their K_c.
HUGE_Q2 = {"L": 65536, "q": 2, "K": critical_coupling(2), "seed": 1, "random_start": False, "sweeps": 200}
HUGE_Q3 = {"L": 65536, "q": 3, "K": critical_coupling(3), "seed": 1, "random_start": False, "sweeps": 200}


# The XY model with embedded clusters (the extension of Sec. 5): K near the
# Kosterlitz-Thouless coupling of the square lattice (T_KT / J ~ 0.893),
# random start; the oracle's CPU timing uses one sweep of the smaller lattice.
K_KT_XY = 1.0 / 0.893
XY_16384 = {"L": 16384, "K": K_KT_XY, "seed": 1, "random_start": True, "cpu_L": 4096}


def random_spins(L: int, q: int, seed: int) -> np.ndarray:
    """Uniform spins in 0..q-1, uint8 [L, L], from numpy's PCG64."""
    rng = np.random.Generator(np.random.PCG64(seed))
    return rng.integers(0, q, size=(L, L), dtype=np.uint8)


def random_bonds(L: int, density: float, seed: int):
    """Independent random bond masks (uint8 [L, L] for +x and +y)."""
    rng = np.random.Generator(np.random.PCG64(seed))
    bx = (rng.random((L, L)) < density).astype(np.uint8)
    by = (rng.random((L, L)) < density).astype(np.uint8)
    return bx, by


def checkerboard(L: int) -> np.ndarray:
    """q = 2 antiferromagnetic pattern (no equal-spin bond when L is even)."""
    y, x = np.indices((L, L))
    return ((x + y) & 1).astype(np.uint8)


def batched_replicas(n: int = 256, seed: int = 2012, Ls=(64, 128, 256, 512, 1024, 2048),
                     qs=(2, 3, 4, 8), sweeps: int = 1000):
    """Independent replicas of uneven L, q and K: L uniform over ``Ls``, q uniform
    over ``qs``, K = K_c(q) * U(0.9, 1.1), seed 1000 + r, random start."""
    rng = np.random.Generator(np.random.PCG64(seed))
    out = []
    for r in range(n):
        L = int(rng.choice(Ls))
        q = int(rng.choice(qs))
        K = critical_coupling(q) * float(rng.uniform(0.9, 1.1))
        out.append({"L": L, "q": q, "K": K, "seed": 1000 + r, "random_start": True, "sweeps": sweeps})
    return out


def serving_jobs(n: int = 2000, seed: int = 2013, L_min: int = 128, L_max: int = 8192,
                 q_min: int = 2, q_max: int = 10, sweeps_min: int = 100, sweeps_max: int = 5000,
                 rate_per_s: float = 1.0):
    """Poisson stream of simulation jobs: L = round(exp U(ln L_min, ln L_max)),
    q uniform on q_min..q_max, K = K_c(q) * U(0.95, 1.05), sweeps uniform on
    sweeps_min..sweeps_max, seed = job id, random start; arrival times from
    exponential gaps of mean 1 / rate_per_s."""
    rng = np.random.Generator(np.random.PCG64(seed))
    t = 0.0
    out = []
    for j in range(n):
        t += float(rng.exponential(1.0 / rate_per_s))
        L = int(round(math.exp(rng.uniform(math.log(L_min), math.log(L_max)))))
        q = int(rng.integers(q_min, q_max + 1))
        K = critical_coupling(q) * float(rng.uniform(0.95, 1.05))
        sw = int(rng.integers(sweeps_min, sweeps_max + 1))
        out.append({"id": j, "arrival": t, "L": L, "q": q, "K": K, "seed": j, "random_start": True,
                    "sweeps": sw})
    return out
