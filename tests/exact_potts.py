"""Exact results for the q-state Potts model of Eq. (1) on small L x L tori.

These are the mathematical pins that the oracle is checked against; they do
not share code with the oracle or with the library.

* ``dos_transfer``: exact number of spin configurations with a given number of
  unsatisfied bonds (the energy of Eq. (1) in units of J), by a row transfer
  matrix whose entries are tracked as polynomials in the bond count.
* ``brute_force_dos``: the same by enumerating every configuration (tiny L).
* ``mean_unsat_transfer``: <n_unsat> at a given coupling K from the plain
  numeric transfer matrix, for sizes where the polynomial form is too big.
* ``kaufman_mean_unsat``: <n_unsat> of the q = 2 model on the L x L torus from
  Kaufman's (1949) exact partition function in the form used by Ferdinand and
  Fisher (1969), via the Potts/Ising mapping Z_P(K) = e^{-K N} Z_I(K / 2).

Bonds: every site has a bond to (x+1, y) and to (x, y+1), both periodic, so an
L x L torus has 2 L^2 bonds (for L = 2 two bonds join the same pair; both
count).
"""
from __future__ import annotations

import itertools

import mpmath
import numpy as np


def _rows(L: int, q: int) -> np.ndarray:
    """All q^L row configurations, shape [q^L, L]."""
    return np.array(list(itertools.product(range(q), repeat=L)), dtype=np.int64)


def _row_energies(L: int, q: int):
    rows = _rows(L, q)
    eh = (rows != np.roll(rows, -1, axis=1)).sum(axis=1)           # bonds inside a row
    ev = (rows[:, None, :] != rows[None, :, :]).sum(axis=2)         # bonds between two rows
    return rows, eh, ev


def dos_transfer(L: int, q: int) -> np.ndarray:
    """g[E] = number of configurations with E unsatisfied bonds, E = 0..2L^2.

    Counts are exact as long as q^(L^2) < 2^53 (float64 matmuls)."""
    if float(q) ** (L * L) >= 2.0 ** 53:
        raise ValueError("counts would not be exact in float64")
    _, eh, ev = _row_energies(L, q)
    S = eh.shape[0]
    D = 2 * L * L + 1
    step = ev + eh[None, :]               # energy added by entering row b from row a
    emax = int(step.max())
    mats = [(step == e).astype(np.float64) for e in range(emax + 1)]
    # V[r0, a, E]: first row r0, current row a, energy so far E
    V = np.zeros((S, S, D))
    V[np.arange(S), np.arange(S), eh] = 1.0
    for _ in range(L - 1):
        W = np.zeros_like(V)
        for e, M in enumerate(mats):
            if not M.any():
                continue
            # sum over a of V[r0, a, E] * M[a, b] -> [r0, E, b]
            t = np.tensordot(V, M, axes=([1], [0]))            # [r0, E, b]
            t = np.transpose(t, (0, 2, 1))                     # [r0, b, E]
            W[:, :, e:] += t[:, :, :D - e]
        V = W
    # close the torus: vertical bonds between the last row a and the first row r0
    g = np.zeros(D)
    for r0 in range(S):
        for e in range(L + 1):
            sel = ev[:, r0] == e
            if sel.any():
                g[e:] += V[r0, sel, :D - e].sum(axis=0)
    return np.rint(g)


def brute_force_dos(L: int, q: int) -> np.ndarray:
    """g[E] by enumerating all q^(L^2) configurations (only for tiny tori)."""
    n = L * L
    if q ** n > 5_000_000:
        raise ValueError("too many configurations")
    g = np.zeros(2 * n + 1, dtype=np.int64)
    chunk = 1 << 16
    total = q ** n
    for start in range(0, total, chunk):
        idx = np.arange(start, min(total, start + chunk), dtype=np.int64)
        digits = np.empty((idx.size, n), dtype=np.int64)
        rem = idx.copy()
        for k in range(n):
            digits[:, k] = rem % q
            rem //= q
        s = digits.reshape(-1, L, L)
        e = (s != np.roll(s, -1, axis=2)).sum(axis=(1, 2)) + (s != np.roll(s, -1, axis=1)).sum(axis=(1, 2))
        g += np.bincount(e, minlength=2 * n + 1)
    return g


def boltzmann(g: np.ndarray, K: float) -> np.ndarray:
    """P(E) proportional to g[E] exp(-K E)."""
    E = np.arange(g.size)
    logw = np.where(g > 0, np.log(np.maximum(g, 1)) - K * E, -np.inf)
    logw -= logw.max()
    w = np.exp(logw)
    return w / w.sum()


def mean_unsat_transfer(L: int, q: int, K: float) -> float:
    """<n_unsat> on the L x L torus from T[a, b] = exp(-K (ev(a, b) + eh(b)))."""
    _, eh, ev = _row_energies(L, q)
    step = (ev + eh[None, :]).astype(np.float64)
    T = np.exp(-K * step)
    TE = step * T
    P = np.linalg.matrix_power(T, L - 1)
    Z = np.trace(P @ T)
    return float(L * np.trace(P @ TE) / Z)


def _log_abs_and_sign(x):
    return mpmath.log(abs(x)), (1 if x >= 0 else -1)


def kaufman_log_z(L: int, K_ising) -> mpmath.mpf:
    """ln Z of the Ising model with coupling K_ising on an L x L torus."""
    K = mpmath.mpf(K_ising)
    m = n = L
    c2, s2 = mpmath.cosh(2 * K), mpmath.sinh(2 * K)

    def gamma(l):
        if l == 0:
            return 2 * K + mpmath.log(mpmath.tanh(K))      # signed
        return mpmath.acosh(c2 * c2 / s2 - mpmath.cos(mpmath.pi * l / n))

    odd = [gamma(2 * r + 1) for r in range(n)]
    even = [gamma(2 * r) for r in range(n)]
    terms = []
    for gs in (odd, even):
        pc = mpmath.mpf(1)
        ps = mpmath.mpf(1)
        for g in gs:
            pc *= 2 * mpmath.cosh(m * g / 2)
            ps *= 2 * mpmath.sinh(m * g / 2)
        terms += [pc, ps]
    total = mpmath.fsum(terms)
    return mpmath.log(total / 2) + (mpmath.mpf(m * n) / 2) * mpmath.log(2 * s2)


def kaufman_mean_unsat(L: int, K: float, dps: int = 60) -> float:
    """<n_unsat> of the q = 2 Potts model (coupling K) on the L x L torus."""
    with mpmath.workdps(dps):
        N = L * L
        d = mpmath.diff(lambda k: kaufman_log_z(L, k), mpmath.mpf(K) / 2)
        return float(N - d / 2)


def critical_coupling(q: int) -> float:
    """K_c(q) = ln(1 + sqrt(q)) of the square-lattice Potts model."""
    return float(np.log1p(np.sqrt(q)))
