"""Exact results for the classical XY model and the clock models it contains.

These are the mathematical pins for the XY oracle; they share no code with the
oracle or with the library.

* ``ring_correlation``: <cos(theta_0 - theta_r)> on a closed ring of n spins
  with nearest-neighbour coupling k, from the character expansion
  exp(k cos t) = sum_m I_m(k) e^{i m t}: the ring's partition function is
  (2 pi)^n sum_m I_m(k)^n and the correlation at distance r is
  sum_m I_m^(n-r) I_(m+1)^r / sum_m I_m^n (modified Bessel functions).
* The L = 2 torus: every site owns a bond to (x+1, y) and to (x, y+1), so the
  four spins form a ring in which each link carries two bonds (coupling 2K).
* ``clock_ring_correlation``: the same ring with the angle restricted to q
  equally spaced values, by an explicit q x q transfer matrix (the route the
  Bessel sums are cross-checked with: for large q they agree to rounding).
* ``clock_mean_cos_sum``: <sum over the 2 L^2 bonds of cos(theta_i - theta_j)>
  of the q-state clock model on the L x L torus (L >= 3), by a row transfer
  matrix over the q^L row configurations.
* The 2- and 4-state clock models are Ising models: q = 2 is Ising at K, and
  q = 4 is two independent Ising models at K / 2 (s_i . s_j =
  (sigma_i sigma_j + tau_i tau_j) / 2 after a 45-degree rotation), so
  Kaufman's torus result covers both (``ising_mean_bond_sum``).
"""
from __future__ import annotations

import itertools

import numpy as np
from scipy import special

import exact_potts as ep


def ring_correlation(n: int, k: float, r: int, mmax: int = 80) -> float:
    m = np.arange(-mmax, mmax + 1)
    i_m = special.ive(m, k)          # e^{-k} I_m(k): the common factor cancels
    i_m1 = special.ive(m + 1, k)
    return float(np.sum(i_m ** (n - r) * i_m1 ** r) / np.sum(i_m ** n))


def clock_ring_correlation(n: int, k: float, r: int, q: int) -> float:
    ang = 2 * np.pi * np.arange(q) / q
    T = np.exp(k * np.cos(ang[:, None] - ang[None, :]))
    C = np.cos(ang)
    S = np.sin(ang)
    Tr = np.linalg.matrix_power(T, r)
    Tn = np.linalg.matrix_power(T, n - r)
    z = np.trace(np.linalg.matrix_power(T, n))
    # <cos(t0 - tr)> = <cos t0 cos tr + sin t0 sin tr>
    num = np.trace(np.diag(C) @ Tr @ np.diag(C) @ Tn) + np.trace(np.diag(S) @ Tr @ np.diag(S) @ Tn)
    return float(num / z)


def xy_L2_bond_cos_sum(K: float) -> float:
    """<Ex + Ey> (sum of cos over the 8 bonds) of the continuous model on the 2 x 2 torus."""
    return 8.0 * ring_correlation(4, 2.0 * K, 1)


def xy_L2_m2(K: float) -> float:
    """<|sum_i s_i|^2> on the 2 x 2 torus: 4 + 2 (4 neighbour pairs + 2 diagonal pairs)."""
    return 4.0 + 8.0 * ring_correlation(4, 2.0 * K, 1) + 4.0 * ring_correlation(4, 2.0 * K, 2)


def clock_mean_cos_sum(L: int, q: int, K: float) -> float:
    if L < 3:
        raise ValueError("the row transfer matrix needs L >= 3 (L = 2 doubles bonds)")
    rows = np.array(list(itertools.product(range(q), repeat=L)), dtype=np.int64)
    ang = 2 * np.pi * rows / q
    h = np.cos(ang - np.roll(ang, -1, axis=1)).sum(axis=1)              # bonds within a row
    v = np.cos(ang[:, None, :] - ang[None, :, :]).sum(axis=2)            # bonds from a row to the next
    E = h[:, None] + v
    shift = K * E.max()                                                  # keep the entries in range
    T = np.exp(K * E - shift)
    TL1 = np.linalg.matrix_power(T, L - 1)
    z = np.trace(TL1 @ T)
    return float(L * np.sum(TL1.T * (E * T)) / z)


def ising_mean_bond_sum(L: int, K_ising: float) -> float:
    """<sum over the 2 L^2 bonds of sigma_i sigma_j> of the Ising model on the L x L
    torus (Kaufman, through the q = 2 Potts mapping: sum = 2N - 2 n_unsat at
    Potts coupling 2 K_ising)."""
    return 2.0 * L * L - 2.0 * ep.kaufman_mean_unsat(L, 2.0 * K_ising)
