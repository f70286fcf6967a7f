"""CPU oracle for the Swendsen-Wang sweep of the 2D q-state Potts model and of
the classical XY model with Wolff's embedded clusters.

TEST INFRASTRUCTURE ONLY.  Only the test suite, ``__graft_entry__.smoke()`` and
the ``cpu_baseline`` leg of ``bench.py`` may import this package.  The library
under ``paper_1208_2080_amd`` never touches it, and it shares no code with the
HIP path.

The arithmetic lives in ``sw_oracle.c`` (plain C, one thread); this module only
compiles it with gcc and marshals arguments.  It follows the paper's three SW
steps (Sec. 2): bond activation, Hoshen-Kopelman cluster labelling with the
smallest label as the proper label, and a random new state per cluster, with
the energy of Eq. (1) counted as the number of unsatisfied bonds.  The XY
sweep (``xy_oracle.c``, the extension of Sec. 5) reuses the same labelling and
random-number generator with its own streams.
"""
from __future__ import annotations

import ctypes
import os
import subprocess

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
_SRCS = [os.path.join(_HERE, f) for f in ("sw_oracle.c", "xy_oracle.c")]
_LIB = os.path.join(_HERE, "liboracle.so")

_lib = None


def _stale() -> bool:
    if not os.path.exists(_LIB):
        return True
    t = os.path.getmtime(_LIB)
    return any(os.path.getmtime(f) > t for f in _SRCS + [f[:-2] + ".h" for f in _SRCS])


def build(force: bool = True) -> str:
    """Compile the oracle with gcc into ``oracle/liboracle.so``."""
    if force or _stale():
        tmp = _LIB + ".tmp%d" % os.getpid()
        subprocess.check_call(["gcc", "-O2", "-std=c11", "-fPIC", "-shared", "-o", tmp, *_SRCS, "-lm"])
        os.replace(tmp, _LIB)
    return _LIB


def lib():
    global _lib
    if _lib is None:
        # SW_ORACLE_LIB: another build of these sources to load instead (the
        # test that plants mistakes in a copy of the oracle runs the pins on it)
        path = os.environ.get("SW_ORACLE_LIB")
        if not path:
            if _stale():
                build(force=True)
            path = _LIB
        L = ctypes.CDLL(path)
        u8p = ctypes.POINTER(ctypes.c_uint8)
        u32p = ctypes.POINTER(ctypes.c_uint32)
        i64p = ctypes.POINTER(ctypes.c_int64)
        L.or_philox.argtypes = [u32p, u32p, u32p]
        L.or_philox.restype = None
        L.or_threshold.argtypes = [ctypes.c_double]
        L.or_threshold.restype = ctypes.c_uint64
        L.or_state_of_draw.argtypes = [ctypes.c_uint32, ctypes.c_uint32]
        L.or_state_of_draw.restype = ctypes.c_uint32
        L.or_newspin.argtypes = [ctypes.c_uint64, ctypes.c_uint32, ctypes.c_uint64, ctypes.c_uint32]
        L.or_newspin.restype = ctypes.c_uint32
        L.or_initspin.argtypes = [ctypes.c_uint64, ctypes.c_uint64, ctypes.c_uint32]
        L.or_initspin.restype = ctypes.c_uint32
        L.or_bond_draws.argtypes = [ctypes.c_uint64, ctypes.c_uint32, ctypes.c_uint64, u32p, u32p]
        L.or_bond_draws.restype = None
        L.or_init.argtypes = [ctypes.c_uint32, ctypes.c_uint32, ctypes.c_uint64, ctypes.c_int, u8p]
        L.or_init.restype = ctypes.c_int
        L.or_observe.argtypes = [ctypes.c_uint32, ctypes.c_uint32, u8p, i64p]
        L.or_observe.restype = None
        L.or_derived.argtypes = [ctypes.c_uint32, ctypes.c_uint32, u8p, ctypes.POINTER(ctypes.c_double)]
        L.or_derived.restype = None
        L.or_label.argtypes = [ctypes.c_uint32, u8p, u8p, u32p]
        L.or_label.restype = None
        L.or_sweep.argtypes = [ctypes.c_uint32, ctypes.c_uint32, ctypes.c_double, ctypes.c_uint64,
                               ctypes.c_uint32, u8p, u8p, u8p, u32p, i64p]
        L.or_sweep.restype = ctypes.c_int
        L.or_bonds.argtypes = [ctypes.c_uint32, ctypes.c_double, ctypes.c_uint64, ctypes.c_uint32, u8p, u8p, u8p]
        L.or_bonds.restype = ctypes.c_int
        L.or_flip.argtypes = [ctypes.c_uint32, ctypes.c_uint32, ctypes.c_uint64, ctypes.c_uint32, u8p, u8p, u8p,
                              u32p, i64p]
        L.or_flip.restype = ctypes.c_int
        L.or_run.argtypes = [ctypes.c_uint32, ctypes.c_uint32, ctypes.c_double, ctypes.c_uint64,
                             ctypes.c_uint32, ctypes.c_uint32, u8p, i64p]
        L.or_run.restype = ctypes.c_int
        u64, u32, dbl = ctypes.c_uint64, ctypes.c_uint32, ctypes.c_double
        for name, res, args in [
            ("or_xy_direction", u32, [u64, u32, u32]),
            ("or_xy_initangle", u32, [u64, u64]),
            ("or_xy_uniform", dbl, [u64, u32, u64, u32]),
            ("or_xy_flipbit", u32, [u64, u32, u64]),
            ("or_xy_sincos", None, [u32, ctypes.POINTER(dbl), ctypes.POINTER(dbl)]),
            ("or_xy_projection", dbl, [u32, u32]),
            ("or_xy_reflect", u32, [u32, u32]),
            ("or_xy_init", ctypes.c_int, [u32, u64, ctypes.c_int, u32p]),
            ("or_xy_observe", None, [u32, u32p, i64p]),
            ("or_xy_derived", None, [u32, dbl, u32p, ctypes.POINTER(dbl)]),
            ("or_xy_bonds", ctypes.c_int, [u32, dbl, u64, u32, u32, u32p, u8p, u8p]),
            ("or_xy_flip", ctypes.c_int, [u32, u64, u32, u32, u32p, u8p, u8p, u32p, i64p]),
            ("or_xy_sweep", ctypes.c_int, [u32, dbl, u64, u32, u32, u32p, u8p, u8p, u32p, i64p]),
            ("or_xy_run", ctypes.c_int, [u32, dbl, u64, u32, u32, u32, u32p, i64p]),
        ]:
            f = getattr(L, name)
            f.argtypes = args
            f.restype = res
        _lib = L
    return _lib


def _p(a: np.ndarray, ct):
    assert a.flags["C_CONTIGUOUS"]
    return a.ctypes.data_as(ctypes.POINTER(ct))


def philox(ctr, key) -> np.ndarray:
    """Philox4x32-10 of one 128-bit counter under one 64-bit key."""
    c = np.asarray(ctr, dtype=np.uint32).copy()
    k = np.asarray(key, dtype=np.uint32).copy()
    out = np.zeros(4, dtype=np.uint32)
    lib().or_philox(_p(c, ctypes.c_uint32), _p(k, ctypes.c_uint32), _p(out, ctypes.c_uint32))
    return out


def threshold(K: float) -> int:
    """floor(2^32 (1 - e^{-K})); 2^32 for K = inf; -1 for invalid K."""
    t = lib().or_threshold(float(K))
    return -1 if t == 2**64 - 1 else int(t)


def state_of_draw(w: int, q: int) -> int:
    return int(lib().or_state_of_draw(w, q))


def newspin(seed: int, sweep: int, root: int, q: int) -> int:
    return int(lib().or_newspin(seed, sweep, root, q))


def initspin(seed: int, site: int, q: int) -> int:
    return int(lib().or_initspin(seed, site, q))


def bond_draws(seed: int, sweep: int, site: int):
    wx = ctypes.c_uint32()
    wy = ctypes.c_uint32()
    lib().or_bond_draws(seed, sweep, site, ctypes.byref(wx), ctypes.byref(wy))
    return int(wx.value), int(wy.value)


def init_spins(L: int, q: int, seed: int, random_start: bool) -> np.ndarray:
    s = np.zeros(L * L, dtype=np.uint8)
    rc = lib().or_init(L, q, seed, 1 if random_start else 0, _p(s, ctypes.c_uint8))
    if rc != 0:
        raise ValueError("oracle init rejected its parameters")
    return s.reshape(L, L)


def observe(s: np.ndarray, q: int) -> np.ndarray:
    """[n_unsat, 0, n_0..n_{q-1}] of a configuration (n_active is not defined here)."""
    s = np.ascontiguousarray(s, dtype=np.uint8)
    L = s.shape[0]
    obs = np.zeros(2 + q, dtype=np.int64)
    lib().or_observe(L, q, _p(s.reshape(-1), ctypes.c_uint8), _p(obs, ctypes.c_int64))
    return obs


def derived(s: np.ndarray, q: int) -> dict:
    """Energy per site e, Potts order parameter m and (q = 2) magnetisation M of
    a configuration, in FP64 straight from the spins."""
    s = np.ascontiguousarray(s, dtype=np.uint8)
    L = s.shape[0]
    out = np.zeros(3, dtype=np.float64)
    lib().or_derived(L, q, _p(s.reshape(-1), ctypes.c_uint8), _p(out, ctypes.c_double))
    d = {"e": float(out[0]), "m": float(out[1])}
    if q == 2:
        d["M"] = float(out[2])
    return d


def cluster_sums(labels: np.ndarray):
    """(S2, S4) = (sum over clusters of |C|^2, of |C|^4) as exact Python ints,
    from cluster labels (each site's cluster root): the cluster sizes that the
    improved estimators of the moments of the magnetisation use (the moment
    ratio of Sec. 4)."""
    sizes = np.bincount(np.asarray(labels, dtype=np.int64).reshape(-1))
    sizes = [int(c) for c in sizes if c]
    return sum(c * c for c in sizes), sum(c ** 4 for c in sizes)


def label(bx: np.ndarray, by: np.ndarray) -> np.ndarray:
    """Minimum-site-index cluster labels of the graph of active bonds."""
    L = bx.shape[0]
    bx = np.ascontiguousarray(bx, dtype=np.uint8).reshape(-1)
    by = np.ascontiguousarray(by, dtype=np.uint8).reshape(-1)
    lab = np.zeros(L * L, dtype=np.uint32)
    lib().or_label(L, _p(bx, ctypes.c_uint8), _p(by, ctypes.c_uint8), _p(lab, ctypes.c_uint32))
    return lab.reshape(L, L)


class OracleLattice:
    """One L x L lattice stepped by the oracle, one sweep at a time.

    ``sweep()`` returns the sweep's bonds (uint8 [L, L] per direction), labels
    (uint32 [L, L]) and observables [n_unsat, n_active, n_0..n_{q-1}] of the
    configuration after the flip; ``self.s`` holds the spins.
    """

    def __init__(self, L: int, q: int, K: float, seed: int, random_start: bool = True,
                 spins: np.ndarray | None = None, sweep: int = 0):
        self.L, self.q, self.K, self.seed = int(L), int(q), float(K), int(seed)
        if spins is None:
            self.s = init_spins(self.L, self.q, self.seed, random_start)
        else:
            self.s = np.ascontiguousarray(spins, dtype=np.uint8).reshape(self.L, self.L).copy()
        self.t = int(sweep)
        n = self.L * self.L
        self.bx = np.zeros(n, dtype=np.uint8)
        self.by = np.zeros(n, dtype=np.uint8)
        self.lab = np.zeros(n, dtype=np.uint32)

    def sweep(self) -> dict:
        obs = np.zeros(2 + self.q, dtype=np.int64)
        flat = self.s.reshape(-1)
        rc = lib().or_sweep(self.L, self.q, self.K, self.seed, self.t, _p(flat, ctypes.c_uint8),
                            _p(self.bx, ctypes.c_uint8), _p(self.by, ctypes.c_uint8),
                            _p(self.lab, ctypes.c_uint32), _p(obs, ctypes.c_int64))
        if rc != 0:
            raise ValueError("oracle sweep rejected its parameters")
        self.t += 1
        L = self.L
        return {"bx": self.bx.reshape(L, L).copy(), "by": self.by.reshape(L, L).copy(),
                "labels": self.lab.reshape(L, L).copy(), "obs": obs}

    def sweep_steps(self, progress=None) -> np.ndarray:
        """One sweep as its three steps of Sec. 2, each a call of its own
        (progress(name) after each, for long runs); returns the observables."""
        obs = np.zeros(2 + self.q, dtype=np.int64)
        flat = self.s.reshape(-1)
        if lib().or_bonds(self.L, self.K, self.seed, self.t, _p(flat, ctypes.c_uint8), _p(self.bx, ctypes.c_uint8),
                          _p(self.by, ctypes.c_uint8)) != 0:
            raise ValueError("oracle bonds rejected its parameters")
        if progress:
            progress("bonds")
        lib().or_label(self.L, _p(self.bx, ctypes.c_uint8), _p(self.by, ctypes.c_uint8), _p(self.lab, ctypes.c_uint32))
        if progress:
            progress("labels")
        if lib().or_flip(self.L, self.q, self.seed, self.t, _p(flat, ctypes.c_uint8), _p(self.bx, ctypes.c_uint8),
                         _p(self.by, ctypes.c_uint8), _p(self.lab, ctypes.c_uint32), _p(obs, ctypes.c_int64)) != 0:
            raise ValueError("oracle flip rejected its parameters")
        if progress:
            progress("flip")
        self.t += 1
        return obs

    def run(self, n: int) -> np.ndarray:
        """n sweeps; returns the int64 observable rows [n, 2+q]."""
        obs = np.zeros((n, 2 + self.q), dtype=np.int64)
        flat = self.s.reshape(-1)
        rc = lib().or_run(self.L, self.q, self.K, self.seed, self.t, n, _p(flat, ctypes.c_uint8),
                          _p(obs.reshape(-1), ctypes.c_int64))
        if rc != 0:
            raise ValueError("oracle run failed")
        self.t += n
        return obs


def pack_bonds(b: np.ndarray) -> np.ndarray:
    """Pack a uint8 [L, L] bond plane into uint64 words, ceil(L/64) per row,
    bit (x mod 64) of word x // 64 holding the bond of site x (padding bits 0)."""
    L = b.shape[0]
    W = (L + 63) // 64
    padded = np.zeros((L, W * 64), dtype=np.uint8)
    padded[:, :L] = b
    bits = np.packbits(padded.reshape(L, W, 64), axis=-1, bitorder="little")  # [L, W, 8]
    return bits.reshape(L, W * 8).view(np.uint64).reshape(L, W)


# ------------------------------------------------------------------ XY model
# The Swendsen-Wang sweep of the classical XY model with Wolff's embedded
# clusters (the extension of Sec. 5); the arithmetic is in ``xy_oracle.c``,
# whose header states every convention.  Angles are uint32 turn fractions.

XY_OBS_WORDS = 7
XY_UNIT = 2.0 ** -30          # one unit of the fixed-point observable sums


def xy_direction(seed: int, sweep: int, dir_bits: int = 32) -> int:
    return int(lib().or_xy_direction(seed, sweep, dir_bits))


def xy_initangle(seed: int, site: int) -> int:
    return int(lib().or_xy_initangle(seed, site))


def xy_uniform(seed: int, sweep: int, site: int, direction: int) -> float:
    return float(lib().or_xy_uniform(seed, sweep, site, direction))


def xy_flipbit(seed: int, sweep: int, root: int) -> int:
    return int(lib().or_xy_flipbit(seed, sweep, root))


def xy_sincos(a: int):
    """(sin, cos) of the angle of a, by the oracle's exact quarter-turn reduction."""
    s, c = ctypes.c_double(), ctypes.c_double()
    lib().or_xy_sincos(a & 0xFFFFFFFF, ctypes.byref(s), ctypes.byref(c))
    return float(s.value), float(c.value)


def xy_projection(a: int, phi: int) -> float:
    return float(lib().or_xy_projection(a & 0xFFFFFFFF, phi & 0xFFFFFFFF))


def xy_reflect(a: int, phi: int) -> int:
    return int(lib().or_xy_reflect(a & 0xFFFFFFFF, phi & 0xFFFFFFFF))


def xy_init_angles(L: int, seed: int, random_start: bool) -> np.ndarray:
    a = np.zeros(L * L, dtype=np.uint32)
    if lib().or_xy_init(L, seed, 1 if random_start else 0, _p(a, ctypes.c_uint32)) != 0:
        raise ValueError("oracle init rejected its parameters")
    return a.reshape(L, L)


def xy_observe(a: np.ndarray) -> np.ndarray:
    """[0, Ex, Ey, Ix, Iy, Mx, My] of a configuration in units of 2^-30."""
    a = np.ascontiguousarray(a, dtype=np.uint32)
    obs = np.zeros(XY_OBS_WORDS, dtype=np.int64)
    lib().or_xy_observe(a.shape[0], _p(a.reshape(-1), ctypes.c_uint32), _p(obs, ctypes.c_int64))
    return obs


def xy_derived(a: np.ndarray, K: float) -> dict:
    """Energy per site e, squared magnetisation per site m2 and the helicity
    estimator Y of one configuration, in FP64 straight from the angles."""
    a = np.ascontiguousarray(a, dtype=np.uint32)
    out = np.zeros(3, dtype=np.float64)
    lib().or_xy_derived(a.shape[0], float(K), _p(a.reshape(-1), ctypes.c_uint32), _p(out, ctypes.c_double))
    return {"e": float(out[0]), "m2": float(out[1]), "Y": float(out[2])}


class XYOracleLattice:
    """One L x L XY lattice stepped by the oracle.

    ``sweep()`` returns the sweep's direction ``phi``, bonds, labels and the
    observable row [n_active, Ex, Ey, Ix, Iy, Mx, My] of the configuration
    after the reflections; ``self.a`` holds the angles (uint32 [L, L]).
    """

    def __init__(self, L: int, K: float, seed: int, random_start: bool = True, dir_bits: int = 32,
                 angles: np.ndarray | None = None, sweep: int = 0):
        self.L, self.K, self.seed, self.dir_bits = int(L), float(K), int(seed), int(dir_bits)
        if angles is None:
            self.a = xy_init_angles(self.L, self.seed, random_start)
        else:
            self.a = np.ascontiguousarray(angles, dtype=np.uint32).reshape(self.L, self.L).copy()
        self.t = int(sweep)
        n = self.L * self.L
        self.bx = np.zeros(n, dtype=np.uint8)
        self.by = np.zeros(n, dtype=np.uint8)
        self.lab = np.zeros(n, dtype=np.uint32)

    def sweep(self) -> dict:
        obs = np.zeros(XY_OBS_WORDS, dtype=np.int64)
        phi = xy_direction(self.seed, self.t, self.dir_bits)
        rc = lib().or_xy_sweep(self.L, self.K, self.seed, self.t, self.dir_bits, _p(self.a.reshape(-1), ctypes.c_uint32),
                               _p(self.bx, ctypes.c_uint8), _p(self.by, ctypes.c_uint8),
                               _p(self.lab, ctypes.c_uint32), _p(obs, ctypes.c_int64))
        if rc != 0:
            raise ValueError("oracle sweep rejected its parameters")
        self.t += 1
        L = self.L
        return {"phi": phi, "bx": self.bx.reshape(L, L).copy(), "by": self.by.reshape(L, L).copy(),
                "labels": self.lab.reshape(L, L).copy(), "obs": obs}

    def sweep_steps(self, progress=None) -> np.ndarray:
        """One sweep as separate calls for its bonds, labels and reflections
        (progress(name) after each, for long runs); returns the observables."""
        obs = np.zeros(XY_OBS_WORDS, dtype=np.int64)
        flat = self.a.reshape(-1)
        if lib().or_xy_bonds(self.L, self.K, self.seed, self.t, self.dir_bits, _p(flat, ctypes.c_uint32),
                             _p(self.bx, ctypes.c_uint8), _p(self.by, ctypes.c_uint8)) != 0:
            raise ValueError("oracle bonds rejected its parameters")
        if progress:
            progress("bonds")
        lib().or_label(self.L, _p(self.bx, ctypes.c_uint8), _p(self.by, ctypes.c_uint8), _p(self.lab, ctypes.c_uint32))
        if progress:
            progress("labels")
        if lib().or_xy_flip(self.L, self.seed, self.t, self.dir_bits, _p(flat, ctypes.c_uint32),
                            _p(self.bx, ctypes.c_uint8), _p(self.by, ctypes.c_uint8), _p(self.lab, ctypes.c_uint32),
                            _p(obs, ctypes.c_int64)) != 0:
            raise ValueError("oracle flip rejected its parameters")
        if progress:
            progress("flip")
        self.t += 1
        return obs

    def run(self, n: int) -> np.ndarray:
        """n sweeps; returns the int64 observable rows [n, 7]."""
        obs = np.zeros((n, XY_OBS_WORDS), dtype=np.int64)
        rc = lib().or_xy_run(self.L, self.K, self.seed, self.t, n, self.dir_bits,
                             _p(self.a.reshape(-1), ctypes.c_uint32), _p(obs.reshape(-1), ctypes.c_int64))
        if rc != 0:
            raise ValueError("oracle run failed")
        self.t += n
        return obs
