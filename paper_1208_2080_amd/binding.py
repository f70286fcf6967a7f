"""Python binding of the C ABI in ``include/sw.h`` and ``include/sw_xy.h``
(argument marshalling only).

Every step of a sweep runs in the HIP kernels of ``libswmi.so``; this module
only allocates the device workspace as a torch tensor, hands torch's HIP stream
to the library and copies results into numpy arrays.  There is no fallback: if
the library is missing or fails to load, every entry point raises.
"""
from __future__ import annotations

import ctypes
import os

import numpy as np
import torch

_HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(_HERE, "libswmi.so")

SW_OK, SW_EINVAL, SW_ESPACE, SW_EHIP, SW_ESTATE, SW_ECONVERGE = 0, -1, -2, -3, -4, -5


class SwError(RuntimeError):
    def __init__(self, code: int, msg: str):
        super().__init__(f"swmi error {code}: {msg}")
        self.code = code


class SwParams(ctypes.Structure):
    _fields_ = [("L", ctypes.c_uint32), ("q", ctypes.c_uint32), ("K", ctypes.c_double),
                ("seed", ctypes.c_uint64), ("init", ctypes.c_uint32), ("obs_capacity", ctypes.c_uint32),
                ("tile_rows", ctypes.c_uint32), ("flags", ctypes.c_uint32)]


SW_CLUSTER_SUMS = 1
SW_TILE_WHOLE = 1          # tile_rows: the whole lattice (L <= 128) in one workgroup's LDS
WHOLE_LMAX = 128


class SwXYParams(ctypes.Structure):
    _fields_ = [("L", ctypes.c_uint32), ("dir_bits", ctypes.c_uint32), ("K", ctypes.c_double),
                ("seed", ctypes.c_uint64), ("init", ctypes.c_uint32), ("obs_capacity", ctypes.c_uint32),
                ("tile_rows", ctypes.c_uint32), ("reserved", ctypes.c_uint32)]


SW_XY_OBS_WORDS = 7
XY_UNIT = 2.0 ** -30


# (name, restype, argtypes) of every function declared in include/sw.h and
# include/sw_xy.h
_VP = ctypes.c_void_p
_PP = ctypes.POINTER(SwParams)
_XP = ctypes.POINTER(SwXYParams)
_U32 = ctypes.c_uint32
SIGNATURES = [
    ("sw_workspace_bytes", ctypes.c_size_t, [_PP]),
    ("sw_threshold", ctypes.c_int, [_PP, ctypes.POINTER(ctypes.c_uint64)]),
    ("sw_init", ctypes.c_int, [_PP, _VP, ctypes.c_size_t, _VP, ctypes.POINTER(_VP)]),
    ("sw_sweep", ctypes.c_int, [_VP, _U32]),
    ("sw_measure", ctypes.c_int, [_VP, _U32, _U32, _VP]),
    ("sw_cluster_sums", ctypes.c_int, [_VP, _U32, _U32, _VP]),
    ("sw_measure_after", ctypes.c_int, [_VP, _VP, _VP, _U32, _U32, _VP]),
    ("sw_read_spins_after", ctypes.c_int, [_VP, _VP, _VP, _VP]),
    ("sw_sweep_profiled", ctypes.c_int, [_VP, _U32, ctypes.POINTER(ctypes.c_double)]),
    ("sw_sweeps_done", ctypes.c_int, [_VP, ctypes.POINTER(_U32)]),
    ("sw_read_spins", ctypes.c_int, [_VP, _VP]),
    ("sw_load_spins", ctypes.c_int, [_VP, _VP, _U32]),
    ("sw_read_labels", ctypes.c_int, [_VP, _VP]),
    ("sw_read_bonds", ctypes.c_int, [_VP, _VP]),
    ("sw_label_equivalence", ctypes.c_int, [_VP, _VP, _VP, _U32, ctypes.POINTER(_U32),
                                            ctypes.POINTER(ctypes.c_double)]),
    ("sw_destroy", ctypes.c_int, [_VP]),
    ("sw_batch_workspace_bytes", ctypes.c_int, [_PP, _U32, ctypes.POINTER(ctypes.c_size_t)]),
    ("sw_batch_init", ctypes.c_int, [_PP, _U32, _VP, ctypes.c_size_t, _VP, ctypes.POINTER(_VP)]),
    ("sw_batch_sweep", ctypes.c_int, [_VP, _VP]),
    ("sw_batch_sweep_all", ctypes.c_int, [_VP, _U32]),
    ("sw_batch_measure", ctypes.c_int, [_VP, _U32, _U32, _U32, _VP]),
    ("sw_batch_read_spins", ctypes.c_int, [_VP, _U32, _VP]),
    ("sw_batch_cluster_sums", ctypes.c_int, [_VP, _U32, _U32, _U32, _VP]),
    ("sw_batch_sweeps_done", ctypes.c_int, [_VP, _U32, ctypes.POINTER(_U32)]),
    ("sw_batch_destroy", ctypes.c_int, [_VP]),
    ("sw_batch_autotune", ctypes.c_int, [_PP, _U32, _VP, _U32, _U32, _VP, ctypes.c_size_t, _VP,
                                         ctypes.POINTER(_U32), ctypes.POINTER(ctypes.c_double)]),
    ("sw_tile_count", ctypes.c_int, [_PP, ctypes.POINTER(_U32)]),
    ("sw_group_workspace_bytes", ctypes.c_int, [_U32, ctypes.c_uint64, ctypes.POINTER(ctypes.c_size_t)]),
    ("sw_group_init", ctypes.c_int, [_U32, ctypes.c_uint64, _U32, _VP, ctypes.c_size_t, _VP, ctypes.POINTER(_VP)]),
    ("sw_group_sweep", ctypes.c_int, [_VP, _VP, _VP, _U32]),
    ("sw_group_destroy", ctypes.c_int, [_VP]),
    ("sw_derived", ctypes.c_int, [_U32, _U32, _VP, _VP]),
    ("sw_sweep_static", ctypes.c_int, [_PP, _VP, _U32, _U32, _VP, _VP, _VP]),
    ("sw_last_error", ctypes.c_char_p, []),
    ("sw_xy_workspace_bytes", ctypes.c_size_t, [_XP]),
    ("sw_xy_init", ctypes.c_int, [_XP, _VP, ctypes.c_size_t, _VP, ctypes.POINTER(_VP)]),
    ("sw_xy_read_angles", ctypes.c_int, [_VP, _VP]),
    ("sw_xy_load_angles", ctypes.c_int, [_VP, _VP, _U32]),
    ("sw_xy_derived", ctypes.c_int, [_U32, ctypes.c_double, _VP, _VP]),
]

_lib = None


def lib():
    """Load ``libswmi.so`` (after torch, so both share torch's HIP runtime)."""
    global _lib
    if _lib is None:
        if not os.path.exists(LIB_PATH):
            raise RuntimeError(f"{LIB_PATH} is missing: build it with paper_1208_2080_amd.build.build()")
        handle = ctypes.CDLL(LIB_PATH)
        for name, res, args in SIGNATURES:
            fn = getattr(handle, name)
            fn.restype = res
            fn.argtypes = args
        runtimes = set()
        with open("/proc/self/maps") as f:
            for line in f:
                if "libamdhip64" in line:
                    runtimes.add(os.path.realpath(line.split()[-1]))
        if len(runtimes) > 1:
            raise RuntimeError(f"two HIP runtimes are loaded ({sorted(runtimes)}); import torch first")
        _lib = handle
    return _lib


def _check(rc: int):
    if rc != SW_OK:
        raise SwError(rc, lib().sw_last_error().decode())


def make_params(L: int, q: int, K: float, seed: int = 1, random_start: bool = True,
                obs_capacity: int = 2, tile_rows: int = 0, cluster_sums: bool = False) -> SwParams:
    return SwParams(int(L), int(q), float(K), int(seed), 1 if random_start else 0, int(obs_capacity),
                    int(tile_rows), SW_CLUSTER_SUMS if cluster_sums else 0)


def _cluster_rows(raw: np.ndarray) -> np.ndarray:
    """[S2, S4 low, S4 high] uint64 rows -> object array of Python ints [S2, S4]."""
    out = np.empty((raw.shape[0], 2), dtype=object)
    for i, (s2, lo, hi) in enumerate(raw.tolist()):
        out[i, 0] = int(s2)
        out[i, 1] = (int(hi) << 64) | int(lo)
    return out


def threshold(K: float) -> int:
    thr = ctypes.c_uint64()
    _check(lib().sw_threshold(ctypes.byref(make_params(2, 2, K)), ctypes.byref(thr)))
    return int(thr.value)


def workspace_bytes(L: int, q: int, obs_capacity: int = 2, tile_rows: int = 0) -> int:
    p = make_params(L, q, 1.0, obs_capacity=obs_capacity, tile_rows=tile_rows)
    n = lib().sw_workspace_bytes(ctypes.byref(p))
    if n == 0:
        raise SwError(SW_EINVAL, lib().sw_last_error().decode())
    return int(n)


def _stream_handle(stream) -> int:
    return int(stream.cuda_stream)


_streams = {}


def default_stream(device):
    """The stream lattices and groups use when none is given: one per device,
    of default priority, shared so that groups can sweep any lattice made
    without an explicit stream.  (Not the legacy NULL stream, which the
    library cannot capture in HIP graphs.)"""
    device = torch.device(device)
    if device not in _streams:
        _streams[device] = torch.cuda.Stream(device)
    return _streams[device]


def derived(row: np.ndarray, L: int, q: int) -> dict:
    """Energy per site e, Potts order parameter m and (q = 2) magnetisation M
    from one int64 observable row [n_unsat, n_active, n_0, ..., n_{q-1}]
    (computed in FP64 by the library's sw_derived)."""
    r = np.ascontiguousarray(row, dtype=np.int64)
    assert r.size == 2 + q
    out = (ctypes.c_double * 3)()
    _check(lib().sw_derived(int(L), int(q), r.ctypes.data_as(ctypes.c_void_p), out))
    d = {"e": float(out[0]), "m": float(out[1])}
    if q == 2:
        d["M"] = float(out[2])
    return d


class Lattice:
    """One L x L lattice resident on the GPU, swept by the HIP kernels."""

    def __init__(self, L: int, q: int, K: float, seed: int = 1, random_start: bool = True,
                 obs_capacity: int = 1024, tile_rows: int = 0, device=None, stream=None, cluster_sums=False):
        self.L, self.q, self.K, self.seed = int(L), int(q), float(K), int(seed)
        self.obs_capacity = int(obs_capacity)
        self.params = make_params(L, q, K, seed, random_start, obs_capacity, tile_rows, cluster_sums)
        nbytes = lib().sw_workspace_bytes(ctypes.byref(self.params))
        if nbytes == 0:
            raise SwError(SW_EINVAL, lib().sw_last_error().decode())
        self.device = torch.device("cuda", 0) if device is None else torch.device(device)
        self.stream = stream if stream is not None else default_stream(self.device)
        self.ws = torch.empty(int(nbytes), dtype=torch.uint8, device=self.device)
        self.ws.record_stream(self.stream)                      # freed only after the stream's work
        torch.cuda.current_stream(self.device).synchronize()   # workspace allocated before first use
        self._h = ctypes.c_void_p()
        _check(lib().sw_init(ctypes.byref(self.params), ctypes.c_void_p(self.ws.data_ptr()), nbytes,
                             ctypes.c_void_p(_stream_handle(self.stream)), ctypes.byref(self._h)))

    @property
    def N(self) -> int:
        return self.L * self.L

    @property
    def W(self) -> int:
        return (self.L + 63) // 64

    def sweep(self, n: int = 1):
        _check(lib().sw_sweep(self._h, int(n)))

    def sweep_profiled(self, n: int) -> np.ndarray:
        """n sweeps with HIP events around every kernel; returns the summed device
        milliseconds of [bonds + tile labels, merge, flip, final measurement,
        the bond kernel alone (part of the first)]."""
        out = (ctypes.c_double * 5)()
        _check(lib().sw_sweep_profiled(self._h, int(n), out))
        return np.array(out[:], dtype=np.float64)

    @property
    def sweeps_done(self) -> int:
        v = ctypes.c_uint32()
        _check(lib().sw_sweeps_done(self._h, ctypes.byref(v)))
        return int(v.value)

    def measure(self, first: int, n: int) -> np.ndarray:
        out = np.zeros((n, 2 + self.q), dtype=np.int64)
        _check(lib().sw_measure(self._h, int(first), int(n), out.ctypes.data_as(ctypes.c_void_p)))
        return out

    def measure_after(self, read_stream, event, first: int, n: int) -> np.ndarray:
        """``measure`` on read_stream once ``event`` (a torch.cuda.Event recorded
        on this lattice's stream, or None) has passed; this lattice's stream
        may keep sweeping meanwhile."""
        out = np.zeros((n, 2 + self.q), dtype=np.int64)
        ev = ctypes.c_void_p(event.cuda_event) if event is not None else None
        _check(lib().sw_measure_after(self._h, ctypes.c_void_p(_stream_handle(read_stream)), ev, int(first), int(n),
                                      out.ctypes.data_as(ctypes.c_void_p)))
        return out

    def spins_after(self, read_stream, event) -> np.ndarray:
        out = np.empty((self.L, self.L), dtype=np.uint8)
        ev = ctypes.c_void_p(event.cuda_event) if event is not None else None
        _check(lib().sw_read_spins_after(self._h, ctypes.c_void_p(_stream_handle(read_stream)), ev,
                                         out.ctypes.data_as(ctypes.c_void_p)))
        return out

    def cluster_sums(self, first: int, n: int) -> np.ndarray:
        """[S2, S4] per sweep (Python ints): sums over the sweep's clusters of
        |C|^2 and |C|^4 (lattices made with cluster_sums=True)."""
        raw = np.zeros((n, 3), dtype=np.uint64)
        _check(lib().sw_cluster_sums(self._h, int(first), int(n), raw.ctypes.data_as(ctypes.c_void_p)))
        return _cluster_rows(raw)

    def spins(self) -> np.ndarray:
        out = np.empty((self.L, self.L), dtype=np.uint8)
        _check(lib().sw_read_spins(self._h, out.ctypes.data_as(ctypes.c_void_p)))
        return out

    def load_spins(self, s: np.ndarray, sweep: int):
        s = np.ascontiguousarray(s, dtype=np.uint8).reshape(self.L, self.L)
        _check(lib().sw_load_spins(self._h, s.ctypes.data_as(ctypes.c_void_p), int(sweep)))

    def labels(self) -> np.ndarray:
        out = np.empty((self.L, self.L), dtype=np.uint32)
        _check(lib().sw_read_labels(self._h, out.ctypes.data_as(ctypes.c_void_p)))
        return out

    def bonds(self):
        """(+x plane, +y plane), each uint64 [L, ceil(L/64)]."""
        out = np.empty((2, self.L, self.W), dtype=np.uint64)
        _check(lib().sw_read_bonds(self._h, out.ctypes.data_as(ctypes.c_void_p)))
        return out[0], out[1]

    def label_equivalence(self, max_iter: int = 1 << 16):
        """The paper's iterated label equivalence on the last sweep's bonds (a
        comparison; no sweep uses it): (labels uint32 [L, L], passes, device ms)."""
        labels = torch.empty(self.N, dtype=torch.int32, device=self.device)
        flag = torch.zeros(1, dtype=torch.int32, device=self.device)
        torch.cuda.current_stream(self.device).synchronize()   # buffers allocated before first use
        it = ctypes.c_uint32()
        ms = ctypes.c_double()
        _check(lib().sw_label_equivalence(self._h, ctypes.c_void_p(labels.data_ptr()), ctypes.c_void_p(flag.data_ptr()),
                                          int(max_iter), ctypes.byref(it), ctypes.byref(ms)))
        out = labels.cpu().numpy().view(np.uint32).reshape(self.L, self.L)
        return out, int(it.value), float(ms.value)

    def close(self, sync: bool = True):
        """Release the lattice.  Its workspace is only reused after the work
        queued on its stream, so sync=False may skip waiting for that stream
        (the lattice must not be in any sweep enqueued later)."""
        if self._h:
            if sync:
                self.stream.synchronize()
            lib().sw_destroy(self._h)
            self._h = ctypes.c_void_p()
        self.ws = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass


def make_xy_params(L: int, K: float, seed: int = 1, random_start: bool = True, obs_capacity: int = 1024,
                   tile_rows: int = 0, dir_bits: int = 32) -> SwXYParams:
    return SwXYParams(int(L), int(dir_bits), float(K), int(seed) & (2**64 - 1), 1 if random_start else 0,
                      int(obs_capacity), int(tile_rows), 0)


def xy_workspace_bytes(L: int, obs_capacity: int = 2, tile_rows: int = 0) -> int:
    p = make_xy_params(L, 1.0, 1, True, obs_capacity, tile_rows)
    n = lib().sw_xy_workspace_bytes(ctypes.byref(p))
    if n == 0:
        raise SwError(SW_EINVAL, lib().sw_last_error().decode())
    return int(n)


def xy_derived(row: np.ndarray, L: int, K: float) -> dict:
    """Energy per site e, squared magnetisation per site m2 and the helicity
    estimator Y from one XY observable row (FP64, by the library's
    sw_xy_derived)."""
    r = np.ascontiguousarray(row, dtype=np.int64)
    assert r.size == SW_XY_OBS_WORDS
    out = (ctypes.c_double * 3)()
    _check(lib().sw_xy_derived(int(L), float(K), r.ctypes.data_as(ctypes.c_void_p), out))
    return {"e": float(out[0]), "m2": float(out[1]), "Y": float(out[2])}


class XYLattice(Lattice):
    """One L x L classical XY lattice (uint32 angles) swept on the GPU with
    Wolff's embedded clusters; the sweep, labels, bonds, timing and release
    calls are those of ``Lattice``.  Observable rows are int64
    [n_active, Ex, Ey, Ix, Iy, Mx, My] (sums in units of 2^-30)."""

    def __init__(self, L: int, K: float, seed: int = 1, random_start: bool = True, obs_capacity: int = 1024,
                 tile_rows: int = 0, dir_bits: int = 32, device=None, stream=None):
        self.L, self.q, self.K, self.seed = int(L), 0, float(K), int(seed)
        self.dir_bits = int(dir_bits)
        self.obs_capacity = int(obs_capacity)
        self.params = make_xy_params(L, K, seed, random_start, obs_capacity, tile_rows, dir_bits)
        nbytes = lib().sw_xy_workspace_bytes(ctypes.byref(self.params))
        if nbytes == 0:
            raise SwError(SW_EINVAL, lib().sw_last_error().decode())
        self.device = torch.device("cuda", 0) if device is None else torch.device(device)
        self.stream = stream if stream is not None else default_stream(self.device)
        self.ws = torch.empty(int(nbytes), dtype=torch.uint8, device=self.device)
        self.ws.record_stream(self.stream)
        torch.cuda.current_stream(self.device).synchronize()
        self._h = ctypes.c_void_p()
        _check(lib().sw_xy_init(ctypes.byref(self.params), ctypes.c_void_p(self.ws.data_ptr()), nbytes,
                                ctypes.c_void_p(_stream_handle(self.stream)), ctypes.byref(self._h)))

    def measure(self, first: int, n: int) -> np.ndarray:
        out = np.zeros((n, SW_XY_OBS_WORDS), dtype=np.int64)
        _check(lib().sw_measure(self._h, int(first), int(n), out.ctypes.data_as(ctypes.c_void_p)))
        return out

    def measure_after(self, read_stream, event, first: int, n: int) -> np.ndarray:
        out = np.zeros((n, SW_XY_OBS_WORDS), dtype=np.int64)
        ev = ctypes.c_void_p(event.cuda_event) if event is not None else None
        _check(lib().sw_measure_after(self._h, ctypes.c_void_p(_stream_handle(read_stream)), ev, int(first), int(n),
                                      out.ctypes.data_as(ctypes.c_void_p)))
        return out

    def angles(self) -> np.ndarray:
        out = np.empty((self.L, self.L), dtype=np.uint32)
        _check(lib().sw_xy_read_angles(self._h, out.ctypes.data_as(ctypes.c_void_p)))
        return out

    def load_angles(self, a: np.ndarray, sweep: int):
        a = np.ascontiguousarray(a, dtype=np.uint32).reshape(self.L, self.L)
        _check(lib().sw_xy_load_angles(self._h, a.ctypes.data_as(ctypes.c_void_p), int(sweep)))


def _replica_params(replicas, obs_capacity: int, tile_rows: int):
    arr = (SwParams * len(replicas))()
    for i, r in enumerate(replicas):
        arr[i] = make_params(r["L"], r["q"], r["K"], r["seed"], r.get("random_start", True),
                             r.get("obs_capacity", obs_capacity), tile_rows, r.get("cluster_sums", False))
    return arr


def _batch_bytes(arr) -> int:
    nbytes = ctypes.c_size_t()
    _check(lib().sw_batch_workspace_bytes(arr, len(arr), ctypes.byref(nbytes)))
    return int(nbytes.value)


TILE_HEIGHTS = (32, 64, 128)


def tile_candidates(replicas):
    """The autotuner's default candidates: the default rule (0), the three tile
    heights, and SW_TILE_WHOLE when every replica can be swept whole."""
    whole = all(r["L"] <= WHOLE_LMAX and not r.get("cluster_sums", False) for r in replicas)
    return (0,) + TILE_HEIGHTS + ((SW_TILE_WHOLE,) if whole else ())


def autotune(replicas, obs_capacity: int = 64, candidates=None, sweeps: int = 8, device=None,
             stream=None):
    """Pick the fastest labelling tile height for this set of replicas (the
    library times each candidate); returns (height, {height: ms per sweep})."""
    replicas = [dict(r) for r in replicas]
    candidates = tile_candidates(replicas) if candidates is None else tuple(candidates)
    cands = (ctypes.c_uint32 * len(candidates))(*[int(c) for c in candidates])
    nbytes = max(_batch_bytes(_replica_params(replicas, obs_capacity, int(c))) for c in candidates)
    device = torch.device("cuda", 0) if device is None else torch.device(device)
    stream = stream if stream is not None else torch.cuda.Stream(device)
    ws = torch.empty(nbytes, dtype=torch.uint8, device=device)
    torch.cuda.current_stream(device).synchronize()   # workspace allocated before first use
    best = ctypes.c_uint32()
    ms = (ctypes.c_double * len(candidates))()
    _check(lib().sw_batch_autotune(_replica_params(replicas, obs_capacity, 0), len(replicas), cands,
                                   len(candidates), int(sweeps), ctypes.c_void_p(ws.data_ptr()), nbytes,
                                   ctypes.c_void_p(_stream_handle(stream)), ctypes.byref(best), ms))
    del ws
    return int(best.value), {int(c): float(ms[i]) for i, c in enumerate(candidates)}


class Batch:
    """Independent replicas of uneven L, q and K swept together, one launch per phase.
    tile_rows="auto" lets the library's autotuner pick the tile height first."""

    def __init__(self, replicas, obs_capacity: int = 64, tile_rows=0, device=None, stream=None):
        self.replicas = [dict(r) for r in replicas]
        n = len(self.replicas)
        self.device = torch.device("cuda", 0) if device is None else torch.device(device)
        # a stream of its own (default priority): HIP graphs cannot capture the NULL stream
        self.stream = stream if stream is not None else torch.cuda.Stream(self.device)
        self.tuned_ms = None
        if tile_rows == "auto":
            tile_rows, self.tuned_ms = autotune(self.replicas, obs_capacity, device=self.device, stream=self.stream)
        self.tile_rows = int(tile_rows)
        arr = _replica_params(self.replicas, obs_capacity, self.tile_rows)
        self.params = arr
        nbytes = ctypes.c_size_t(_batch_bytes(arr))
        self.ws = torch.empty(int(nbytes.value), dtype=torch.uint8, device=self.device)
        self.ws.record_stream(self.stream)                      # freed only after the stream's work
        torch.cuda.current_stream(self.device).synchronize()   # workspace allocated before first use
        self._h = ctypes.c_void_p()
        _check(lib().sw_batch_init(arr, n, ctypes.c_void_p(self.ws.data_ptr()), nbytes.value,
                                   ctypes.c_void_p(_stream_handle(self.stream)), ctypes.byref(self._h)))

    def __len__(self):
        return len(self.replicas)

    def sweep(self, n_each):
        v = np.ascontiguousarray(n_each, dtype=np.uint32)
        assert v.size == len(self)
        _check(lib().sw_batch_sweep(self._h, v.ctypes.data_as(ctypes.c_void_p)))

    def sweep_all(self, n: int):
        _check(lib().sw_batch_sweep_all(self._h, int(n)))

    def sweeps_done(self, r: int) -> int:
        v = ctypes.c_uint32()
        _check(lib().sw_batch_sweeps_done(self._h, int(r), ctypes.byref(v)))
        return int(v.value)

    def measure(self, r: int, first: int, n: int) -> np.ndarray:
        q = self.replicas[r]["q"]
        out = np.zeros((n, 2 + q), dtype=np.int64)
        _check(lib().sw_batch_measure(self._h, int(r), int(first), int(n), out.ctypes.data_as(ctypes.c_void_p)))
        return out

    def cluster_sums(self, r: int, first: int, n: int) -> np.ndarray:
        raw = np.zeros((n, 3), dtype=np.uint64)
        _check(lib().sw_batch_cluster_sums(self._h, int(r), int(first), int(n), raw.ctypes.data_as(ctypes.c_void_p)))
        return _cluster_rows(raw)

    def spins(self, r: int) -> np.ndarray:
        L = self.replicas[r]["L"]
        out = np.empty((L, L), dtype=np.uint8)
        _check(lib().sw_batch_read_spins(self._h, int(r), out.ctypes.data_as(ctypes.c_void_p)))
        return out

    def close(self):
        if self._h:
            self.stream.synchronize()
            lib().sw_batch_destroy(self._h)
            self._h = ctypes.c_void_p()
        self.ws = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass



def tile_count(L: int, q: int = 2, tile_rows: int = 0) -> int:
    v = ctypes.c_uint32()
    _check(lib().sw_tile_count(ctypes.byref(make_params(L, q, 1.0, tile_rows=tile_rows)), ctypes.byref(v)))
    return int(v.value)


class Group:
    """One launch per phase over any set of ``Lattice`` objects (continuous batching)."""

    def __init__(self, max_lattices: int, max_tiles: int, tile_rows: int = 0, device=None, stream=None):
        self.max_lattices, self.max_tiles = int(max_lattices), int(max_tiles)
        nbytes = ctypes.c_size_t()
        _check(lib().sw_group_workspace_bytes(self.max_lattices, self.max_tiles, ctypes.byref(nbytes)))
        self.device = torch.device("cuda", 0) if device is None else torch.device(device)
        self.stream = stream if stream is not None else default_stream(self.device)
        self.ws = torch.empty(int(nbytes.value), dtype=torch.uint8, device=self.device)
        self.ws.record_stream(self.stream)                      # freed only after the stream's work
        torch.cuda.current_stream(self.device).synchronize()   # workspace allocated before first use
        self._h = ctypes.c_void_p()
        _check(lib().sw_group_init(self.max_lattices, self.max_tiles, int(tile_rows),
                                   ctypes.c_void_p(self.ws.data_ptr()), nbytes.value,
                                   ctypes.c_void_p(_stream_handle(self.stream)), ctypes.byref(self._h)))

    def sweep(self, lattices, n_each):
        n = len(lattices)
        handles = (ctypes.c_void_p * max(1, n))(*[lat._h.value for lat in lattices])
        counts = np.ascontiguousarray(n_each, dtype=np.uint32)
        assert counts.size == n
        _check(lib().sw_group_sweep(self._h, handles, counts.ctypes.data_as(ctypes.c_void_p), n))

    def close(self):
        if self._h:
            self.stream.synchronize()
            lib().sw_group_destroy(self._h)
            self._h = ctypes.c_void_p()
        self.ws = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass
