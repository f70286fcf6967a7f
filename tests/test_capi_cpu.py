"""The C-ABI library builds, loads without a GPU and exports every function that
include/*.h declares; host-side logic (parameter checks, workspace sizes, the
bond threshold) behaves as documented.  No kernel runs here."""
import ctypes
import math
import os
import re

import pytest

import oracle
from paper_1208_2080_amd import binding
from paper_1208_2080_amd import workloads as wl

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


def _declared_functions():
    inc = os.path.join(ROOT, "include")
    text = "".join(open(os.path.join(inc, f)).read() for f in sorted(os.listdir(inc)) if f.endswith(".h"))
    text = re.sub(r"/\*.*?\*/", "", text, flags=re.S)
    return sorted(set(re.findall(r"\b(sw_[a-z_]+)\s*\(", text)))


def test_library_exports_every_declared_symbol():
    lib = binding.lib()
    names = _declared_functions()
    assert len(names) >= 20
    for name in names:
        assert hasattr(lib, name), name
    # the binding marshals exactly the declared set
    assert sorted(n for n, _, _ in binding.SIGNATURES) == names


def test_threshold_matches_oracle():
    for K in [0.0, 0.1, 0.5, wl.critical_coupling(2), wl.critical_coupling(3), 2.0, 7.5, 40.0, float("inf")]:
        assert binding.threshold(K) == oracle.threshold(K)
    with pytest.raises(binding.SwError) as e:
        binding.threshold(-1.0)
    assert e.value.code == binding.SW_EINVAL
    with pytest.raises(binding.SwError):
        binding.threshold(float("nan"))


def _ws(L, q=2, cap=2, ty=0):
    p = binding.make_params(L, q, 1.0, obs_capacity=cap, tile_rows=ty)
    return binding.lib().sw_workspace_bytes(ctypes.byref(p))


def test_workspace_sizes():
    # spins + labels + bond planes + edge records + ring, each 256-byte aligned
    for L in [2, 64, 100, 4096, 16384]:
        n = _ws(L)
        assert n >= 5 * L * L + 2 * L * math.ceil(L / 64) * 8
        assert n % 256 == 0
    big = _ws(65536, 2, 1024)
    # ~5.25 B/site + tile edge records (0.13 B/site) + edge-forest nodes (0.5 B/site)
    assert 22.0 * 2**30 < big < 24.0 * 2**30
    assert _ws(1000, 2, 1000) > _ws(1000, 2, 2)


@pytest.mark.parametrize("L,q,K,cap,ty", [(1, 2, 1.0, 2, 0), (65537, 2, 1.0, 2, 0), (8, 1, 1.0, 2, 0),
                                          (8, 256, 1.0, 2, 0), (8, 2, -0.5, 2, 0), (8, 2, float("nan"), 2, 0),
                                          (8, 2, 1.0, 1, 0), (8, 2, 1.0, 2, 48)])
def test_invalid_params_rejected(L, q, K, cap, ty):
    p = binding.make_params(L, q, K, obs_capacity=cap, tile_rows=ty)
    assert binding.lib().sw_workspace_bytes(ctypes.byref(p)) == 0
    assert binding.lib().sw_last_error().decode() != ""


def test_flags_are_checked():
    p = binding.make_params(64, 2, 1.0, obs_capacity=4)
    p.flags = 2                                   # unknown flag
    assert binding.lib().sw_workspace_bytes(ctypes.byref(p)) == 0
    for L, cap in [(40000, 4), (64, 0)]:          # cluster sums: L <= 32768 and a ring
        p = binding.make_params(L, 2, 1.0, obs_capacity=cap, cluster_sums=True)
        assert binding.lib().sw_workspace_bytes(ctypes.byref(p)) == 0
    plain = binding.make_params(64, 2, 1.0, obs_capacity=4)
    sums = binding.make_params(64, 2, 1.0, obs_capacity=4, cluster_sums=True)
    # the cluster sums need one more word per edge-forest node
    assert binding.lib().sw_workspace_bytes(ctypes.byref(sums)) > binding.lib().sw_workspace_bytes(ctypes.byref(plain))


def test_init_rejects_bad_workspace_without_touching_the_gpu():
    lib = binding.lib()
    p = binding.make_params(16, 2, 1.0)
    h = ctypes.c_void_p()
    need = lib.sw_workspace_bytes(ctypes.byref(p))
    # NULL / misaligned / too small workspaces are refused before any HIP call
    assert lib.sw_init(ctypes.byref(p), None, need, None, ctypes.byref(h)) == binding.SW_ESPACE
    assert lib.sw_init(ctypes.byref(p), ctypes.c_void_p(0x1001), need, None, ctypes.byref(h)) == binding.SW_ESPACE
    assert lib.sw_init(ctypes.byref(p), ctypes.c_void_p(0x10000), need - 256, None,
                       ctypes.byref(h)) == binding.SW_ESPACE
    assert not h.value
    bad = binding.make_params(16, 2, -1.0)
    assert lib.sw_init(ctypes.byref(bad), ctypes.c_void_p(0x10000), need, None, ctypes.byref(h)) == binding.SW_EINVAL
    n = ctypes.c_size_t()
    arr = (binding.SwParams * 2)(binding.make_params(16, 2, 1.0, tile_rows=32), binding.make_params(16, 2, 1.0))
    assert lib.sw_batch_workspace_bytes(arr, 2, ctypes.byref(n)) == binding.SW_EINVAL   # mixed tile heights
    arr = (binding.SwParams * 2)(binding.make_params(16, 2, 1.0), binding.make_params(40, 3, 0.5))
    assert lib.sw_batch_workspace_bytes(arr, 2, ctypes.byref(n)) == binding.SW_OK
    assert n.value >= _ws(16) + _ws(40, 3)


def test_autotune_rejects_bad_arguments_before_any_launch():
    lib = binding.lib()
    arr = (binding.SwParams * 2)(binding.make_params(64, 2, 1.0), binding.make_params(100, 3, 0.9))
    best = ctypes.c_uint32(7)
    ms = (ctypes.c_double * 3)()

    def call(cands, sweeps=4, ws=0x10000, nbytes=1 << 40, n=2):
        c = (ctypes.c_uint32 * max(1, len(cands)))(*cands)
        return lib.sw_batch_autotune(arr, n, c, len(cands), sweeps, ctypes.c_void_p(ws), nbytes, None,
                                     ctypes.byref(best), ms)

    assert call([32, 48]) == binding.SW_EINVAL            # 48 is not a tile height
    assert call([]) == binding.SW_EINVAL                  # no candidate
    assert call([32] * 9) == binding.SW_EINVAL            # too many candidates
    assert call([64], sweeps=0) == binding.SW_EINVAL
    assert call([64], n=0) == binding.SW_EINVAL
    # the workspace must fit the largest candidate layout, and be aligned
    need = max(binding._batch_bytes(binding._replica_params(
        [{"L": 64, "q": 2, "K": 1.0, "seed": 1}, {"L": 100, "q": 3, "K": 0.9, "seed": 1}], 2, ty))
        for ty in (32, 128))
    assert call([32, 128], nbytes=need - 256) == binding.SW_ESPACE
    assert call([32, 128], ws=0x10001, nbytes=need) == binding.SW_ESPACE
    assert best.value == 7                                 # nothing written on failure


@pytest.mark.parametrize("L,q", [(2, 2), (7, 2), (16, 3), (33, 8), (5, 255)])
def test_derived_matches_oracle(L, q):
    """sw_derived (host FP64 arithmetic of the library) on int64 rows of random
    configurations against the oracle's values computed from the spins."""
    import numpy as np
    rng = np.random.Generator(np.random.PCG64(L + 100 * q))
    for _ in range(4):
        s = rng.integers(0, q, (L, L), dtype=np.uint8)
        row = oracle.observe(s, q)
        got, ref = binding.derived(row, L, q), oracle.derived(s, q)
        assert set(got) == set(ref)
        for k in ref:
            assert math.isclose(got[k], ref[k], rel_tol=1e-12, abs_tol=1e-300) or got[k] == ref[k]


def test_derived_rejects_bad_rows():
    import numpy as np
    row = np.array([0, 0, 3, 1], dtype=np.int64)      # counts add up to 4 = N for L = 2
    assert binding.derived(row, 2, 2)["M"] == 2.0
    out = (ctypes.c_double * 3)()
    for bad, L, q in [(np.array([0, 0, 3, 2], dtype=np.int64), 2, 2),
                      (np.array([0, 0, 5, -1], dtype=np.int64), 2, 2),
                      (row, 1, 2), (row, 65537, 2), (row, 2, 1), (row, 2, 256)]:
        rc = binding.lib().sw_derived(L, q, bad.ctypes.data_as(ctypes.c_void_p), out)
        assert rc == binding.SW_EINVAL, (bad, L, q)


# ------------------------------------------------------------------ XY model

def _xy_ws(L, cap=2, ty=0, bits=32, K=1.0):
    p = binding.make_xy_params(L, K, obs_capacity=cap, tile_rows=ty, dir_bits=bits)
    return binding.lib().sw_xy_workspace_bytes(ctypes.byref(p))


def test_xy_parameter_checks_and_workspace():
    assert _xy_ws(64) > 0 and _xy_ws(64) % 256 == 0
    # angles are 4 bytes a site: 3 more than a Potts lattice's states
    for L in (64, 1000, 4096):
        assert _xy_ws(L) - _ws(L) >= 3 * L * L - 1024      # (regions are 256-byte aligned)
    assert 34.0 * 2**30 < _xy_ws(65536, 1024) < 37.0 * 2**30     # ~8.3 B/site + edge records and forest
    for bad in [dict(L=1), dict(L=65537), dict(bits=0), dict(bits=33), dict(K=-1.0), dict(K=float("nan")),
                dict(ty=48), dict(cap=1)]:
        args = dict(L=64, cap=2, ty=0, bits=32, K=1.0)
        args.update(bad)
        assert _xy_ws(**args) == 0, bad
    p = binding.make_xy_params(64, 1.0)
    p.reserved = 1
    assert binding.lib().sw_xy_workspace_bytes(ctypes.byref(p)) == 0
    assert _xy_ws(64, K=float("inf")) > 0


def test_xy_derived_matches_oracle_values():
    """sw_xy_derived from the oracle's fixed-point row against the oracle's own
    FP64 values from the angles: each of the six sums is off by at most N 2^-31
    (one rounding to 2^-30 per term)."""
    import numpy as np
    rng = np.random.Generator(np.random.PCG64(4))
    for L, K in [(16, 0.7), (33, 1.3), (64, 0.0)]:
        a = rng.integers(0, 2**32, (L, L), dtype=np.uint64).astype(np.uint32)
        row = oracle.xy_observe(a)
        got = binding.xy_derived(row, L, K)
        ref = oracle.xy_derived(a, K)
        N = L * L
        eps = N * 2.0**-31                       # bound on each sum's rounding
        assert abs(got["e"] - ref["e"]) <= 2 * eps / N * (1 + 1e-9)
        mx, my = row[5] * binding.XY_UNIT, row[6] * binding.XY_UNIT
        assert abs(got["m2"] - ref["m2"]) <= (2 * (abs(mx) + abs(my)) * eps + 2 * eps * eps) / N**2 * (1 + 1e-6)
        ix, iy = row[3] * binding.XY_UNIT, row[4] * binding.XY_UNIT
        bound = (eps + K * ((abs(ix) + abs(iy)) * eps + eps * eps)) / N
        assert abs(got["Y"] - ref["Y"]) <= bound * (1 + 1e-6) + 1e-15
    with pytest.raises(binding.SwError):
        binding.xy_derived(np.array([0, 2**62, 0, 0, 0, 0, 0]), 16, 1.0)    # |Ex| > N


def test_whole_lattice_tile_rows():
    assert _ws(128, ty=binding.SW_TILE_WHOLE) > 0
    assert _ws(129, ty=binding.SW_TILE_WHOLE) == 0
    p = binding.make_params(64, 2, 1.0, obs_capacity=4, tile_rows=binding.SW_TILE_WHOLE, cluster_sums=True)
    assert binding.lib().sw_workspace_bytes(ctypes.byref(p)) == 0
    assert _ws(64, ty=binding.SW_TILE_WHOLE) == _ws(64)          # the same workspace layout
    assert _ws(64, ty=5) == 0
    assert _xy_ws(64, ty=binding.SW_TILE_WHOLE) == 0


def test_missing_library_fails_loudly(tmp_path):
    """Without the built HIP library every entry point raises; nothing falls
    back to another implementation (fresh interpreter, library path unbuilt)."""
    import subprocess
    import sys
    code = (
        "from paper_1208_2080_amd import binding\n"
        f"binding.LIB_PATH = {str(tmp_path / 'libswmi.so')!r}\n"
        "for call in (binding.lib, lambda: binding.threshold(1.0)):\n"
        "    try:\n"
        "        call()\n"
        "    except RuntimeError as e:\n"
        "        assert 'missing' in str(e), e\n"
        "    else:\n"
        "        raise SystemExit('no error without the library')\n"
        "print('raised')\n")
    r = subprocess.run([sys.executable, "-c", code], cwd=ROOT, capture_output=True, text=True, timeout=300)
    assert r.returncode == 0 and "raised" in r.stdout, r.stdout + r.stderr
