"""Host code under AddressSanitizer and UndefinedBehaviorSanitizer (CPU only).

Two builds, both made here from the committed sources:

* the library's host side: every translation unit of the HIP library compiled
  with the sanitizers on its host pass only (device code is built as usual and
  never runs), linked into the driver ``tests/sanitize/capi_host.cpp``, which
  walks the C ABI's parameter checks, workspace sizes, threshold, derived
  observables, argument checks before any launch and calls on missing handles;
* the CPU oracles (plain C) with both sanitizers, whose runs must also equal
  the ordinary build's value for value.

Any sanitizer report aborts the driver (no recovery), and leaks are reported
at exit.
"""
import ctypes
import math
import os
import shutil
import subprocess

import numpy as np
import pytest

import oracle

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
CSRC = os.path.join(ROOT, "paper_1208_2080_amd", "csrc")
HERE = os.path.join(ROOT, "tests", "sanitize")
LIB_SOURCES = ["sw_capi.cpp", "sw_kernels.hip", "sw_xy.hip", "sw_whole.hip", "sw_ablation.hip"]
SAN = ["-fsanitize=address", "-fsanitize=undefined", "-fno-sanitize-recover=all"]
ENV = dict(os.environ, ASAN_OPTIONS="detect_leaks=1:abort_on_error=0", UBSAN_OPTIONS="print_stacktrace=1")


def _clang():
    for c in (shutil.which("amdclang++"), "/opt/rocm/lib/llvm/bin/clang++"):
        if c and os.path.exists(c):
            return c
    pytest.skip("no ROCm clang++ for the sanitized host build")


def _host_flags():
    # each sanitizer flag applies to the host pass only
    out = []
    for f in SAN:
        out += ["-Xarch_host", f]
    return out


def test_host_capi_under_asan_and_ubsan(tmp_path):
    cxx = _clang()
    common = ["-std=c++17", "-O1", "-g", "-I" + os.path.join(ROOT, "include"), "-I" + CSRC]
    procs, objs = [], []
    for src in LIB_SOURCES:
        obj = str(tmp_path / (os.path.splitext(src)[0] + ".o"))
        cmd = [cxx, "-x", "hip", "--offload-arch=gfx950", "-Xclang", "-target-feature", "-Xclang", "-packed-fp32-ops",
               *_host_flags(), *common, "-c", os.path.join(CSRC, src), "-o", obj]
        procs.append(subprocess.Popen(cmd, stdout=subprocess.PIPE, stderr=subprocess.STDOUT, text=True))
        objs.append(obj)
    drv = str(tmp_path / "capi_host.o")
    procs.append(subprocess.Popen([cxx, *SAN, *common, "-c", os.path.join(HERE, "capi_host.cpp"), "-o", drv],
                                  stdout=subprocess.PIPE, stderr=subprocess.STDOUT, text=True))
    for p in procs:
        out, _ = p.communicate(timeout=600)
        assert p.returncode == 0, out
    exe = str(tmp_path / "capi_host")
    subprocess.run([cxx, *SAN, drv, *objs, "-L/opt/rocm/lib", "-lamdhip64", "-Wl,-rpath,/opt/rocm/lib", "-o", exe],
                   check=True, capture_output=True, timeout=300)
    r = subprocess.run([exe], capture_output=True, text=True, timeout=300, env=ENV)
    assert r.returncode == 0, r.stdout + r.stderr
    assert "host C-ABI checks passed" in r.stdout
    assert "Sanitizer" not in r.stderr, r.stderr


# (kind, L, q or None, K, seed, random_start, first_sweep, n_sweeps, dir_bits)
RUNS = [
    ("potts", 2, 2, 0.5, 1, 0, 0, 4, 0),
    ("potts", 3, 3, 1.0, 2, 1, 0, 5, 0),
    ("potts", 5, 2, math.log(1 + math.sqrt(2)), 3, 1, 0, 10, 0),
    ("potts", 8, 4, 1.0986, 4, 1, 7, 6, 0),
    ("potts", 9, 255, 2.0, 5, 1, 0, 3, 0),
    ("potts", 16, 2, float("inf"), 6, 1, 0, 3, 0),
    ("potts", 7, 3, 0.0, 7, 0, 0, 3, 0),
    ("xy", 6, None, 1.12, 7, 1, 3, 5, 32),
    ("xy", 4, None, 0.7, 9, 0, 0, 3, 2),
    ("xy", 11, None, 0.0, 2, 1, 0, 2, 5),
]


def _line(run):
    kind, L, q, K, seed, rs, first, n, bits = run
    k = repr(K) if math.isfinite(K) else "inf"
    if kind == "potts":
        return f"potts {L} {q} {k} {seed} {rs} {first} {n}"
    return f"xy {L} {k} {seed} {rs} {first} {n} {bits}"


def _ordinary(run):
    """The same run through the ordinary oracle build: (state, obs, rc)."""
    kind, L, q, K, seed, rs, first, n, bits = run
    lib = oracle.lib()
    N = L * L
    if kind == "potts":
        s = np.zeros(N, dtype=np.uint8)
        obs = np.zeros(n * (2 + q), dtype=np.int64)
        u8 = s.ctypes.data_as(ctypes.POINTER(ctypes.c_uint8))
        rc = lib.or_init(L, q, seed, rs, u8) or lib.or_run(L, q, K, seed, first, n, u8,
                                                          obs.ctypes.data_as(ctypes.POINTER(ctypes.c_int64)))
        return s.tolist(), obs.tolist(), rc
    a = np.zeros(N, dtype=np.uint32)
    obs = np.zeros(n * 7, dtype=np.int64)
    u32 = a.ctypes.data_as(ctypes.POINTER(ctypes.c_uint32))
    rc = lib.or_xy_init(L, seed, rs, u32) or lib.or_xy_run(L, K, seed, first, n, bits, u32,
                                                           obs.ctypes.data_as(ctypes.POINTER(ctypes.c_int64)))
    return a.tolist(), obs.tolist(), rc


def test_oracles_under_asan_and_ubsan_match_the_ordinary_build(tmp_path):
    cc = shutil.which("gcc")
    if not cc:
        pytest.skip("no gcc")
    exe = str(tmp_path / "oracle_runs")
    odir = os.path.join(ROOT, "oracle")
    subprocess.run([cc, "-std=c11", "-O1", "-g", *SAN, "-I" + odir, os.path.join(HERE, "oracle_runs.c"),
                    os.path.join(odir, "sw_oracle.c"), os.path.join(odir, "xy_oracle.c"), "-lm", "-o", exe],
                   check=True, capture_output=True, timeout=300)
    stdin = "".join(_line(r) + "\n" for r in RUNS)
    r = subprocess.run([exe], input=stdin, capture_output=True, text=True, timeout=300, env=ENV)
    assert r.returncode == 0, r.stdout + r.stderr
    assert "Sanitizer" not in r.stderr, r.stderr
    lines = r.stdout.splitlines()
    assert len(lines) == 4 * len(RUNS)
    for i, run in enumerate(RUNS):
        kind, state, obs, rc = lines[4 * i: 4 * i + 4]
        assert kind == run[0]
        want_state, want_obs, want_rc = _ordinary(run)
        assert [int(v) for v in state.split()] == want_state, run
        assert [int(v) for v in obs.split()] == want_obs, run
        assert rc == f"rc {want_rc}" and want_rc == 0, run
