"""Build the HIP library ``libswmi.so`` (gfx950) in-tree with hipcc."""
from __future__ import annotations

import os
import shutil
import subprocess

HERE = os.path.dirname(os.path.abspath(__file__))
CSRC = os.path.join(HERE, "csrc")
LIB = os.path.join(HERE, "libswmi.so")
SOURCES = ["sw_kernels.hip", "sw_xy.hip", "sw_whole.hip", "sw_ablation.hip", "sw_capi.cpp"]
ARCH = "gfx950"

# hipcc flags for every HIP translation unit: gfx950 only, no packed-FP32 ops.
HIP_FLAGS = ["--offload-arch=" + ARCH, "-O3", "-std=c++17", "-fPIC", "-Wall",
             "-Xclang", "-target-feature", "-Xclang", "-packed-fp32-ops"]


def hipcc() -> str:
    exe = shutil.which("hipcc") or "/opt/rocm/bin/hipcc"
    if not os.path.exists(exe):
        raise RuntimeError("hipcc not found: the HIP library cannot be built")
    return exe


def _run(cmd, verbose: bool):
    if verbose:
        print(" ".join(cmd), flush=True)
    res = subprocess.run(cmd, capture_output=True, text=True)
    # hipcc's host pass warns that it does not know the packed-FP32 feature; drop that line
    noise = "is not a recognized feature for this target"
    text = "\n".join(l for l in (res.stdout + res.stderr).splitlines() if noise not in l)
    if res.returncode != 0:
        raise RuntimeError("command failed: %s\n%s" % (" ".join(cmd), text))
    if verbose and text.strip():
        print(text, flush=True)


# The profiling build: the same sources with the kernels' phase clocks on
# (-DSW_PHASE_CLOCKS), linked apart from the product library.
PHASE_LIB = os.path.join(HERE, "libswmi_phase.so")


def build(verbose: bool = False, lib: str = LIB, defines=()) -> str:
    """Compile every source for gfx950 and link ``lib`` (by default
    ``libswmi.so`` next to this file) with the given preprocessor defines."""
    tag = ".phase" if defines else ""
    objs = []
    for src in SOURCES:
        obj = os.path.join(CSRC, src + tag + ".o")
        _run([hipcc()] + HIP_FLAGS + ["-D" + d for d in defines] + ["-c", os.path.join(CSRC, src), "-o", obj],
             verbose)
        objs.append(obj)
    tmp = lib + ".tmp%d" % os.getpid()
    _run([hipcc(), "--offload-arch=" + ARCH, "-shared", "-fPIC", "-o", tmp] + objs, verbose)
    os.replace(tmp, lib)
    for obj in objs:
        os.remove(obj)
    return lib


def build_phase_clocks(verbose: bool = False) -> str:
    """The profiling library with the kernels' phase clocks (``libswmi_phase.so``)."""
    return build(verbose, PHASE_LIB, ("SW_PHASE_CLOCKS",))


if __name__ == "__main__":
    import sys
    print(build_phase_clocks(verbose=True) if "--phase-clocks" in sys.argv else build(verbose=True))
