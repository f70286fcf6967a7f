"""The oracles' pins catch plausible mistakes (CPU).

Each case plants one mistake in a copy of ``oracle/sw_oracle.c`` or
``oracle/xy_oracle.c`` (a dropped term, a wrong constant, index or sign, a
transposed operand), builds that copy and runs the pins of that oracle
(``tests/test_oracle_pins.py``, ``tests/test_xy_oracle_pins.py``) against it in
a fresh process: at least one pin must fail.  The unchanged copy, built and run
the same way, must pass both, which shows that the pins really load the copy.
"""
import os
import shutil
import subprocess
import sys
from concurrent.futures import ThreadPoolExecutor

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
ODIR = os.path.join(ROOT, "oracle")

# (what the mistake is, text in sw_oracle.c, text it becomes)
POTTS_MUTANTS = [
    ("the +x bond that wraps around the torus dropped",
     "if (bx[i]) join(label, i, (uint32_t)((uint64_t)y * L));",
     "if (0 && bx[i]) join(label, i, (uint32_t)((uint64_t)y * L));"),
    ("bond probability for 2K instead of K",
     "double p = -expm1(-K);", "double p = -expm1(-2.0 * K);"),
    ("a transposed neighbour in the energy",
     "unsat += (si != s[(uint64_t)yd * L + x]);", "unsat += (si != s[(uint64_t)x * L + yd]);"),
    ("the new state keyed by the site instead of its root",
     "s[i] = (uint8_t)or_newspin(seed, sweep, label[i], q);", "s[i] = (uint8_t)or_newspin(seed, sweep, i, q);"),
    ("the +y bond tested against the wrong neighbour",
     "by[i] = (s[i] == s[(uint64_t)yd * L + x])", "by[i] = (s[i] == s[(uint64_t)yd * L + xr])"),
    ("the +x and +y bond words swapped",
     "*wx = w[2 * b];\n    *wy = w[2 * b + 1];", "*wx = w[2 * b + 1];\n    *wy = w[2 * b];"),
    ("the bond words of a site pair interleaved the other way",
     "*wx = w[2 * b];\n    *wy = w[2 * b + 1];", "*wx = w[b];\n    *wy = w[b + 2];"),
    ("a wrong Weyl constant in Philox", "k1 += 0xBB67AE85u;", "k1 += 0xBB67AE84u;"),
    ("a draw mapped to a state by a modulo", "return (uint32_t)(((uint64_t)w * (uint64_t)q) >> 32);",
     "return w % q;"),
    ("the larger root kept instead of the smaller",
     "if (ra < rb) label[rb] = ra;\n    else label[ra] = rb;", "if (ra < rb) label[ra] = rb;\n    else label[rb] = ra;"),
    ("the initial spins drawn from the new-state stream",
     "draw(seed, site, 0u, 2u, w);", "draw(seed, site, 0u, 1u, w);"),
    ("only the +x bonds counted as active", "active += bx[i] + by[i];", "active += bx[i];"),
]

# (what the mistake is, text in xy_oracle.c, text it becomes)
XY_MUTANTS = [
    ("the embedded coupling K instead of 2K", "double k2 = 2.0 * K;", "double k2 = K;"),
    ("bonds whatever the sides of the spins (no sign test)",
     "bx[i] = (ci * cr > 0.0) && (ux < -expm1(-(k2 * ci) * cr));",
     "bx[i] = (ux < -expm1(-fabs((k2 * ci) * cr)));"),
    ("the reflection without the half turn", "return 2u * phi + 0x80000000u - a;", "return 2u * phi - a;"),
    ("the wrong words for the 53-bit uniform",
     "uint32_t hi = w[2 * (dir & 1u)], lo = w[2 * (dir & 1u) + 1];",
     "uint32_t hi = w[dir & 1u], lo = w[(dir & 1u) + 2];"),
    ("a transposed neighbour in the +y projection",
     "double cd = or_xy_projection(a[(uint64_t)yd * L + x], phi);",
     "double cd = or_xy_projection(a[(uint64_t)x * L + yd], phi);"),
    ("the reflection keyed by the site instead of its root",
     "if (or_xy_flipbit(seed, sweep, label[i]))", "if (or_xy_flipbit(seed, sweep, i))"),
    ("Ey summing the x terms", "ey += fx(cy);", "ey += fx(cx);"),
    ("the low bit as the reflection bit", "return w[0] >> 31;", "return w[0] & 1u;"),
    ("a wrong quarter-turn rotation", "case 1: *s = cx; *c = -sx; break;", "case 1: *s = cx; *c = sx; break;"),
    ("My summing cosines", "my += fx(st);", "my += fx(ct);"),
]

PINS = {"sw_oracle.c": "test_oracle_pins.py", "xy_oracle.c": "test_xy_oracle_pins.py"}
MUTANTS = [("sw_oracle.c",) + m for m in POTTS_MUTANTS] + [("xy_oracle.c",) + m for m in XY_MUTANTS]


def _build(tmp, name, src_file, old, new):
    d = os.path.join(tmp, name)
    os.makedirs(d)
    for f in ("sw_oracle.c", "sw_oracle.h", "xy_oracle.c", "xy_oracle.h"):
        shutil.copy(os.path.join(ODIR, f), d)
    if old is not None:
        path = os.path.join(d, src_file)
        src = open(path).read()
        assert src.count(old) == 1, f"mutation site not found once: {old!r}"
        open(path, "w").write(src.replace(old, new))
    so = os.path.join(d, "liboracle.so")
    subprocess.run(["gcc", "-O2", "-std=c11", "-fPIC", "-shared", "-o", so, os.path.join(d, "sw_oracle.c"),
                    os.path.join(d, "xy_oracle.c"), "-lm"], check=True, capture_output=True, timeout=300)
    return so


def _pins(job):
    so, files = job
    env = dict(os.environ, SW_ORACLE_LIB=so)
    # each run keeps its temporary files apart (concurrent sessions prune a shared one)
    r = subprocess.run([sys.executable, "-m", "pytest", *[os.path.join(ROOT, "tests", f) for f in files], "-q",
                        "-p", "no:cacheprovider", "--timeout", "300",
                        "--basetemp", os.path.join(os.path.dirname(so), "pytest-tmp")],
                       cwd=ROOT, env=env, capture_output=True, text=True, timeout=900)
    return r.returncode, r.stdout[-2000:]


def test_every_planted_mistake_fails_a_pin(tmp_path):
    if not shutil.which("gcc"):
        pytest.skip("no gcc")
    jobs = {"control": (_build(str(tmp_path), "control", None, None, None), list(PINS.values()))}
    for i, (src_file, _, old, new) in enumerate(MUTANTS):
        jobs[f"m{i}"] = (_build(str(tmp_path), f"m{i}", src_file, old, new), [PINS[src_file]])
    with ThreadPoolExecutor(max_workers=min(6, os.cpu_count() or 1)) as ex:
        results = dict(zip(jobs, ex.map(_pins, jobs.values())))
    rc, out = results["control"]
    assert rc == 0, "the unchanged copy must pass its pins:\n" + out
    survivors = []
    for i, (_, what, _, _) in enumerate(MUTANTS):
        rc, out = results[f"m{i}"]
        assert rc in (0, 1), f"{what}: the pins did not run (exit {rc}):\n{out}"
        if rc == 0:
            survivors.append(what)
    assert not survivors, f"mistakes no pin caught: {survivors}"
