import os
import shutil
import subprocess
import sys

import numpy as np
import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
if ROOT not in sys.path:
    sys.path.insert(0, ROOT)
HERE = os.path.dirname(os.path.abspath(__file__))
if HERE not in sys.path:
    sys.path.insert(0, HERE)


def pytest_configure(config):
    config.addinivalue_line("markers", "gpu: needs an MI355X (gfx950) GPU")
    config.addinivalue_line("markers", "slow: long-running; opt in with -m slow")


# Philox4x32-10 from rocRAND's own engine, built for and run on the host: the
# independent generator that the oracles' random streams are pinned to.
@pytest.fixture(scope="session")
def rocrand_philox(tmp_path_factory):
    hipcc = shutil.which("hipcc") or "/opt/rocm/bin/hipcc"
    if not os.path.exists(hipcc):
        pytest.skip("hipcc not available to build the rocRAND host reference")
    exe = str(tmp_path_factory.mktemp("rocrand") / "philox_ref")
    subprocess.check_call([hipcc, "-x", "hip", "--cuda-host-only", "-O1", "-o", exe,
                           os.path.join(HERE, "rocrand_ref", "philox_ref.cpp")])

    def run(rows):
        text = "\n".join(" ".join(str(int(v)) for v in r) for r in rows) + "\n"
        out = subprocess.run([exe], input=text, capture_output=True, text=True, check=True).stdout
        return np.array([[int(v) for v in line.split()] for line in out.strip().splitlines()],
                        dtype=np.uint64)

    return run
