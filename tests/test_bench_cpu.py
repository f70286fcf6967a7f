"""bench.py on the CPU: the one-GPU contract and the counter-summary reader."""
import os
import subprocess
import sys

import bench

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


def test_more_than_one_gpu_is_refused_with_a_message():
    p = subprocess.run([sys.executable, os.path.join(ROOT, "bench.py"), "--gpus", "2"], capture_output=True,
                       text=True, timeout=120)
    assert p.returncode == 2
    assert "one GPU" in p.stderr


def test_traffic_is_read_only_for_the_current_kernel_source(tmp_path, monkeypatch):
    prof = tmp_path / "profiles"
    prof.mkdir()
    body = ("kernel: k_bond_label\nfetch_kib_per_dispatch: 1000.0\nwrite_kib_per_dispatch: 500.0\n"
            "fetch_scale_bytes_per_kib: 2048.0\nwrite_scale_bytes_per_kib: 1024.0\n")
    f = prof / "k_bond_label_L16384_ty64_pmc.txt"
    monkeypatch.setattr(bench, "ROOT", str(tmp_path))
    src = tmp_path / "paper_1208_2080_amd" / "csrc"
    src.mkdir(parents=True)
    for name in ("sw_kernels.hip", "sw_device.hpp", "sw_layout.hpp"):
        (src / name).write_text(name)
    f.write_text(f"kernel_source_sha256_16: {bench.kernel_source_digest()}\n" + body)
    assert bench.measured_traffic("k_bond_label", "L16384", 64) == 1000.0 * 2048.0 + 500.0 * 1024.0
    # counters taken on another kernel source are not reported
    f.write_text("kernel_source_sha256_16: 0000000000000000\n" + body)
    assert bench.measured_traffic("k_bond_label", "L16384", 64) is None
    assert bench.measured_traffic("k_flip", "L16384", 64) is None


def test_workloads_match_the_throughput_configurations():
    w = bench.workloads()
    assert w["L16384"]["L"] == 16384 and w["L16384"]["q"] == 2
    assert w["L65536q2"]["L"] == 65536 and not w["L65536q2"]["random_start"]
    assert w["L65536q3"]["q"] == 3
