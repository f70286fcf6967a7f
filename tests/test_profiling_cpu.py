"""The rocprofv3 summariser behind the committed profiles (CPU, synthetic CSVs).

Every figure in the profile summaries comes out of these functions: kernel
averages from a kernel trace, HBM bytes from FETCH_SIZE / WRITE_SIZE scaled by
a device copy of known size, and instruction counts per wave.  Each check feeds
a small hand-written CSV whose expected summary is worked out by hand.
"""
import csv
import re

from paper_1208_2080_amd import profiling


def _write(path, fields, rows):
    with open(path, "w", newline="") as f:
        w = csv.DictWriter(f, fieldnames=fields)
        w.writeheader()
        for r in rows:
            w.writerow(r)


TRACE_FIELDS = ["Kernel_Name", "Grid_Size", "Start_Timestamp", "End_Timestamp"]
PMC_FIELDS = ["Dispatch_Id", "Kernel_Name", "Grid_Size", "Counter_Name", "Counter_Value"]


def _row(text, name):
    return next(line for line in text.splitlines() if line.startswith(name))


def test_stats_averages_each_kernel_at_its_largest_grid(tmp_path):
    _write(tmp_path / "run_kernel_trace.csv", TRACE_FIELDS, [
        # two dispatches of the measured grid, 10 us and 20 us
        {"Kernel_Name": "void swmi::k_a<64>(swmi::LatDesc const*, unsigned int)", "Grid_Size": 100,
         "Start_Timestamp": 0, "End_Timestamp": 10000},
        {"Kernel_Name": "void swmi::k_a<64>(swmi::LatDesc const*, unsigned int)", "Grid_Size": 100,
         "Start_Timestamp": 50000, "End_Timestamp": 70000},
        # a smaller side run of the same kernel does not count
        {"Kernel_Name": "void swmi::k_a<64>(swmi::LatDesc const*, unsigned int)", "Grid_Size": 50,
         "Start_Timestamp": 0, "End_Timestamp": 1000000},
        {"Kernel_Name": "swmi::(anonymous namespace)::k_b(unsigned int)", "Grid_Size": 10,
         "Start_Timestamp": 0, "End_Timestamp": 30000},
    ])
    out = profiling.stats(str(tmp_path), "CMD")
    assert "# command: CMD" in out
    assert f"# kernel_source_sha256_16: {profiling.kernel_source_digest()}" in out
    a = _row(out, "k_a<64>").split()
    assert a[1:] == ["100", "2", "15.00", "0.030", "50.00"]
    b = _row(out, "k_b").split()
    assert b[1:] == ["10", "1", "30.00", "0.030", "50.00"]


def test_pmc_scales_kib_by_the_device_copy(tmp_path):
    fetch, write = tmp_path / "f", tmp_path / "w"
    fetch.mkdir()
    write.mkdir()
    k = "void swmi::k_flip<64, false>(swmi::LatDesc const*)"
    copy = "__amd_rocclr_copyBuffer"
    # FETCH_SIZE: the kernel's dispatches read 100 + 200 and 500 KiB (instances
    # of one dispatch are summed); the 1 GiB copy reads 524288 KiB, so a
    # fetched KiB stands for 2048 bytes
    _write(fetch / "run_counter_collection.csv", PMC_FIELDS, [
        {"Dispatch_Id": 1, "Kernel_Name": k, "Grid_Size": 64, "Counter_Name": "FETCH_SIZE", "Counter_Value": 100},
        {"Dispatch_Id": 1, "Kernel_Name": k, "Grid_Size": 64, "Counter_Name": "FETCH_SIZE", "Counter_Value": 200},
        {"Dispatch_Id": 2, "Kernel_Name": k, "Grid_Size": 64, "Counter_Name": "FETCH_SIZE", "Counter_Value": 500},
        {"Dispatch_Id": 3, "Kernel_Name": k, "Grid_Size": 8, "Counter_Name": "FETCH_SIZE", "Counter_Value": 9999},
        {"Dispatch_Id": 4, "Kernel_Name": copy, "Grid_Size": 4, "Counter_Name": "FETCH_SIZE", "Counter_Value": 524288},
        {"Dispatch_Id": 5, "Kernel_Name": copy, "Grid_Size": 4, "Counter_Name": "FETCH_SIZE", "Counter_Value": 16},
    ])
    # WRITE_SIZE: 100 KiB per dispatch; the copy writes 1048576 KiB (1024 bytes each)
    _write(write / "run_counter_collection.csv", PMC_FIELDS, [
        {"Dispatch_Id": 1, "Kernel_Name": k, "Grid_Size": 64, "Counter_Name": "WRITE_SIZE", "Counter_Value": 100},
        {"Dispatch_Id": 2, "Kernel_Name": k, "Grid_Size": 64, "Counter_Name": "WRITE_SIZE", "Counter_Value": 100},
        {"Dispatch_Id": 4, "Kernel_Name": copy, "Grid_Size": 4, "Counter_Name": "WRITE_SIZE", "Counter_Value": 1048576},
    ])
    out = profiling.pmc(str(fetch), str(write), "k_flip<64, false>", "CF", "CW")
    vals = dict(line.split(": ", 1) for line in out.splitlines() if not line.startswith("#"))
    assert vals["dispatches"] == "2"
    assert float(vals["fetch_kib_per_dispatch"]) == 400.0
    assert float(vals["write_kib_per_dispatch"]) == 100.0
    assert float(vals["fetch_scale_bytes_per_kib"]) == 2048.0
    assert float(vals["write_scale_bytes_per_kib"]) == 1024.0
    assert int(vals["traffic_bytes_per_dispatch"]) == 400 * 2048 + 100 * 1024


def test_counters_give_instructions_per_wave_and_per_wave_row(tmp_path):
    a, b = tmp_path / "a", tmp_path / "b"
    a.mkdir()
    b.mkdir()
    k = "void swmi::k_bond_label<64, false>(swmi::LatDesc const*)"
    # pass a: 16 waves issue 1760 vector instructions; pass b: the same waves, 880 scalar
    _write(a / "run_counter_collection.csv", PMC_FIELDS, [
        {"Dispatch_Id": 1, "Kernel_Name": k, "Grid_Size": 1024, "Counter_Name": "SQ_WAVES", "Counter_Value": 16},
        {"Dispatch_Id": 1, "Kernel_Name": k, "Grid_Size": 1024, "Counter_Name": "SQ_INSTS_VALU", "Counter_Value": 1760},
    ])
    _write(b / "run_counter_collection.csv", PMC_FIELDS, [
        {"Dispatch_Id": 1, "Kernel_Name": k, "Grid_Size": 1024, "Counter_Name": "SQ_INSTS_SALU", "Counter_Value": 880},
    ])
    out = profiling.counters([str(a), str(b)], ["k_bond_label<64, false>"], ["C1", "C2"], rows_per_wave=16)
    assert "# command: C1" in out and "# command: C2" in out
    assert "SQ_INSTS_VALU: 1760.0 per dispatch (1 dispatches, grid 1024)" in out
    # 1760 / 16 = 110 per wave, 110 / 16 = 6.875 per wave-row
    assert re.search(r"SQ_INSTS_VALU per wave: 110\.0, per wave-row 6\.9", out)
    assert re.search(r"SQ_INSTS_SALU per wave: 55\.0, per wave-row 3\.4", out)


def test_kernel_names_are_shortened_to_their_instantiation():
    assert profiling._short("void swmi::k_merge<64>(swmi::LatDesc const*, swmi::WorkItem const*, unsigned int)") \
        == "k_merge<64>"
    assert profiling._short("void swmi::(anonymous namespace)::k_xy_bonds<64>(swmi::LatDesc const*)") \
        == "k_xy_bonds<64>"


def test_source_digest_is_a_stable_16_hex_prefix():
    d = profiling.kernel_source_digest()
    assert re.fullmatch(r"[0-9a-f]{16}", d)
    assert d == profiling.kernel_source_digest()
