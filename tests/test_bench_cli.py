"""CPU checks of bench.py's host logic: the multi-GPU refusal and the HBM
traffic extraction from rocprofv3 counter files (synthetic files here; no
GPU and no profiler involved)."""
from __future__ import annotations

import csv
import os
import subprocess
import sys

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
sys.path.insert(0, ROOT)


def test_more_than_one_gpu_is_refused():
    r = subprocess.run([sys.executable, os.path.join(ROOT, "bench.py"), "--gpus", "2"], capture_output=True,
                       text=True, timeout=120, cwd=ROOT)
    assert r.returncode == 2
    assert "one GPU" in r.stderr
    assert r.stdout == ""


def _write_counters(path, counter, rows):
    with open(path, "w", newline="") as f:
        w = csv.DictWriter(f, fieldnames=["Dispatch_Id", "Kernel_Name", "Counter_Name", "Counter_Value"])
        w.writeheader()
        for i, (name, kib) in enumerate(rows):
            w.writerow({"Dispatch_Id": i, "Kernel_Name": name, "Counter_Name": counter, "Counter_Value": kib})


def test_traffic_extraction_scales_by_the_copy(tmp_path):
    import bench

    copy = "__amd_rocclr_copyBuffer"
    GiB_KiB = 1 << 20
    # the copy of 4 GiB reads 2x its size on the fetch counter and 1x on the write counter
    # the one-chunk fills run as k_fill_lanes<K, S>, the other shapes as k_fill<K, U, S>
    lanes0 = "void (anonymous namespace)::k_fill_lanes<0, false>(FillLaneArgs)"
    lanes2 = "void (anonymous namespace)::k_fill_lanes<2, false>(FillLaneArgs)"
    fetch = [(copy, 1024.0), (copy, 8 * GiB_KiB), (lanes0, 20.0),
             ("void (anonymous namespace)::k_fill<0, 1, false>(FillArgs)", 40.0),
             (lanes2, 64.0),
             ("void (anonymous namespace)::k_reduce_queue<1, 2, false>(ReduceArgs)", 70.0),
             ("void (anonymous namespace)::k_reduce_queue<3, 2, false>(ReduceArgs)", 72.0),
             ("void (anonymous namespace)::k_fill<0, 4, true>(FillArgs)", 9999.0)]  # strided: not a step kernel
    write = [(copy, 4 * GiB_KiB), (lanes0, 16 * GiB_KiB), (lanes2, 32 * GiB_KiB),
             ("void (anonymous namespace)::k_reduce_queue<1, 2, false>(ReduceArgs)", 2176.0),
             ("void (anonymous namespace)::k_reduce_queue<3, 2, false>(ReduceArgs)", 2176.0)]
    fp, wp = str(tmp_path / "fetch.csv"), str(tmp_path / "write.csv")
    _write_counters(fp, "FETCH_SIZE", fetch)
    _write_counters(wp, "WRITE_SIZE", write)
    t = bench.traffic_from_pmc(fp, wp, 32)
    assert t["factors"] == {"fetch": 0.5, "write": 1.0, "copy_bytes": 4 << 30}
    assert t["detail"]["sq32_fill"] == {"fetch_bytes": 15360, "write_bytes": 16 << 30}  # mean of 20 and 40 KiB, halved
    assert t["kernels"]["sq64_fill"] == 32 * 1024 + (32 << 30)
    assert t["kernels"]["fused_f32_sum"] == 35 * 1024 + 2176 * 1024
    assert t["source_sha"] == bench.kernel_source_sha()


def test_kernel_summary_keeps_full_size_dispatches(tmp_path):
    import bench

    p = str(tmp_path / "trace.csv")
    with open(p, "w", newline="") as f:
        w = csv.DictWriter(f, fieldnames=["Kernel_Name", "Grid_Size", "Start_Timestamp", "End_Timestamp"])
        w.writeheader()
        big, small = 1 << 31, 1 << 22
        for name, grid, ns in [("void (anonymous namespace)::k_fill_lanes<2, false>(FillLaneArgs)", big, 4_800_000),
                               ("void (anonymous namespace)::k_fill<2, 1, false>(FillArgs)", big, 4_600_000),
                               ("void (anonymous namespace)::k_fill<2, 1, false>(FillArgs)", small, 3_000),
                               ("void (anonymous namespace)::k_fill<0, 1, false>(FillArgs)", 1 << 30, 2_500_000),
                               ("void (anonymous namespace)::k_store_chunk(unsigned char*, unsigned int, unsigned int)",
                                big, 5_000_000)]:
            w.writerow({"Kernel_Name": name, "Grid_Size": grid, "Start_Timestamp": 1000, "End_Timestamp": 1000 + ns})
    s = bench.kernel_summary(p)
    assert "| sq64_fill | 2 | 4.7000 | 4.6000 | 4.8000 |" in s
    assert "| sq32_fill | 1 | 2.5000 |" in s
    assert "| store_ceiling | 1 | 5.0000 |" in s


def test_clock_from_samples():
    import numpy as np

    import bench

    # shader clock counter at 2.0 GHz against the 100 MHz real-time counter
    wall = np.arange(0, 100_000, 1000, dtype=np.uint64)
    clk = wall * np.uint64(20) + np.uint64(12345)
    raw = np.stack([clk, wall], axis=1).reshape(-1)
    c = bench.clock_from_samples(raw)
    assert c["mean_ghz"] == 2.0 and c["p10_ghz"] == 2.0 and c["samples"] == 100


def test_git_revision_falls_back_to_the_build_record(tmp_path):
    """Outside a git checkout the revision comes from the library build's
    build_info.json; without either it is unknown."""
    import json

    import bench

    assert bench.git_revision(str(tmp_path)) == (None, None)
    (tmp_path / "paper_2004_06278_amd").mkdir()
    with open(tmp_path / "paper_2004_06278_amd" / "build_info.json", "w") as f:
        json.dump({"git_rev": "0123456789ab", "tree_had_changes": True}, f)
    assert bench.git_revision(str(tmp_path)) == ("0123456789ab", "library build (tree had changes)")
    if os.path.isdir(os.path.join(bench.ROOT, ".git")):
        rev, source = bench.git_revision()
        assert source == "checkout" and rev
