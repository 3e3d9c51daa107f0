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
    fetch = [(copy, 1024.0), (copy, 8 * GiB_KiB), ("void (anonymous namespace)::k_fill<0, 1, false>(FillArgs)", 20.0),
             ("void (anonymous namespace)::k_fill<0, 1, false>(FillArgs)", 40.0),
             ("void (anonymous namespace)::k_fill<2, 1, false>(FillArgs)", 64.0),
             ("void (anonymous namespace)::k_reduce_queue<1, 2, false>(ReduceArgs)", 70.0),
             ("void (anonymous namespace)::k_reduce_queue<3, 2, false>(ReduceArgs)", 72.0),
             ("void (anonymous namespace)::k_fill<0, 4, true>(FillArgs)", 9999.0)]  # strided: not a step kernel
    write = [(copy, 4 * GiB_KiB), ("void (anonymous namespace)::k_fill<0, 1, false>(FillArgs)", 16 * GiB_KiB),
             ("void (anonymous namespace)::k_fill<2, 1, false>(FillArgs)", 32 * GiB_KiB),
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
