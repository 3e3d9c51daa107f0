#!/usr/bin/env python3
"""Benchmark of the Squares RNG hot path on one MI355X.

Workload (single-key throughput): one distinct-digit key, a uniformly random
64-bit starting counter, n = 2^32 outputs per operation.  One step is
    squares32 fill to HBM     (16 GiB of uint32)
    squares64 fill to HBM     (32 GiB of uint64)
    fused f32 sum             (squares32 -> 24-bit uniform, summed exactly in registers, no per-element writes)
    fused f64 sum             (squares64 -> 53-bit uniform, summed exactly in registers)
so a step produces 4 * 2^32 numbers.  The timed region holds exactly --steps
steps with a device synchronisation on both sides; inputs are scalars, so
nothing is transferred.  The JSON line carries the whole-step rate, each
kernel's average duration from HIP events on the launch stream, the
roofline of the dominant kernel (and of every kernel, in the step and
repeated back to back), the CPU oracle's rate on a bounded sample,
and (unless --no-extras) the split-word variant of squares64, the counter
modes (increments other than one, key-counter mode, key generation), the
ragged-batch speedup over per-stream launches and serving latency
percentiles.

Usage: python bench.py [--gpus 1] [--steps K] [--warmup W] [--log2n 32] [--no-extras]
                       [--extras concurrent,uniform,pair,split,modes,batch,serving] [--no-cpu]
"""
from __future__ import annotations

import argparse
import json
import os
import sys
import time

ROOT = os.path.dirname(os.path.abspath(__file__))
if ROOT not in sys.path:
    sys.path.insert(0, ROOT)

HBM_PEAK_GBS = 8000.0           # MI355X HBM3E, published
CUS, CLOCK_HZ = 256, 2.4e9      # MI355X compute units and peak engine clock
# VALU issue model (measured on this part with paper_2004_06278_amd/calib):
# v_mad_u64_u32, v_mul_lo_u32, v_lshl_add_u32 and 64-bit adds issue at the
# full 64 lanes per CU per clock (one "slot"); two-operand 32-bit ops
# (add, shift, xor) issue up to twice as fast and count half a slot.
# Peak = 256 CUs * 2.4 GHz * 64 lanes (matching fp64 vector 78.6 TFLOP/s).
ALU_PEAK_SLOTS = CUS * CLOCK_HZ * 64
# Algorithmic VALU work per output in slots, as the fused sums compute it: a
# round is one 32x32->64 multiply-add (1) + one 32-bit multiply (1) + one
# shift-add (1); round 1 of every counter after a run's first comes from
# running differences (r1 += d, d += 2*key*key: two 64-bit adds, 2 slots
# instead of the squaring's 3); the Weyl step to the next counter is one
# 64-bit add (1).
SLOTS = {
    "sq32": 3 * 3.0 + 2.0 + 1.0,           # 12
    "sq64": 4 * 3.0 + 2.0 + 0.5 + 1.0,     # 15.5 (+ the xor of round 5)
    "sum_f32": 0.5 + 1.0,                  # >> 8, 32-bit accumulate (half a 3-input add) + flush share
    "sum_f64": 1.0 + 1.0,                  # 64-bit >> 11, 64-bit accumulate
    "pair_f32": 0.5 + 0.5,                 # the paired sum's F32 term: >> 40, 32-bit accumulate
}
KERNEL_SOURCES = ["paper_2004_06278_amd/csrc/sq_device.hpp", "paper_2004_06278_amd/csrc/sq_kernels.hip"]
# rocprofv3 kernel names (spaces and namespace removed) of the four step
# operations: the unit-step instantiations of the fill and reduce templates
KERNEL_NAMES = {"sq32_fill": r"k_fill(_lanes)?<0,(\d+,)?false>", "sq64_fill": r"k_fill(_lanes)?<2,(\d+,)?false>",
                "fused_f32_sum": r"k_reduce(_queue)?<1,\d+,false>", "fused_f64_sum": r"k_reduce(_queue)?<3,\d+,false>"}


def kernel_source_sha() -> str:
    import hashlib

    h = hashlib.sha256()
    for rel in KERNEL_SOURCES:
        with open(os.path.join(ROOT, rel), "rb") as f:
            h.update(f.read())
    return h.hexdigest()[:16]


def traffic_from_pmc(fetch_csv: str, write_csv: str, log2n: int) -> dict:
    """HBM bytes per launch of each step kernel from two rocprofv3 --pmc runs
    (FETCH_SIZE, WRITE_SIZE; KiB per dispatch), each scaled by what the same
    counter reads for the plain 4 GiB device copy that --calib-copy runs
    first (the largest __amd_rocclr_copyBuffer dispatch)."""
    import csv
    import re

    pats = dict(KERNEL_NAMES)
    pats["batch_fill"] = r"k_batch_fill<\d+>"

    def load(path):
        rows = list(csv.DictReader(open(path)))
        copy = max((r for r in rows if "copyBuffer" in r["Kernel_Name"]), key=lambda r: float(r["Counter_Value"]))
        per = {}
        for name, pat in pats.items():
            # fills: only the 2^32-output launches (one workgroup per 4 KiB chunk,
            # at least 2^30 work-items), not the batch extra's per-stream launches
            vals = [float(r["Counter_Value"]) * 1024 for r in rows
                    if re.search(pat, r["Kernel_Name"].replace(" ", "").replace("(anonymousnamespace)::", ""))
                    and (not name.endswith("_fill") or name == "batch_fill"
                         or int(r.get("Grid_Size") or (1 << 31)) >= (1 << 30))]
            per[name] = sum(vals) / len(vals) if vals else None
        return float(copy["Counter_Value"]) * 1024, per

    copy_f, fetch = load(fetch_csv)
    copy_w, write = load(write_csv)
    ref = float(4 << 30)
    ff, fw = ref / copy_f, ref / copy_w
    kernels, detail = {}, {}
    for name in pats:
        if fetch[name] is None or write[name] is None:
            continue
        kernels[name] = round(fetch[name] * ff + write[name] * fw)
        detail[name] = {"fetch_bytes": round(fetch[name] * ff), "write_bytes": round(write[name] * fw)}
    return {"source_sha": kernel_source_sha(), "log2n": log2n,
            "factors": {"fetch": round(ff, 4), "write": round(fw, 4), "copy_bytes": int(ref)},
            "kernels": kernels, "detail": detail}


def measure_lib():
    """libsqmeasure.so (paper_2004_06278_amd/calib/sq_measure.hip): the store-only
    ceiling kernel and the clock sampler.  Built by __graft_entry__.build()."""
    import ctypes

    from paper_2004_06278_amd import build as b

    if not os.path.exists(b.MEASURE_LIB):
        raise RuntimeError(f"{b.MEASURE_LIB} is missing: build it first (__graft_entry__.build())")
    L = ctypes.CDLL(b.MEASURE_LIB)
    L.sqm_store_ceiling.restype = ctypes.c_int
    L.sqm_store_ceiling.argtypes = [ctypes.c_void_p, ctypes.c_uint64, ctypes.c_uint32, ctypes.c_void_p]
    L.sqm_clock_sampler.restype = ctypes.c_int
    L.sqm_clock_sampler.argtypes = [ctypes.c_void_p, ctypes.c_uint32, ctypes.c_uint64, ctypes.c_void_p]
    return L


def git_revision(root: str = ROOT) -> tuple[str | None, str | None]:
    """(revision, where it came from): the checkout's HEAD, else the revision
    the library build recorded in build_info.json (runs made where the tree
    was copied without its git history), else (None, None)."""
    import subprocess

    try:
        rev = subprocess.run(["git", "-C", root, "rev-parse", "--short=12", "HEAD"], capture_output=True, text=True,
                             timeout=10).stdout.strip()
        if rev:
            return rev, "checkout"
    except (OSError, subprocess.SubprocessError):
        pass
    try:
        with open(os.path.join(root, "paper_2004_06278_amd", "build_info.json")) as f:
            info = json.load(f)
    except (OSError, ValueError):
        return None, None
    if not info.get("git_rev"):
        return None, None
    return info["git_rev"], "library build" + (" (tree had changes)" if info.get("tree_had_changes") else "")


def run_metadata(torch) -> dict:
    """Where and on what the line was measured."""
    rev, source = git_revision()
    prop = torch.cuda.get_device_properties(0)
    return {"git_rev": rev, "git_rev_source": source, "kernel_source_sha": kernel_source_sha(), "device": prop.name,
            "gfx_arch": getattr(prop, "gcnArchName", None), "cus": prop.multi_processor_count,
            "hip": getattr(torch.version, "hip", None), "torch": torch.__version__}


def clock_from_samples(raw) -> dict:
    """Mean shader clock over the sampler's window from (clock64, wall_clock64)
    pairs: the shader clock counter against the 100 MHz real-time counter."""
    import numpy as np

    s = np.asarray(raw, dtype=np.uint64).reshape(-1, 2).astype(np.float64)
    dc, dw = np.diff(s[:, 0]), np.diff(s[:, 1])
    ok = dw > 0
    per = dc[ok] / dw[ok] * 0.1  # GHz over each interval
    mean = (s[-1, 0] - s[0, 0]) / max(s[-1, 1] - s[0, 1], 1) * 0.1
    return {"mean_ghz": round(float(mean), 3), "p10_ghz": round(float(np.percentile(per, 10)), 3),
            "p90_ghz": round(float(np.percentile(per, 90)), 3), "samples": int(s.shape[0]),
            "window_ms": round(float((s[-1, 1] - s[0, 1]) * 1e-5), 2),
            "method": "one wave on a side stream records the shader clock counter (s_memtime) and the 100 MHz "
                      "real-time counter (s_memrealtime) at a fixed spacing over the timed steps; one XCD"}


def valu_from_pmc(csv_path: str, log2n: int) -> dict:
    """Measured VALU instructions per output and shader clock of the step and
    uniform-fill kernels, and of the ragged batch's fill kernel, from a
    rocprofv3 --pmc GRBM_GUI_ACTIVE SQ_INSTS_VALU run of this benchmark
    (SQ_INSTS_VALU counts wave instructions: x 64 lanes / outputs)."""
    import csv
    import re

    from paper_2004_06278_amd import workloads as W

    n = 1 << log2n
    pats = dict(KERNEL_NAMES)
    pats.update({"uniform_f32_fill": r"k_fill(_lanes)?<1,(\d+,)?false>",
                 "uniform_f64_fill": r"k_fill(_lanes)?<3,(\d+,)?false>",
                 "batch_fill": r"k_batch_fill<\d+>"})
    outputs = {k: n for k in pats}
    outputs["batch_fill"] = W.ragged_batch(seed=3).total_outputs
    disp = {}
    for r in csv.DictReader(open(csv_path)):
        d = disp.setdefault(int(r["Dispatch_Id"]), {"name": r["Kernel_Name"].replace(" ", "").replace(
            "(anonymousnamespace)::", ""), "ns": int(r["End_Timestamp"]) - int(r["Start_Timestamp"])})
        d[r["Counter_Name"]] = float(r["Counter_Value"])
    kernels = {}
    for key, pat in pats.items():
        rows = [d for d in disp.values() if re.search(pat, d["name"]) and "SQ_INSTS_VALU" in d]
        # the batch extra also replays small batches; keep dispatches of the full workload's size
        rows = [d for d in rows if d["SQ_INSTS_VALU"] * 64 / outputs[key] > 5]
        if not rows:
            continue
        valu = sorted(d["SQ_INSTS_VALU"] * 64 / outputs[key] for d in rows)
        clk = sorted(d.get("GRBM_GUI_ACTIVE", 0) / 8 / d["ns"] for d in rows)
        kernels[key] = {"valu_instr_per_output": round(valu[len(valu) // 2], 3), "dispatches": len(rows),
                        "clock_ghz_min_median_max": [round(clk[0], 2), round(clk[len(clk) // 2], 2),
                                                     round(clk[-1], 2)]}
    return {"source_sha": kernel_source_sha(), "log2n": log2n, "kernels": kernels}


def kernel_summary(trace_csv: str) -> str:
    """Markdown table of the full-size dispatches of the step kernels, the
    uniform fills and the store ceiling (at least 2^30 work-items: one
    workgroup per 4 KiB chunk of a 2^32-output fill; the per-stream launches
    of the batch extras use the same fill instantiations on far smaller
    grids and are left out), of the sums, and of the batch fill's dispatches
    that take at least 1 ms (the 4096- and 65536-stream batches) in a
    rocprofv3 --kernel-trace csv of this benchmark."""
    import csv
    import re

    pats = dict(KERNEL_NAMES)
    pats.update({"uniform_f32_fill": r"k_fill(_lanes)?<1,(\d+,)?false>",
                 "uniform_f64_fill": r"k_fill(_lanes)?<3,(\d+,)?false>",
                 "store_ceiling": r"k_store_chunk", "batch_fill": r"k_batch_fill<\d+>"})
    rows = {k: [] for k in pats}
    for r in csv.DictReader(open(trace_csv)):
        name = r["Kernel_Name"].replace(" ", "").replace("(anonymousnamespace)::", "")
        grid = int(r.get("Grid_Size", r.get("Grid_Size_X", 0)) or 0)
        ms = (int(r["End_Timestamp"]) - int(r["Start_Timestamp"])) / 1e6
        for k, pat in pats.items():
            if not re.search(pat, name):
                continue
            if ("fill" in k or k == "store_ceiling") and k != "batch_fill" and grid < (1 << 30):
                continue
            if k == "batch_fill" and ms < 1.0:
                continue
            rows[k].append(ms)
    out = ["| Kernel | Dispatches | Average (ms) | Min (ms) | Max (ms) |", "|---|---|---|---|---|"]
    for k, v in rows.items():
        if v:
            out.append(f"| {k} | {len(v)} | {sum(v) / len(v):.4f} | {min(v):.4f} | {max(v):.4f} |")
    return "\n".join(out)


def parse():
    p = argparse.ArgumentParser()
    p.add_argument("--gpus", type=int, default=1)
    p.add_argument("--steps", type=int, default=20)
    p.add_argument("--warmup", type=int, default=3)
    p.add_argument("--log2n", type=int, default=32)
    p.add_argument("--no-extras", action="store_true")
    p.add_argument("--extras", default="concurrent,uniform,pair,split,modes,batch,batch_wrap,serving",
                   help="comma list of extra measurements after the step "
                        "(concurrent, uniform, pair, split, modes, batch, batch_wrap, serving)")
    p.add_argument("--no-cpu", action="store_true")
    p.add_argument("--no-per-stream", action="store_true",
                   help="batch extra without its 4096 per-stream launches (counter-collection runs, which need "
                        "only the batch kernels)")
    p.add_argument("--calib-copy", action="store_true",
                   help="run a plain 4 GiB device copy first (scales HBM byte counters)")
    p.add_argument("--traffic", nargs=2, metavar=("FETCH_CSV", "WRITE_CSV"),
                   help="write profiles/traffic.json from two rocprofv3 --pmc counter_collection.csv files")
    p.add_argument("--kernel-summary", metavar="TRACE_CSV",
                   help="print a table of the full-size kernel dispatches in a rocprofv3 --kernel-trace csv")
    p.add_argument("--valu", metavar="PMC_CSV",
                   help="write profiles/valu.json from a rocprofv3 --pmc GRBM_GUI_ACTIVE SQ_INSTS_VALU "
                        "counter_collection.csv of this benchmark")
    return p.parse_args()


def cpu_baseline(key: int, ctr0: int, log2_sample: int = 31) -> dict:
    """The oracle as it stands, on the host cores, over the same four
    operations for 2^log2_sample counters each (same key and start).  The
    fills write into a reused host buffer of 2^26 elements, one chunk at a
    time; the sums write nothing."""
    import numpy as np

    from oracle import oracle

    threads = max(1, min(16, os.cpu_count() or 1))
    n = 1 << log2_sample
    chunk = min(n, 1 << 26)
    u32 = np.zeros(chunk, dtype=np.uint32)
    u64 = np.zeros(chunk, dtype=np.uint64)
    t0 = time.perf_counter()
    for base in range(0, n, chunk):
        oracle.fill_into(oracle.U32, key, (ctr0 + base) % 2**64, u32, threads=threads)
    for base in range(0, n, chunk):
        oracle.fill_into(oracle.U64, key, (ctr0 + base) % 2**64, u64, threads=threads)
    oracle.exact_sum(oracle.F32, key, ctr0, n, threads=threads)
    oracle.exact_sum(oracle.F64, key, ctr0, n, threads=threads)
    dt = time.perf_counter() - t0
    # one thread, squares32 only: the figure the paper quotes for one core
    n1 = 1 << 26
    t1 = time.perf_counter()
    oracle.fill_into(oracle.U32, key, ctr0, u32[:n1], threads=1)
    dt1 = time.perf_counter() - t1
    model = ""
    try:
        with open("/proc/cpuinfo") as f:
            model = next((ln.split(":", 1)[1].strip() for ln in f if ln.startswith("model name")), "")
    except OSError:
        pass
    return {"value": round(4 * n / dt / 1e9, 3), "unit": "Gnum/s", "cores": threads, "kind": "oracle",
            "sample": f"2^{log2_sample} counters of each of the 4 step operations (same key and ctr0; fills "
                      f"into a reused 2^26-element host buffer), {threads} host threads, {dt:.2f} s wall, "
                      f"about {threads * dt:.0f} thread-seconds of CPU work",
            "one_thread_sq32_gnum_s": round(n1 / dt1 / 1e9, 3), "host_cpu": model,
            "host_cpus_visible": os.cpu_count()}


def timed_wall(torch, fn, reps: int, warm: int = 2) -> float:
    """Wall-clock seconds per call of fn over `reps` calls issued back to back
    (after `warm` untimed calls), with a device synchronisation on both sides:
    host launch costs count, and the device runs the calls as a caller that
    issues them in a loop would."""
    for _ in range(warm):
        fn()
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    for _ in range(reps):
        fn()
    torch.cuda.synchronize()
    return (time.perf_counter() - t0) / reps


def batch_speedup(sq, torch, per_stream_baseline: bool = True) -> dict:
    """4096 keys, log-uniform lengths in [2^10, 2^24], U32/F32: replays of the
    captured batch plan (scan, map and fill kernels) against the same batch as
    4096 separate fill launches on one stream, each timed per call over calls
    issued back to back (timed_wall: the graph 20 replays after 8, as the
    steady rooflines, the per-stream launches 8 calls after 2).  per_stream_baseline=False skips the
    4096 launches (counter-collection runs need only the batch kernels)."""
    from paper_2004_06278_amd import workloads as W

    b = W.ragged_batch(seed=3)
    db = sq.batch_to_device(b.keys, b.ctr0s, b.lens, b.offs, b.kinds, b.arena_bytes)
    plan = sq.BatchPlan(db)

    def per_stream():
        sq.fill_streams(b.keys, b.ctr0s, b.lens, b.offs, b.kinds, db.out, b.arena_bytes)

    # graph replays as the steady rooflines (20 after 8: the shader clock
    # takes about a dozen HBM-bound launches to settle); the first 10 after 2
    # are reported beside them.  The per-stream side is bound by the host's
    # launch rate, not the clock: 8 after 2.
    t_cold = timed_wall(torch, plan.launch, 10, warm=2)
    t_plan = timed_wall(torch, plan.launch, 20, warm=8)
    t_each = timed_wall(torch, per_stream, 8, warm=2) if per_stream_baseline else None
    plan.close()
    n = b.total_outputs
    del db
    torch.cuda.empty_cache()
    # the same batch with streams starting at random 4-byte offsets
    bm = W.ragged_batch(seed=3, misalign=True)
    dbm = sq.batch_to_device(bm.keys, bm.ctr0s, bm.lens, bm.offs, bm.kinds, bm.arena_bytes)
    planm = sq.BatchPlan(dbm)
    t_mis = timed_wall(torch, planm.launch, 20, warm=8)
    planm.close()
    del dbm
    torch.cuda.empty_cache()
    r = {"workload": "4096 keys, log-uniform lengths 2^10..2^24, U32/F32", "outputs": n,
         "graph_ms": round(t_plan * 1e3, 3), "per_stream_ms": None, "graph_gnum_s": round(n / t_plan / 1e9, 1),
         "per_stream_gnum_s": None, "speedup": None, "graph_gb_s": round(4 * n / t_plan / 1e9, 1),
         "misaligned_graph_ms": round(t_mis * 1e3, 3), "graph_ms_first_10_after_2": round(t_cold * 1e3, 3),
         "timing": "graph and misaligned graph: wall clock of 20 replays after 8 (the first 10 after 2 beside "
                   "them); per-stream: 8 after 2 calls of the 4096 launches"}
    if t_each is not None:
        r.update({"per_stream_ms": round(t_each * 1e3, 3), "per_stream_gnum_s": round(n / t_each / 1e9, 1),
                  "speedup": round(t_each / t_plan, 2)})
    return r


def batch_wrap_speedup(sq, torch) -> dict:
    """The wrap and width stress: 65536 squares64 streams (U64/F64), lengths
    uniform in [1, 65536], counters starting within 2^16 of 2^64 (about half
    pass 2^64 - 1): replays of the captured batch plan against the 65536
    per-stream fill launches (timed_wall: the graph 20 replays after 8, the
    per-stream launches, bound by the host's launch rate, 2 calls after 1).  Outputs of both are compared with each other and
    sampled against the oracle outside the timed region."""
    import numpy as np

    from oracle import oracle
    from paper_2004_06278_amd import workloads as W

    b = W.wrap_batch(seed=4)
    db = sq.batch_to_device(b.keys, b.ctr0s, b.lens, b.offs, b.kinds, b.arena_bytes)
    plan = sq.BatchPlan(db)

    def per_stream():
        sq.fill_streams(b.keys, b.ctr0s, b.lens, b.offs, b.kinds, db.out, b.arena_bytes)

    t_plan = timed_wall(torch, plan.launch, 20, warm=8)
    a = db.out[: b.arena_bytes].clone()
    t_each = timed_wall(torch, per_stream, 2, warm=1)
    same = bool(torch.equal(a, db.out[: b.arena_bytes]))
    del a
    # a few streams against the oracle (the parity tests compare every output)
    g = np.random.Generator(np.random.PCG64(44))
    host = db.out[: b.arena_bytes]
    bad = 0
    for s in g.integers(0, b.m, size=16):
        s = int(s)
        k, W8 = int(b.kinds[s]), 8
        off, ln = int(b.offs[s]), int(b.lens[s])
        got = host[off: off + W8 * ln].cpu().numpy().tobytes()
        ref = oracle.fill(k, int(b.keys[s]), int(b.ctr0s[s]), ln).view(np.uint8).tobytes()
        bad += got != ref
    plan.close()
    n = b.total_outputs
    del db, host
    torch.cuda.empty_cache()
    gbs = 8 * n / t_plan / 1e9
    return {"workload": "65536 squares64 streams, lengths uniform 1..65536, ctr0 within 2^16 of 2^64 (wrapping), "
                        "U64/F64", "outputs": n, "bytes": 8 * n,
            "graph_ms": round(t_plan * 1e3, 3), "per_stream_ms": round(t_each * 1e3, 3),
            "graph_gnum_s": round(n / t_plan / 1e9, 1), "per_stream_gnum_s": round(n / t_each / 1e9, 1),
            "speedup": round(t_each / t_plan, 2), "graph_gb_s": round(gbs, 1),
            "hbm_frac": round(gbs / HBM_PEAK_GBS, 4), "graph_equals_per_stream": same,
            "oracle_sampled_streams": 16, "oracle_mismatches": int(bad)}


def paired_sums(sq, torch, key: int, ctr0: int, n: int, steady_ms: dict) -> dict:
    """The F32 and F64 sums of the step in one pass (sq_reduce_pair: one
    squares64 per counter gives both terms, squares32 being its high word),
    back to back (mean of 10 after 3), against the two separate sums back
    to back; the results are checked against the separate sums.  Also the
    step with its two sums taken as one paired pass (10 steps after 3)."""
    r32, r64, ws = sq.result_tensor(), sq.result_tensor(), sq.reduce_workspace(n)
    ms = _event_ms(torch, lambda: sq.reduce_pair_async(sq.F32, key, ctr0, n, r32, r64, ws), reps=10, warm=3)
    (s32, _, _), (s64, _, _) = sq.read_result(r32), sq.read_result(r64)
    assert (s32, s64) == (sq.reduce(sq.F32, key, ctr0, n)[0], sq.reduce(sq.F64, key, ctr0, n)[0])
    separate = steady_ms["fused_f32_sum"] + steady_ms["fused_f64_sum"]
    slots = SLOTS["sq64"] + SLOTS["sum_f64"] + SLOTS["pair_f32"]
    rate = slots * n / (ms * 1e-3)
    # the step with the two sums taken as one paired pass (the headline step
    # keeps the separate calls)
    out32 = torch.empty(n, dtype=torch.uint32, device="cuda")
    out64 = torch.empty(n, dtype=torch.uint64, device="cuda")

    def step():
        sq.fill(sq.U32, key, ctr0, n, out=out32)
        sq.fill(sq.U64, key, ctr0, n, out=out64)
        sq.reduce_pair_async(sq.F32, key, ctr0, n, r32, r64, ws)

    for _ in range(3):
        step()
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    for _ in range(10):
        step()
    torch.cuda.synchronize()
    step_ms = (time.perf_counter() - t0) * 1e3 / 10
    del out32, out64
    torch.cuda.empty_cache()
    return {"ms": round(ms, 4), "sums_gnum_s": round(2 * n / (ms * 1e-3) / 1e9, 1),
            "separate_sums_ms": round(separate, 4), "vs_separate": round(separate / ms, 3),
            "step_with_paired_sums_ms": round(step_ms, 4),
            "step_with_paired_sums_gnum_s": round(4 * n / (step_ms * 1e-3) / 1e9, 1),
            "roofline": {"bound": "alu", "achieved": round(rate / 1e12, 3), "peak": round(ALU_PEAK_SLOTS / 1e12, 3),
                         "unit": "T VALU-slot/s", "frac": round(rate / ALU_PEAK_SLOTS, 4),
                         "slots_per_counter": slots}}


def split_words(sq, torch, key: int, ctr0: int, n: int, per_op_ms: dict) -> dict:
    """squares64 split into two 32-bit outputs per call (Section 5): a 2^32-output
    U32X2 fill and F32X2 fused sum, timed like the step kernels (mean of 10
    after 2 warm-up), beside the squares32 fill and F32 sum of the step."""
    out = torch.empty(n, dtype=torch.uint32, device="cuda")
    res, ws = sq.result_tensor(), sq.reduce_workspace(n)
    ops = {"u32x2_fill": lambda: sq.fill(sq.U32X2, key, ctr0, n, out=out),
           "fused_f32x2_sum": lambda: sq.reduce_async(sq.F32X2, key, ctr0, n, res, ws)}
    r = {}
    for name, fn in ops.items():
        for _ in range(2):
            fn()
        evs = []
        for _ in range(10):
            a, b = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
            a.record()
            fn()
            b.record()
            evs.append((a, b))
        torch.cuda.synchronize()
        ms = sum(a.elapsed_time(b) for a, b in evs) / len(evs)
        r[name] = {"ms": round(ms, 4), "gnum_s": round(n / (ms * 1e-3) / 1e9, 1)}
    r["u32x2_fill"]["vs_sq32_fill"] = round(per_op_ms["sq32_fill"] / r["u32x2_fill"]["ms"], 3)
    r["fused_f32x2_sum"]["vs_fused_f32_sum"] = round(per_op_ms["fused_f32_sum"] / r["fused_f32x2_sum"]["ms"], 3)
    del out
    torch.cuda.empty_cache()
    return r


def _event_ms(torch, fn, reps: int = 10, warm: int = 2) -> float:
    """Mean duration of fn() from HIP events on the current stream."""
    for _ in range(warm):
        fn()
    evs = []
    for _ in range(reps):
        a, b = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
        a.record()
        fn()
        b.record()
        evs.append((a, b))
    torch.cuda.synchronize()
    return sum(a.elapsed_time(b) for a, b in evs) / len(evs)


def concurrent_step(sq, torch, key: int, ctr0: int, n: int, serial_ms: float, steps: int = 10) -> dict:
    """The same step with the two fills on one stream and the two fused sums
    on another (HBM-bound and VALU-bound work overlapping), timed over
    `steps` steps like the serial step."""
    out32 = torch.empty(n, dtype=torch.uint32, device="cuda")
    out64 = torch.empty(n, dtype=torch.uint64, device="cuda")
    r1, r2 = sq.result_tensor(), sq.result_tensor()
    w1, w2 = sq.reduce_workspace(n), sq.reduce_workspace(n)
    sa, sb = torch.cuda.Stream(), torch.cuda.Stream()
    main = torch.cuda.current_stream()

    def step():
        start = torch.cuda.Event()
        start.record(main)
        sa.wait_event(start)
        sb.wait_event(start)
        sq.fill(sq.U32, key, ctr0, n, out=out32, stream=sa)
        sq.fill(sq.U64, key, ctr0, n, out=out64, stream=sa)
        sq.reduce_async(sq.F32, key, ctr0, n, r1, w1, stream=sb)
        sq.reduce_async(sq.F64, key, ctr0, n, r2, w2, stream=sb)
        ea, eb = torch.cuda.Event(), torch.cuda.Event()
        ea.record(sa)
        eb.record(sb)
        main.wait_event(ea)
        main.wait_event(eb)

    for _ in range(2):
        step()
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    for _ in range(steps):
        step()
    torch.cuda.synchronize()
    ms = (time.perf_counter() - t0) * 1e3 / steps
    del out32, out64
    torch.cuda.empty_cache()
    return {"ms_per_step": round(ms, 4), "gnum_s": round(4 * n / (ms * 1e-3) / 1e9, 1),
            "vs_serial_step": round(serial_ms / ms, 3), "streams": 2}


def uniform_fills(sq, torch, key: int, ctr0: int, n: int, valu: dict | None = None) -> dict:
    """The uniform fills over the same n counters: F32 (16 GiB) and F64
    (32 GiB), conversion fused into the generating kernel, back to back
    (mean of 20 after 8, as the steady rooflines)."""
    r = {}
    for name, kind, W in (("uniform_f32", sq.F32, 4), ("uniform_f64", sq.F64, 8)):
        out = torch.empty(n * W, dtype=torch.uint8, device="cuda")
        ms = _event_ms(torch, lambda: sq.fill(kind, key, ctr0, n, out=out), reps=20, warm=8)
        gbs = W * n / (ms * 1e-3) / 1e9
        r[name] = {"n": n, "ms": round(ms, 4), "gnum_s": round(n / (ms * 1e-3) / 1e9, 1), "gb_s": round(gbs, 1),
                   "hbm_frac": round(gbs / HBM_PEAK_GBS, 4)}
        if valu and name + "_fill" in valu:
            r[name]["valu_instr_per_output_measured"] = valu[name + "_fill"]["valu_instr_per_output"]
        del out
        torch.cuda.empty_cache()
    return r


def counter_modes(sq, torch, key: int, ctr0: int, n: int, per_op_ms: dict) -> dict:
    """The counter modes of Section 4 beside the unit-step kernels: a squares32
    fill and F32 sum over n outputs whose counters are 3 apart, key-counter
    mode over 2^28 device-generated distinct-digit keys at counter 0 (U32 and
    U64 outputs; bytes counted are the 8-byte key read plus the output
    written), and the key generator itself."""
    step = 3
    out = torch.empty(n, dtype=torch.uint32, device="cuda")
    res, ws = sq.result_tensor(), sq.reduce_workspace(n)
    r = {}
    ms = _event_ms(torch, lambda: sq.fill_strided(sq.U32, key, ctr0, step, n, out=out))
    gbs = 4 * n / (ms * 1e-3) / 1e9
    r["strided_u32_fill"] = {"step": step, "n": n, "ms": round(ms, 4), "gnum_s": round(n / (ms * 1e-3) / 1e9, 1),
                             "gb_s": round(gbs, 1), "hbm_frac": round(gbs / HBM_PEAK_GBS, 4),
                             "vs_unit_step": round(per_op_ms["sq32_fill"] / ms, 3)}
    ms = _event_ms(torch, lambda: sq.reduce_strided_async(sq.F32, key, ctr0, step, n, res, ws))
    r["strided_f32_sum"] = {"step": step, "n": n, "ms": round(ms, 4), "gnum_s": round(n / (ms * 1e-3) / 1e9, 1),
                            "vs_unit_step": round(per_op_ms["fused_f32_sum"] / ms, 3)}
    del out
    torch.cuda.empty_cache()
    m = 1 << 28
    keys = torch.empty(m, dtype=torch.uint64, device="cuda")
    gen_key = 0x9E3779B97F4A7C15
    ms = _event_ms(torch, lambda: sq.make_keys(gen_key, 0, m, out=keys), reps=5)
    r["make_keys"] = {"m": m, "ms": round(ms, 4), "gkeys_s": round(m / (ms * 1e-3) / 1e9, 1)}
    kout = torch.empty(m, dtype=torch.uint64, device="cuda")
    for name, kind, W in (("key_counter_u32", sq.U32, 4), ("key_counter_u64", sq.U64, 8)):
        ms = _event_ms(torch, lambda: sq.fill_keys(kind, 0, keys, out=kout))
        gbs = (8 + W) * m / (ms * 1e-3) / 1e9
        r[name] = {"m": m, "ctr": 0, "ms": round(ms, 4), "gnum_s": round(m / (ms * 1e-3) / 1e9, 1),
                   "gb_s": round(gbs, 1), "hbm_frac": round(gbs / HBM_PEAK_GBS, 4)}
    del keys, kout
    torch.cuda.empty_cache()
    return r


def main() -> int:
    args = parse()
    if args.kernel_summary:
        print(kernel_summary(args.kernel_summary))
        return 0
    if args.valu:
        t = valu_from_pmc(args.valu, args.log2n)
        with open(os.path.join(ROOT, "profiles", "valu.json"), "w") as f:
            json.dump(t, f, indent=1)
        print(json.dumps(t))
        return 0
    if args.traffic:
        t = traffic_from_pmc(args.traffic[0], args.traffic[1], args.log2n)
        with open(os.path.join(ROOT, "profiles", "traffic.json"), "w") as f:
            json.dump(t, f, indent=1)
        print(json.dumps(t))
        return 0
    if args.gpus != 1 or int(os.environ.get("WORLD_SIZE", "1")) > 1:
        print("bench.py measures one GPU only: the library has no multi-GPU path "
              "(run with --gpus 1).", file=sys.stderr)
        return 2
    import torch

    from paper_2004_06278_amd import squares as sq
    from paper_2004_06278_amd import workloads as W

    assert torch.cuda.is_available(), "bench.py needs a GPU"
    torch.cuda.set_device(0)
    sq.check(sq.lib().sq_init())
    case = W.single_key_case()
    key, ctr0, n = case.key, case.ctr0, 1 << args.log2n

    if args.calib_copy:
        src = torch.empty(4 << 30, dtype=torch.uint8, device="cuda")
        dst = torch.empty_like(src)
        dst.copy_(src)
        torch.cuda.synchronize()
        del src, dst
        torch.cuda.empty_cache()

    out32 = torch.empty(n, dtype=torch.uint32, device="cuda")
    out64 = torch.empty(n, dtype=torch.uint64, device="cuda")
    res32, res64 = sq.result_tensor(), sq.result_tensor()
    ws32, ws64 = sq.reduce_workspace(n), sq.reduce_workspace(n)
    ops = [
        ("sq32_fill", lambda: sq.fill(sq.U32, key, ctr0, n, out=out32)),
        ("sq64_fill", lambda: sq.fill(sq.U64, key, ctr0, n, out=out64)),
        ("fused_f32_sum", lambda: sq.reduce_async(sq.F32, key, ctr0, n, res32, ws32)),
        ("fused_f64_sum", lambda: sq.reduce_async(sq.F64, key, ctr0, n, res64, ws64)),
    ]
    ev = {name: [] for name, _ in ops}

    def step(record: bool):
        for name, fn in ops:
            if record:
                a, b = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
                a.record()
                fn()
                b.record()
                ev[name].append((a, b))
            else:
                fn()

    mlib = measure_lib()
    est_ms = 1e30
    for _ in range(args.warmup):
        tw = time.perf_counter()
        step(False)
        torch.cuda.synchronize()
        est_ms = min(est_ms, (time.perf_counter() - tw) * 1e3)
    # The clock sampler runs on a side stream over the first ~70% of the timed
    # region (its length is fixed when it is launched, so it must end before
    # the timed steps do: the final device synchronisation waits for it).
    nsamp = 2048
    samples = torch.zeros(2 * nsamp, dtype=torch.int64, device="cuda")
    side = torch.cuda.Stream()
    window_ms = 0.7 * est_ms * args.steps
    sample_clock = args.warmup > 0 and window_ms < 10_000  # no estimate without warm-up steps
    if sample_clock:
        spacing = max(int(window_ms * 1e5 / nsamp), 100)  # 100 MHz ticks
        rc = mlib.sqm_clock_sampler(samples.data_ptr(), nsamp, spacing, side.cuda_stream)
        assert rc == 0, f"clock sampler launch failed ({rc})"
    t0 = time.perf_counter()
    for _ in range(args.steps):
        step(True)
    torch.cuda.synchronize()
    t1 = time.perf_counter()
    clock = clock_from_samples(samples.cpu().numpy()) if sample_clock else None
    ms_per_step = (t1 - t0) * 1e3 / args.steps
    per_op_ms = {name: sum(a.elapsed_time(b) for a, b in ev[name]) / len(ev[name]) for name in ev}
    per_op_sorted = {name: sorted(a.elapsed_time(b) for a, b in ev[name]) for name in ev}
    value = 4 * n / (ms_per_step * 1e-3) / 1e9

    # spot check of the timed outputs against the oracle (outside the timed region)
    from oracle import oracle
    import numpy as np

    idx = torch.tensor([0, 1, n // 3, n - 1], dtype=torch.int64, device="cuda")
    got32 = out32.view(torch.int32)[idx].cpu().numpy().view(np.uint32)
    got64 = out64.view(torch.int64)[idx].cpu().numpy().view(np.uint64)
    for i, g32, g64 in zip(idx.cpu().tolist(), got32, got64):
        assert int(g32) == oracle.squares32((ctr0 + i) % 2**64, key), "sq32 spot check failed"
        assert int(g64) == oracle.squares64((ctr0 + i) % 2**64, key), "sq64 spot check failed"
    s32, v32, _ = sq.read_result(res32)
    s64, v64, _ = sq.read_result(res64)
    assert abs(v32 / n - 0.5) < 1e-3 and abs(v64 / n - 0.5) < 1e-3

    # Store-only ceiling in exactly the squares64 fill's launch shape and size
    # (one 4 KiB chunk per workgroup, 256 lanes x one 16-byte store, 2^n x 8
    # bytes of constant data), back to back, outside the timed region.
    store_ms = _event_ms(torch, lambda: mlib.sqm_store_ceiling(out64.data_ptr(), 8 * n, 7,
                                                               torch.cuda.current_stream().cuda_stream),
                         reps=10, warm=3)
    store_gbs = 8 * n / (store_ms * 1e-3) / 1e9
    store_ceiling = {"ms": round(store_ms, 4), "gb_s": round(store_gbs, 1), "hbm_frac": round(store_gbs / HBM_PEAK_GBS, 4),
                     "kernel": "k_store_chunk (paper_2004_06278_amd/calib/sq_measure.hip)",
                     "shape": f"one 4 KiB chunk per workgroup, 256 lanes x one 16-byte global_store_dwordx4, "
                              f"2^{args.log2n} x 8 B, constant data, back to back"}
    valu_file = os.path.join(ROOT, "profiles", "valu.json")
    valu = {}
    if os.path.exists(valu_file):
        with open(valu_file) as f:
            vt = json.load(f)
        # counts taken on other kernel sources or another size do not apply
        if vt.get("source_sha") == kernel_source_sha() and vt.get("log2n") == args.log2n:
            valu = vt.get("kernels", {})

    def hbm_roof(name, nbytes, ms_by_op=per_op_ms):
        ms = ms_by_op[name]
        gbs = nbytes / (ms * 1e-3) / 1e9
        r = {"bound": "hbm", "achieved": round(gbs, 1), "peak": HBM_PEAK_GBS, "unit": "GB/s",
             "frac": round(gbs / HBM_PEAK_GBS, 4), "traffic": None,
             "kernel": name, "avg_ms": round(ms, 4), "algorithmic_bytes": nbytes,
             "measured_store_ceiling_gbs": round(store_gbs, 1)}
        if name in valu:
            r["valu_instr_per_output_measured"] = valu[name]["valu_instr_per_output"]
        return r

    def alu_roof(name, slots, ms_by_op=per_op_ms):
        ms = ms_by_op[name]
        rate = slots * n / (ms * 1e-3)
        r = {"bound": "alu", "achieved": round(rate / 1e12, 3), "peak": round(ALU_PEAK_SLOTS / 1e12, 3),
             "unit": "T VALU-slot/s", "frac": round(rate / ALU_PEAK_SLOTS, 4), "traffic": None,
             "kernel": name, "avg_ms": round(ms, 4), "slots_per_output": slots}
        if name in valu:
            # the same roofline from the executed instruction count (rocprofv3
            # SQ_INSTS_VALU), every VALU instruction counted as one issue slot
            v = valu[name]["valu_instr_per_output"]
            irate = v * n / (ms * 1e-3)
            r["measured"] = {"valu_instr_per_output": v, "achieved": round(irate / 1e12, 3),
                             "unit": "T VALU-instr/s", "frac": round(irate / ALU_PEAK_SLOTS, 4)}
        return r

    rooflines = {
        "sq32_fill": hbm_roof("sq32_fill", 4 * n),
        "sq64_fill": hbm_roof("sq64_fill", 8 * n),
        "fused_f32_sum": alu_roof("fused_f32_sum", SLOTS["sq32"] + SLOTS["sum_f32"]),
        "fused_f64_sum": alu_roof("fused_f64_sum", SLOTS["sq64"] + SLOTS["sum_f64"]),
    }
    # The same kernels repeated back to back (20 timed after 8 untimed): in the
    # step, a kernel that follows one of the other class meets the shader
    # clock of the other operating point, and the clock moves to its own over
    # tens of milliseconds (a dozen launches), so the warm-up covers that.
    steady_ms = {name: _event_ms(torch, fn, reps=20, warm=8) for name, fn in ops}
    rooflines_steady = {
        "sq32_fill": hbm_roof("sq32_fill", 4 * n, steady_ms),
        "sq64_fill": hbm_roof("sq64_fill", 8 * n, steady_ms),
        "fused_f32_sum": alu_roof("fused_f32_sum", SLOTS["sq32"] + SLOTS["sum_f32"], steady_ms),
        "fused_f64_sum": alu_roof("fused_f64_sum", SLOTS["sq64"] + SLOTS["sum_f64"], steady_ms),
    }
    dominant = max(per_op_ms, key=per_op_ms.get)
    traffic_file = os.path.join(ROOT, "profiles", "traffic.json")
    if os.path.exists(traffic_file):
        with open(traffic_file) as f:
            tr = json.load(f)
        # counters taken on other kernel sources or another size do not apply
        if tr.get("source_sha") == kernel_source_sha() and tr.get("log2n") == args.log2n:
            for k, r in rooflines.items():
                if k in tr.get("kernels", {}):
                    r["traffic"] = tr["kernels"][k]

    line = {
        "metric": "Gnum/s squares32/64 (fill vs fused) and % HBM/VALU roofline; batch speedup; p99",
        "value": round(value, 2),
        "unit": "Gnum/s",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": round(ms_per_step, 4),
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "u64",
        "data": "synthetic",
        "config": {"workload": f"single-key throughput: squares32+squares64 fill to HBM and fused "
                               f"f32/f64 exact sums, n=2^{args.log2n} each, one distinct-digit key, "
                               f"random 64-bit ctr0", "n": n, "key": hex(key), "ctr0": hex(ctr0),
                   "parallelism": "single GPU"},
        "per_kernel_gnum_s": {k: round(n / (v * 1e-3) / 1e9, 1) for k, v in per_op_ms.items()},
        "per_kernel_ms": {k: round(v, 4) for k, v in per_op_ms.items()},
        "per_kernel_median_min_ms": {k: [round(v[len(v) // 2], 4), round(v[0], 4)] for k, v in per_op_sorted.items()},
        "roofline": rooflines[dominant],
        "rooflines": rooflines,
        "rooflines_steady": rooflines_steady,
        "store_ceiling": store_ceiling,
        "clock_in_step": clock,
        "run": run_metadata(torch),
    }
    del out32, out64
    torch.cuda.empty_cache()
    extras = set() if args.no_extras else set(args.extras.split(","))
    if "concurrent" in extras:
        line["concurrent_step"] = concurrent_step(sq, torch, key, ctr0, n, ms_per_step)
    if "uniform" in extras:
        line["uniform_fills"] = uniform_fills(sq, torch, key, ctr0, n, valu)
    if "pair" in extras:
        line["paired_sums"] = paired_sums(sq, torch, key, ctr0, n, steady_ms)
    if "split" in extras:
        line["split_words"] = split_words(sq, torch, key, ctr0, n, per_op_ms)
    if "modes" in extras:
        line["counter_modes"] = counter_modes(sq, torch, key, ctr0, n, per_op_ms)
    if "batch" in extras:
        line["batch"] = batch_speedup(sq, torch, per_stream_baseline=not args.no_per_stream)
        if "batch_fill" in valu:
            line["batch"]["valu_instr_per_output_measured"] = valu["batch_fill"]["valu_instr_per_output"]
    if "batch_wrap" in extras:
        line["batch_wrap"] = batch_wrap_speedup(sq, torch)
    if "serving" in extras:
        from paper_2004_06278_amd import serve_bench

        line["serving"] = serve_bench.run_short(sq, torch)
    if not args.no_cpu:
        line["cpu_baseline"] = cpu_baseline(key, ctr0)
    print(json.dumps(line), flush=True)
    return 0


if __name__ == "__main__":
    sys.exit(main())
