"""Open-loop load generator for the continuous-batching server.

Requests (kind, key, ctr0, size) come from the seeded serving trace: sizes
log-uniform in [2^10, 2^28] outputs, 70% 32-bit (U32/F32) and 30% 64-bit
(U64/F64), Poisson arrivals.  The load generator submits each request at its
scheduled arrival time (busy-waiting in between), most with the discard
flag, so the server frees their output as soon as they complete; a sample
of the requests is kept and compared with plain fills after the run.
Latency is measured by the server from submit to completion, so it includes
queueing.

The server runs four tick lanes: HIP binds each stream to one of a few
hardware queues (four per process by default) when the stream first runs
work, so in a process whose other streams already hold queues, two lanes can
land on one queue and run one after the other; four lanes keep at least two
queues apart whatever else the process has run.
"""
from __future__ import annotations

import time

import numpy as np

from . import workloads as W


def saturated(sq, trace: W.ServeTrace, budget: int, chunk_cap: int, n_streams: int = 4) -> dict:
    """Throughput with every request submitted at once (closed system)."""
    with sq.Server(budget, max_slots=4096, chunk_cap=chunk_cap, n_streams=n_streams) as srv:
        t0 = time.perf_counter()
        for i in range(trace.r):
            srv.submit(int(trace.kinds[i]), int(trace.keys[i]), int(trace.ctr0s[i]), int(trace.sizes[i]),
                       sq.SERVE_DISCARD)
        while srv.stats()["completed"] < trace.r:
            time.sleep(0.0005)
        dt = time.perf_counter() - t0
        st = srv.stats()
    return {"requests": trace.r, "seconds": dt, "req_per_s": trace.r / dt,
            "gnum_s": st["outputs"] / dt / 1e9, "gb_s": st["bytes"] / dt / 1e9, "ticks": st["ticks"]}


def open_loop(sq, trace: W.ServeTrace, budget: int, chunk_cap: int, warmup: int, n_streams: int = 4,
              verify_every: int = 250, verify_cap_bytes: int = 8 << 30) -> dict:
    """Submits request i at trace.arrival_s[i] (busy-waiting in between); the
    first `warmup` requests are kept out of the server's latency statistics.
    Every `verify_every`-th measured request (while their outputs total at
    most `verify_cap_bytes`, so that holding them cannot starve admission) is
    submitted without the discard flag and counts in the statistics like the
    others; all other requests are discarded on completion.  After the run,
    outside the latency window, each kept output is compared bitwise with a
    plain fill of the same (kind, key, ctr0, n) on the device, then released.
    The load generator does nothing but submit, so it keeps to the schedule;
    the server measures each latency from submit() to completion, and the
    throughput window starts at the first measured submit."""
    import torch

    keep, kept_bytes = set(), 0
    for i in range(warmup, trace.r, verify_every):
        nb = int(trace.sizes[i]) * (8 if int(trace.kinds[i]) in (2, 3) else 4)
        if kept_bytes + nb <= verify_cap_bytes:
            keep.add(i)
            kept_bytes += nb
    kept = []
    lag_max = 0.0
    with sq.Server(budget, max_slots=4096, chunk_cap=chunk_cap, n_streams=n_streams) as srv:
        t0 = time.perf_counter()
        t_first = t0
        for i in range(trace.r):
            due = t0 + float(trace.arrival_s[i])
            while True:
                now = time.perf_counter()
                if now >= due:
                    break
            if i >= warmup:
                lag_max = max(lag_max, now - due)
            if i == warmup:
                t_first = now
            flags = (0 if i in keep else sq.SERVE_DISCARD) | (sq.SERVE_NO_STATS if i < warmup else 0)
            rid = srv.submit(int(trace.kinds[i]), int(trace.keys[i]), int(trace.ctr0s[i]), int(trace.sizes[i]), flags)
            if i in keep:
                kept.append((i, rid))
        while srv.stats()["completed"] < trace.r:
            time.sleep(0.0002)
        t_end = time.perf_counter()
        st = srv.stats()
        mismatches = 0
        for i, rid in kept:
            got = srv.result_bytes(rid)
            ref = sq.fill(int(trace.kinds[i]), int(trace.keys[i]), int(trace.ctr0s[i]), int(trace.sizes[i]))
            mismatches += not torch.equal(got, ref.view(torch.uint8))
            srv.release(rid)
            del got, ref
        torch.cuda.empty_cache()
    span = float(trace.arrival_s[-1] - trace.arrival_s[warmup])
    measured = trace.sizes[warmup:]
    bytes_ = sum(int(s) * (4 if k < 2 or k > 3 else 8) for s, k in zip(measured, trace.kinds[warmup:]))
    window = t_end - t_first
    return {"requests": trace.r - warmup, "qps_offered": (trace.r - warmup) / span if span > 0 else None,
            "p50_ms": st["p50_s"] * 1e3, "p90_ms": st["p90_s"] * 1e3, "p99_ms": st["p99_s"] * 1e3,
            "max_ms": st["max_s"] * 1e3, "mean_ms": st["mean_s"] * 1e3,
            "gnum_s": float(measured.sum()) / window / 1e9, "gb_s": bytes_ / window / 1e9,
            "driver_lag_max_ms": lag_max * 1e3, "ticks": st["ticks"],
            "verified": len(kept), "verified_bytes": kept_bytes, "verify_mismatches": int(mismatches)}


def run_short(sq, torch, budget: int = 32 << 30, chunk_cap: int = 1 << 24) -> dict:
    """Capacity with all requests queued at once, then open-loop runs at half
    and at 0.8 of that rate (each rate is stated in the result; 1000 warm-up
    plus 20000 measured requests each)."""
    cap_trace = W.serve_trace(seed=5, r=2000, qps=1e9)
    cap = saturated(sq, cap_trace, budget, chunk_cap)
    out = {"workload": "Poisson arrivals, sizes log-uniform 2^10..2^28 outputs, 70% 32-bit / 30% 64-bit",
           "hbm_budget_gib": budget >> 30, "chunk_cap": chunk_cap, "n_streams": 4,
           "saturated_req_per_s": round(cap["req_per_s"], 1), "saturated_gnum_s": round(cap["gnum_s"], 1)}
    for frac, seed in ((0.5, 6), (0.8, 7)):
        qps = frac * cap["req_per_s"]
        tr = W.serve_trace(seed=seed, r=21000, qps=qps)
        ol = open_loop(sq, tr, budget, chunk_cap, warmup=1000)
        torch.cuda.synchronize()
        row = {"qps": round(qps, 1), **{k: (round(v, 4) if isinstance(v, float) else v) for k, v in ol.items()}}
        if frac == 0.5:
            out.update(row)  # the half-capacity run is the headline row
        else:
            out["at_0.8_capacity"] = row
    return out
