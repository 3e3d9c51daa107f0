"""GPU tests of the autotuner: runs on small scratch buffers write a
table of valid configurations, and fills, sums and batches launched with the tuned table still
match the oracle.  The shipped table is restored afterwards."""
from __future__ import annotations

import json

import numpy as np
import pytest

from gpu_helpers import HOST_THREADS, log, to_host_bytes

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def sq():
    from paper_2004_06278_amd import squares

    squares.lib()
    return squares


def test_autotune_fill_table_valid_and_exact(sq, oracle_mod, tmp_path):
    import torch

    path = str(tmp_path / "tuned.json")
    log("autotune fill, max 32 MiB")
    try:
        sq.autotune(1 << sq.OP_FILL, 32 << 20, path)
        with open(path) as f:
            rows = json.load(f)
        fills = [r for r in rows if r["op"] == sq.OP_FILL]
        assert len(fills) == 6 * 5  # every kind and size bucket
        assert sq.lib().sq_tune_load(path.encode()) == 0  # every row passes the library's validity check
        key = 0x9E3779B97F4A7C15
        for kind in range(6):
            for n in (1000, (1 << 20) + 7, (1 << 22) + 3):
                got = sq.fill(kind, key, 2**64 - 100, n).view(torch.uint8).cpu().numpy()
                ref = oracle_mod.fill(kind, key, 2**64 - 100, n).view(np.uint8)
                assert got.tobytes() == ref.tobytes(), (kind, n)
    finally:
        assert sq.lib().sq_tune_load(sq.TUNE_TABLE.encode()) == 0


def test_autotune_reduce_and_batch_table_valid_and_exact(sq, oracle_mod, tmp_path):
    """The reduce and batch phases of the tuner: every (kind, bucket) gets a
    valid configuration, and sums and batches launched with the tuned table
    equal the oracle's."""
    from paper_2004_06278_amd import workloads as W

    path = str(tmp_path / "tuned_rb.json")
    log("autotune reduce + batch, max 64 MiB")
    try:
        sq.autotune((1 << sq.OP_REDUCE) | (1 << sq.OP_BATCH), 64 << 20, path)
        with open(path) as f:
            rows = json.load(f)
        assert len([r for r in rows if r["op"] == sq.OP_REDUCE]) == 6 * 5
        assert len([r for r in rows if r["op"] == sq.OP_BATCH]) >= 6
        assert sq.lib().sq_tune_load(path.encode()) == 0
        key = 0x9E3779B97F4A7C15
        for kind in range(6):
            for n in (1000, (1 << 20) + 7, (1 << 25) + 3):
                s, v, _ = sq.reduce(kind, key, 2**64 - 100, n)
                ref = oracle_mod.exact_sum(kind, key, 2**64 - 100, n, threads=HOST_THREADS)
                assert s == ref and v == oracle_mod.rounded_value(kind, ref), (kind, n)
        b = W.small_random_batch(seed=13, m=120, max_len=40000, kinds=(0, 1, 2, 3, 4, 5))
        db = sq.batch_to_device(b.keys, b.ctr0s, b.lens, b.offs, b.kinds, b.arena_bytes)
        sq.fill_batch(db)
        got = to_host_bytes(db.out)[: b.arena_bytes]
        ref = oracle_mod.fill_batch(b.keys, b.ctr0s, b.lens, b.offs, b.kinds, b.arena_bytes)
        assert got.tobytes() == ref.tobytes()
    finally:
        assert sq.lib().sq_tune_load(sq.TUNE_TABLE.encode()) == 0


def test_acceptance_check_rejects_partial_output():
    """The tuner accepts a candidate only if a run of it alone, into a
    poisoned buffer, reproduces the reference: shapes that write every byte
    pass, runs that skip the first or last output, write half, or write
    nothing (fills and sums) are rejected (tests/tune_check.hip)."""
    import os
    import subprocess

    exe = os.path.join(os.path.dirname(os.path.abspath(__file__)), "tune_check")
    assert os.path.exists(exe), "tests/tune_check is not built (run __graft_entry__.build())"
    log("tune_check program")
    r = subprocess.run([exe], capture_output=True, text=True, timeout=120)
    print(r.stdout)
    assert r.returncode == 0, r.stdout + r.stderr
    assert r.stdout.strip().endswith("ok")
