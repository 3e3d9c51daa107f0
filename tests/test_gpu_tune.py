"""GPU test of the autotuner: a fill-only run on small scratch buffers writes a
table of valid configurations, and fills launched with the tuned table still
match the oracle.  The shipped table is restored afterwards."""
from __future__ import annotations

import json

import numpy as np
import pytest

from gpu_helpers import log

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
