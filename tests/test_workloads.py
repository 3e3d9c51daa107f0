"""CPU checks of the seeded input generators: the shapes and properties each
workload promises (key digits, length ranges, packing, wrap proximity)."""
from __future__ import annotations

import numpy as np

from paper_2004_06278_amd import workloads as W


def _digits(k: int) -> list[int]:
    return [(k >> (60 - 4 * i)) & 15 for i in range(16)]


def test_keys_have_distinct_digit_halves_and_odd_last_digit():
    g = W.rng(123)
    keys = W.distinct_digit_keys(g, 5000)
    assert np.unique(keys).size == keys.size
    last = []
    for k in (int(v) for v in keys):
        d = _digits(k)
        assert len(set(d[:8])) == 8 and len(set(d[8:])) == 8
        assert d[15] % 2 == 1
        last.append(d[15])
    cnt = np.bincount(last, minlength=16)[1::2]
    assert cnt.min() > 5000 / 8 * 0.8  # every odd digit appears about equally often


def test_ragged_batch_shape():
    b = W.ragged_batch(seed=3, m=4096, misalign=True)
    assert b.m == 4096
    assert b.lens.min() >= 2**10 and b.lens.max() <= 2**24
    assert set(np.unique(b.kinds)) <= {W.U32, W.F32}
    ends = b.offs + b.lens * np.array([W.KIND_BYTES[int(k)] for k in b.kinds], dtype=np.uint64)
    order = np.argsort(b.offs)
    assert np.all(b.offs[order][1:] >= ends[order][:-1])  # no overlap
    assert np.all(b.offs % 4 == 0) and int(ends.max()) == b.arena_bytes
    mean = W.expected_log_uniform_mean(10, 24)
    assert abs(b.total_outputs / b.m / mean - 1) < 0.1


def test_wrap_batch_wraps_about_half():
    b = W.wrap_batch(seed=4, m=65536)
    d = (np.uint64(0) - b.ctr0s).astype(np.uint64)
    assert d.min() >= 1 and d.max() <= 2**16
    frac = float(np.mean(b.lens > d))
    assert 0.4 < frac < 0.6
    assert np.all(b.offs % 8 == 0)


def test_serve_trace_mix():
    t = W.serve_trace(seed=5, r=20000, qps=1000.0)
    is32 = np.isin(t.kinds, [W.U32, W.F32])
    assert abs(is32.mean() - 0.7) < 0.02
    assert t.sizes.min() >= 2**10 and t.sizes.max() <= 2**28
    gaps = np.diff(t.arrival_s)
    assert abs(gaps.mean() * 1000.0 - 1) < 0.05
