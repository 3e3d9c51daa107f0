"""GPU parity of the fused exact reduce against the oracle's exact sum and its
round-to-nearest-even double."""
from __future__ import annotations

import numpy as np
import pytest

from gpu_helpers import HOST_THREADS, log

pytestmark = pytest.mark.gpu

KINDS = [0, 1, 2, 3, 4, 5]


@pytest.fixture(scope="module")
def sq():
    from paper_2004_06278_amd import squares

    squares.lib()
    return squares


@pytest.mark.parametrize("kind", KINDS)
def test_reduce_small_and_ragged(sq, oracle_mod, kind):
    g = np.random.Generator(np.random.PCG64(200 + kind))
    sizes = [0, 1, 2, 3, 63, 64, 65, 255, 256, 257, 1000, 65536 + 3, 1 << 20, (1 << 22) + 11]
    for n in sizes:
        key = int(g.integers(0, 2**64, dtype=np.uint64))
        ctr0 = 2**64 - int(g.integers(1, 1 << 21)) if n % 2 else int(g.integers(0, 2**64, dtype=np.uint64))
        log(f"reduce kind={kind} n={n} key={key:#x} ctr0={ctr0:#x}")
        s, v, nn = sq.reduce(kind, key, ctr0, n)
        ref = oracle_mod.exact_sum(kind, key, ctr0, n, threads=HOST_THREADS)
        assert s == ref, (n, s, ref)
        assert v == oracle_mod.rounded_value(kind, ref)
        assert nn == n


@pytest.mark.parametrize("kind", KINDS)
def test_reduce_every_config(sq, oracle_mod, kind):
    n = (1 << 21) + 77
    key, ctr0 = 0x51A8F3C2E9D07B64, 2**64 - 12345
    ref = oracle_mod.exact_sum(kind, key, ctr0, n, threads=HOST_THREADS)
    cfgs = [sq.cfg(256, u, g) for u in (1, 2, 4) for g in (1, 2, 8, 32, 64)]
    cfgs += [sq.cfg(256, u, g, 1, pl) for u in (1, 4) for g in (1, 8, 64) for pl in (6, 9, 12, 16)]
    for c in cfgs:
        log(f"reduce kind={kind} cfg={c.as_dict()}")
        s, v, _ = sq.reduce(kind, key, ctr0, n, launch_cfg=c)
        assert s == ref, c.as_dict()


@pytest.mark.parametrize("kind", KINDS)
def test_reduce_queue_order_small_and_ragged(sq, oracle_mod, kind):
    """The chunk-queue order (a resident grid taking chunks from a counter in
    the workspace) on sizes from 0 to a few chunks plus a ragged tail, twice
    in a row on the same workspace (the counter is reset by each call)."""
    g = np.random.Generator(np.random.PCG64(300 + kind))
    res, ws = sq.result_tensor(), sq.reduce_workspace()
    for n in (0, 1, 2, 3, 255, 256 * 64 - 1, 256 * 64 + 1, 1000003):
        key = int(g.integers(0, 2**64, dtype=np.uint64))
        ctr0 = 2**64 - int(g.integers(1, 1 << 20))
        ref = oracle_mod.exact_sum(kind, key, ctr0, n, threads=HOST_THREADS)
        for rep in range(2):
            c = sq.cfg(256, 4, 4, 1, 6)
            log(f"reduce queue kind={kind} n={n} rep={rep}")
            sq.reduce_async(kind, key, ctr0, n, res, ws, launch_cfg=c)
            s, v, nn = sq.read_result(res)
            assert s == ref and nn == n and v == oracle_mod.rounded_value(kind, ref)


@pytest.mark.parametrize("kind", KINDS)
def test_reduce_additive(sq, kind):
    """reduce[a, b) + reduce[b, c) == reduce[a, c), across the counter wrap."""
    key, a = 0x0F1E2D3C4B5A6978, 2**64 - 3_000_000
    whole, _, _ = sq.reduce(kind, key, a, 10_000_000)
    per_ctr = 2 if kind in (4, 5) else 1  # split kinds: a part starting at an even output starts a counter
    for b in (2, 2_999_998, 3_000_000, 7_777_778):
        l, _, _ = sq.reduce(kind, key, a, b)
        r, _, _ = sq.reduce(kind, key, (a + b // per_ctr) % 2**64, 10_000_000 - b)
        assert l + r == whole


@pytest.mark.parametrize("kind", [1, 3, 5])
def test_reduce_full_size_exact(sq, oracle_mod, kind):
    """The fused F32 / F64 consumers over n = 2^32 outputs from a random
    counter (the single-key workload), compared with the oracle's exact sum
    computed on all host threads."""
    from paper_2004_06278_amd import workloads as W

    c = W.single_key_case()
    n = 1 << 32
    log(f"full-size reduce kind={kind} key={c.key:#x} ctr0={c.ctr0:#x}")
    s, v, _ = sq.reduce(kind, c.key, c.ctr0, n)
    ref = oracle_mod.exact_sum(kind, c.key, c.ctr0, n, threads=HOST_THREADS)
    assert s == ref
    assert v == oracle_mod.rounded_value(kind, ref)
    # mean of uniforms on [0,1) over 2^32 draws
    assert abs(v / n - 0.5) < 1e-4


@pytest.mark.parametrize("kind", [1, 2, 4])
def test_reduce_past_2p32_counters(sq, oracle_mod, kind):
    """Sums over more than 2^32 counters (chunk and thread offsets past 32
    bits), ragged, with the counter passing 2^64 - 1 -> 0 near the end: equal
    to the oracle's exact sum.  The split kind sums 2^33 + 2^21 + 12345
    outputs (an odd count: the last counter's low word only)."""
    from paper_2004_06278_amd import workloads as W

    key = W.single_key_case().key
    counters = (1 << 32) + (1 << 20) + 12345
    n = 2 * counters - 1 if kind in (4, 5) else counters
    ctr0 = 2**64 - counters + 1000
    log(f"reduce past 2^32 counters kind={kind} key={key:#x} ctr0={ctr0:#x} n={n}")
    s, v, nn = sq.reduce(kind, key, ctr0, n)
    ref = oracle_mod.exact_sum(kind, key, ctr0, n, threads=HOST_THREADS)
    assert s == ref
    assert v == oracle_mod.rounded_value(kind, ref)
    assert nn == n


def test_reduce_pair_past_2p32_counters(sq, oracle_mod):
    """The paired F32 + F64 sums over 2^32 + 2^20 + 12345 counters equal the
    oracle's two exact sums."""
    from paper_2004_06278_amd import workloads as W

    key = W.single_key_case().key
    n = (1 << 32) + (1 << 20) + 12345
    ctr0 = 2**64 - n + 1000
    log(f"paired reduce past 2^32 counters key={key:#x} ctr0={ctr0:#x} n={n}")
    (s32, v32, _), (s64, v64, _) = sq.reduce_pair(1, key, ctr0, n)
    r32 = oracle_mod.exact_sum(1, key, ctr0, n, threads=HOST_THREADS)
    r64 = oracle_mod.exact_sum(3, key, ctr0, n, threads=HOST_THREADS)
    assert (s32, s64) == (r32, r64)
    assert (v32, v64) == (oracle_mod.rounded_value(1, r32), oracle_mod.rounded_value(3, r64))


def test_reduce_u64_carries(sq, oracle_mod):
    """A U64 sum over 2^24 outputs exceeds 2^64: the high word must carry."""
    key, ctr0, n = 0xC3A5C85C97CB3127, 99, 1 << 24
    s, v, _ = sq.reduce(2, key, ctr0, n)
    assert s == oracle_mod.exact_sum(2, key, ctr0, n, threads=HOST_THREADS)
    assert s > 2**64


def test_reduce_rejects_bad_workspace(sq):
    import torch

    res = sq.result_tensor()
    small = torch.empty(64, dtype=torch.uint8, device="cuda")
    with pytest.raises(sq.SquaresError) as e:
        sq.reduce_async(0, 1, 0, 100, res, small)
    assert e.value.status == -3
    with pytest.raises(sq.SquaresError) as e:
        sq.reduce_async(9, 1, 0, 100, res, sq.reduce_workspace())
    assert e.value.status == -1


# ---------------------------------------------------------------- paired sums
@pytest.mark.parametrize("kind32", [0, 1])
def test_reduce_pair_small_and_ragged(sq, oracle_mod, kind32):
    """The paired sum (U32+U64 or F32+F64 from one squares64 per counter)
    equals the oracle's two separate exact sums, which evaluate squares32
    and squares64 independently."""
    kind64 = kind32 + 2
    g = np.random.Generator(np.random.PCG64(300 + kind32))
    for n in [0, 1, 2, 63, 255, 256, 257, 1000, 65536 + 3, (1 << 20) + 1, (1 << 22) + 11]:
        key = int(g.integers(0, 2**64, dtype=np.uint64))
        ctr0 = 2**64 - int(g.integers(1, 1 << 21)) if n % 2 else int(g.integers(0, 2**64, dtype=np.uint64))
        log(f"reduce pair kind32={kind32} n={n} key={key:#x} ctr0={ctr0:#x}")
        (s32, v32, n32), (s64, v64, n64) = sq.reduce_pair(kind32, key, ctr0, n)
        ref32 = oracle_mod.exact_sum(kind32, key, ctr0, n, threads=HOST_THREADS)
        ref64 = oracle_mod.exact_sum(kind64, key, ctr0, n, threads=HOST_THREADS)
        assert (s32, s64) == (ref32, ref64), n
        assert v32 == oracle_mod.rounded_value(kind32, ref32) and v64 == oracle_mod.rounded_value(kind64, ref64)
        assert n32 == n64 == n


@pytest.mark.parametrize("kind32", [0, 1])
def test_reduce_pair_every_config_and_keys(sq, oracle_mod, kind32):
    n = (1 << 21) + 77
    kind64 = kind32 + 2
    for key in (0, 1, 2**63, 0x9E3779B97F4A7C15):
        ctr0 = 2**64 - 1000
        ref32 = oracle_mod.exact_sum(kind32, key, ctr0, n, threads=HOST_THREADS)
        ref64 = oracle_mod.exact_sum(kind64, key, ctr0, n, threads=HOST_THREADS)
        for u in (1, 2, 4):
            for gpc in (1, 8):
                for pl in (6, 8, 12):
                    c = sq.cfg(block=256, unroll=u, grid_per_cu=gpc, xcd_map=1, tile_log2=pl)
                    log(f"reduce pair kind32={kind32} key={key:#x} cfg={c.as_dict()}")
                    (s32, _, _), (s64, _, _) = sq.reduce_pair(kind32, key, ctr0, n, launch_cfg=c)
                    assert (s32, s64) == (ref32, ref64), (key, c.as_dict())


def test_reduce_pair_full_size_equals_separate_sums(sq, oracle_mod):
    """The single-key workload (n = 2^32): the paired F32+F64 sum equals the
    oracle's exact sums."""
    from paper_2004_06278_amd import workloads as W

    c = W.single_key_case()
    n = 1 << 32
    log(f"full-size reduce pair key={c.key:#x} ctr0={c.ctr0:#x}")
    (s32, v32, _), (s64, v64, _) = sq.reduce_pair(1, c.key, c.ctr0, n)
    assert s32 == oracle_mod.exact_sum(1, c.key, c.ctr0, n, threads=HOST_THREADS)
    assert s64 == oracle_mod.exact_sum(3, c.key, c.ctr0, n, threads=HOST_THREADS)
    assert v32 == oracle_mod.rounded_value(1, s32) and v64 == oracle_mod.rounded_value(3, s64)
