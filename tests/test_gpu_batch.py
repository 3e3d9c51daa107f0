"""GPU parity of the ragged batch (tile scan + persistent kernel), its graph
plan, and descriptor validation."""
from __future__ import annotations

import numpy as np
import pytest

from gpu_helpers import HOST_THREADS, KIND_BYTES, compare_batch_arena, first_diff, log, to_host_bytes

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def sq():
    from paper_2004_06278_amd import squares

    squares.lib()
    return squares


def _oracle_arena(o, b):
    return o.fill_batch(b.keys, b.ctr0s, b.lens, b.offs, b.kinds, b.arena_bytes)


@pytest.mark.parametrize("seed", [1, 2, 3])
def test_batch_small_random(sq, oracle_mod, seed):
    """Mixed kinds, empty streams, misaligned starts, counters near 2^64,
    zero and even keys; several tile sizes so streams span many tiles."""
    from paper_2004_06278_amd import workloads as W

    b = W.small_random_batch(seed=seed, m=300, max_len=20000, kinds=(0, 1, 2, 3, 4, 5))
    ref = _oracle_arena(oracle_mod, b)
    db = sq.batch_to_device(b.keys, b.ctr0s, b.lens, b.offs, b.kinds, b.arena_bytes)
    cfgs = [sq.cfg(block=blk, grid_per_cu=gpc, tile_log2=tl) for tl in (12, 13, 16, 24) for blk in (256, 1024)
            for gpc in (1, 8)]
    cfgs += [sq.cfg(block=blk, grid_per_cu=1, xcd_map=2, tile_log2=tl) for tl in (10, 11, 12, 14)
             for blk in (64, 128, 256)]
    cfgs += [sq.cfg(block=blk, grid_per_cu=gpc, xcd_map=1, tile_log2=tl) for tl in (10, 12, 14, 16)
             for blk in (64, 256, 1024) for gpc in (1, 4)]
    cfgs += [sq.cfg(block=blk, unroll=u, grid_per_cu=2, xcd_map=o, tile_log2=tl) for u in (1, 2, 4)
             for o in (0, 1) for tl in (11, 15) for blk in (64, 256)]
    for c in cfgs:
        log(f"batch seed={seed} m={b.m} cfg={c.as_dict()}")
        db.out.zero_()
        sq.fill_batch(db, launch_cfg=c)
        got = to_host_bytes(db.out)[: b.arena_bytes]
        assert got.tobytes() == ref.tobytes(), (c.as_dict(), first_diff(got, ref))
        assert sq.batch_errors(db) == 0


def test_batch_equals_per_stream_fills(sq):
    """Each stream of a batch is bit-identical to a standalone sq_fill of the
    same (kind, key, ctr0, len)."""
    import torch

    from paper_2004_06278_amd import workloads as W

    b = W.small_random_batch(seed=9, m=150, max_len=50000, kinds=(0, 1, 2, 3, 4, 5))
    db = sq.batch_to_device(b.keys, b.ctr0s, b.lens, b.offs, b.kinds, b.arena_bytes)
    sq.fill_batch(db)
    arena = to_host_bytes(db.out)
    for s in range(b.m):
        k, L, off = int(b.kinds[s]), int(b.lens[s]), int(b.offs[s])
        if L == 0:
            continue
        alone = sq.fill(k, int(b.keys[s]), int(b.ctr0s[s]), L)
        assert to_host_bytes(alone).tobytes() == arena[off: off + L * KIND_BYTES[k]].tobytes(), s
    torch.cuda.synchronize()


def test_batch_stream_past_2p32_outputs(sq, oracle_mod):
    """A batch whose middle stream holds 2^32 + 3 * 2^14 + 7 U32 outputs (16
    GiB: tile offsets inside the stream past 32 bits; its counter wraps 200
    outputs after index 2^32) between a short F32 stream at a misaligned
    start and a short F64 stream: the short streams whole, the big stream's
    outputs from index 2^32 - 2^16 to its end and 2^12 random positions of it
    equal the oracle's."""
    import torch

    from paper_2004_06278_amd import workloads as W

    big = (1 << 32) + 3 * (1 << 14) + 7
    keys = np.array([0x1234567890ABCDEF, W.single_key_case().key, 0xFEDCBA0987654321], dtype=np.uint64)
    ctr0s = np.array([5, 2**64 - (1 << 32) - 200, 2**64 - 3], dtype=np.uint64)
    lens = np.array([1001, big, 4099], dtype=np.uint64)
    kinds = np.array([1, 0, 3], dtype=np.uint8)
    o0 = 4
    o1 = o0 + 1001 * 4
    o2 = (o1 + big * 4 + 7) & ~7
    offs = np.array([o0, o1, o2], dtype=np.uint64)
    arena_bytes = o2 + 4099 * 8
    log(f"batch with a stream past 2^32 outputs: lens={lens.tolist()} offs={offs.tolist()}")
    db = sq.batch_to_device(keys, ctr0s, lens, offs, kinds, arena_bytes)
    sq.fill_batch(db)
    assert sq.batch_errors(db) == 0
    got0 = to_host_bytes(db.out[o0: o0 + 1001 * 4])
    assert np.array_equal(got0, oracle_mod.fill(1, int(keys[0]), 5, 1001).view(np.uint8))
    got2 = to_host_bytes(db.out[o2: o2 + 4099 * 8])
    assert np.array_equal(got2, oracle_mod.fill(3, int(keys[2]), 2**64 - 3, 4099).view(np.uint8))
    start = (1 << 32) - (1 << 16)
    tail = to_host_bytes(db.out[o1 + start * 4: o1 + big * 4])
    want = oracle_mod.fill(0, int(keys[1]), (int(ctr0s[1]) + start) % 2**64, big - start,
                           threads=HOST_THREADS).view(np.uint8)
    assert np.array_equal(tail, want), first_diff(tail, want)
    g = np.random.Generator(np.random.PCG64(91))
    idx = g.integers(0, big, size=1 << 12)
    iv = db.out[o1: o1 + big * 4].view(torch.int32)
    got = iv[torch.from_numpy(idx.astype(np.int64)).cuda()].cpu().numpy().view(np.uint32)
    for v, i in zip(got, idx):
        assert v == oracle_mod.fill(0, int(keys[1]), (int(ctr0s[1]) + int(i)) % 2**64, 1)[0], f"position {int(i)}"
    del db, iv
    torch.cuda.empty_cache()


def test_batch_one_tile_per_workgroup_grid_cap(sq, oracle_mod):
    """One tile per workgroup with 4 KiB tiles and 1024-lane workgroups over a
    16 GiB stream: the tile bound (2^22 + 2 tiles) times 1024 lanes passes
    2^32 work-items, so the grid is capped and workgroups stride over the
    remaining tiles.  The arena equals the
    plain fill of the same stream, and its last 2^12 and 2^12 random outputs
    equal the oracle's."""
    import torch

    n, key, ctr0 = (1 << 32) + 1000, 0x6A09E667F3BCC909, 0xBB67AE8584CAA73B
    log(f"batch one tile per workgroup, grid cap: n={n}")
    db = sq.batch_to_device(np.array([key], dtype=np.uint64), np.array([ctr0], dtype=np.uint64),
                            np.array([n], dtype=np.uint64), np.array([0], dtype=np.uint64),
                            np.array([0], dtype=np.uint8), 4 * n)
    sq.fill_batch(db, launch_cfg=sq.cfg(block=1024, unroll=1, grid_per_cu=1, xcd_map=2, tile_log2=10))
    assert sq.batch_errors(db) == 0
    got = db.out[: 4 * n].view(torch.int32)
    ref = sq.fill(0, key, ctr0, n).view(torch.int32)
    assert torch.equal(got, ref)
    del ref
    g = np.random.Generator(np.random.PCG64(92))
    idx = np.unique(np.concatenate([n - 1 - np.arange(1 << 12), g.integers(0, n, size=1 << 12)])).astype(np.int64)
    vals = got[torch.from_numpy(idx).cuda()].cpu().numpy().view(np.uint32)
    want = np.array([oracle_mod.fill(0, key, (ctr0 + int(i)) % 2**64, 1)[0] for i in idx], dtype=np.uint32)
    assert np.array_equal(vals, want)
    del db, got
    torch.cuda.empty_cache()


def test_per_stream_launches_equal_oracle_and_batch(sq, oracle_mod):
    """sq_fill_streams (one fill launch per stream, the batch's baseline)
    writes the oracle's arena, byte for byte the same as sq_fill_batch, for
    every kind at misaligned offsets, with empty streams and wrapping
    counters."""
    import torch

    from paper_2004_06278_amd import workloads as W

    b = W.small_random_batch(seed=12, m=200, max_len=30000, kinds=(0, 1, 2, 3, 4, 5))
    ref = _oracle_arena(oracle_mod, b)
    log(f"per-stream launches m={b.m} arena={b.arena_bytes}")
    db = sq.batch_to_device(b.keys, b.ctr0s, b.lens, b.offs, b.kinds, b.arena_bytes)
    sq.fill_streams(b.keys, b.ctr0s, b.lens, b.offs, b.kinds, db.out, b.arena_bytes)
    streams = to_host_bytes(db.out)[: b.arena_bytes]
    assert streams.tobytes() == ref.tobytes(), first_diff(streams, ref)
    db.out.zero_()
    sq.fill_batch(db)
    batch = to_host_bytes(db.out)[: b.arena_bytes]
    assert batch.tobytes() == streams.tobytes(), first_diff(batch, streams)
    torch.cuda.synchronize()


def test_batch_invalid_descriptors_skipped(sq, oracle_mod):
    """Streams with an unknown kind, a misaligned offset or a range past the
    arena are skipped (nothing written) and counted; valid ones are exact."""
    keys = np.array([11, 12, 13, 14, 15], dtype=np.uint64)
    ctr0s = np.array([0, 5, 9, 2**64 - 3, 7], dtype=np.uint64)
    lens = np.array([100, 100, 100, 100, 10**9], dtype=np.uint64)
    kinds = np.array([0, 9, 2, 3, 1], dtype=np.uint8)
    offs = np.array([0, 512, 1028, 2048, 4096], dtype=np.uint64)  # stream 2 (u64) misaligned, 4 too long
    arena = 8192
    db = sq.batch_to_device(keys, ctr0s, lens, offs, kinds, arena)
    db.out.fill_(0xCD)
    sq.fill_batch(db)
    host = to_host_bytes(db.out)
    assert sq.batch_errors(db) == 3
    ref0 = oracle_mod.fill(0, 11, 0, 100).view(np.uint8)
    ref3 = oracle_mod.fill(3, 14, 2**64 - 3, 100).view(np.uint8)
    assert host[0:400].tobytes() == ref0.tobytes()
    assert host[2048:2848].tobytes() == ref3.tobytes()
    untouched = np.ones(arena, dtype=bool)
    untouched[0:400] = False
    untouched[2048:2848] = False
    assert np.all(host[:arena][untouched] == 0xCD)


def test_batch_graph_plan_replays_current_descriptors(sq, oracle_mod):
    """A captured plan replays with whatever the descriptor arrays hold at
    launch time; every replay equals the eager batch."""
    import torch

    from paper_2004_06278_amd import workloads as W

    b1 = W.small_random_batch(seed=21, m=64, max_len=30000, misalign=False)
    b2 = W.small_random_batch(seed=22, m=64, max_len=30000, misalign=False)
    size = max(b1.arena_bytes, b2.arena_bytes)
    db = sq.batch_to_device(b1.keys, b1.ctr0s, b1.lens, b1.offs, b1.kinds, size)
    plan = sq.BatchPlan(db)
    for rep, b in enumerate([b1, b2, b1, b2]):
        log(f"plan replay {rep}")
        for dst, src in ((db.keys, b.keys), (db.ctr0s, b.ctr0s), (db.lens, b.lens), (db.offs, b.offs)):
            dst.copy_(torch.from_numpy(np.ascontiguousarray(src).view(np.int64)))
        db.kinds.copy_(torch.from_numpy(b.kinds))
        db.out.zero_()
        torch.cuda.synchronize()
        plan.launch()
        torch.cuda.synchronize()
        got = to_host_bytes(db.out)[: b.arena_bytes]
        ref = _oracle_arena(oracle_mod, b)
        assert got.tobytes() == ref.tobytes(), first_diff(got, ref)
    plan.close()


def test_batch_wrap_and_width_stress_full(sq, oracle_mod):
    """65536 squares64 streams, lengths 1..65536, counters starting within 2^16
    of 2^64 (about half wrap to 0), U64 and F64 outputs: every output compared."""
    import torch

    from paper_2004_06278_amd import workloads as W

    b = W.wrap_batch()
    log(f"wrap stress m={b.m} outputs={b.total_outputs} bytes={b.arena_bytes}")
    wraps = int(np.sum(b.lens > (np.uint64(0) - b.ctr0s)))
    assert wraps > b.m // 3
    db = sq.batch_to_device(b.keys, b.ctr0s, b.lens, b.offs, b.kinds, b.arena_bytes)
    sq.fill_batch(db)
    torch.cuda.synchronize()
    assert sq.batch_errors(db) == 0
    errors = compare_batch_arena(oracle_mod, db.out, b)
    assert not errors, errors[:5]
    del db
    torch.cuda.empty_cache()


@pytest.mark.parametrize("misalign", [False, True])
def test_batch_ragged_4096_complete(sq, oracle_mod, misalign):
    """The 4096-key ragged workload (lengths log-uniform in [2^10, 2^24], U32/F32,
    uniform counters; streams packed back to back or at random 4-byte gaps), in
    the launch configuration the benchmark's graph plan uses: every output of
    every stream equals the oracle's."""
    import torch

    from paper_2004_06278_amd import workloads as W

    b = W.ragged_batch(misalign=misalign)
    log(f"ragged m={b.m} outputs={b.total_outputs} bytes={b.arena_bytes} misalign={misalign}")
    db = sq.batch_to_device(b.keys, b.ctr0s, b.lens, b.offs, b.kinds, b.arena_bytes)
    plan = sq.BatchPlan(db)
    plan.launch()
    torch.cuda.synchronize()
    plan.close()
    assert sq.batch_errors(db) == 0
    errors = compare_batch_arena(oracle_mod, db.out, b)
    assert not errors, errors[:5]
    del db
    torch.cuda.empty_cache()
