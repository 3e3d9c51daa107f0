"""GPU parity of the bulk fills (squares32/squares64, integer and uniform
kinds) against the CPU oracle, element by element."""
from __future__ import annotations

import numpy as np
import pytest

from gpu_helpers import HOST_THREADS, KIND_ALIGN, KIND_BYTES, first_diff, log, oracle_bytes, oracle_element, to_host_bytes

pytestmark = pytest.mark.gpu

KINDS = [0, 1, 2, 3, 4, 5]  # U32, F32, U64, F64, U32X2, F32X2


@pytest.fixture(scope="module")
def sq():
    import torch

    from paper_2004_06278_amd import squares

    squares.lib()
    assert torch.cuda.is_available()
    return squares


@pytest.mark.parametrize("kind", KINDS)
def test_fill_small_random_misaligned(sq, oracle_mod, kind):
    """Random keys, counters and lengths 0..5000 at element-aligned start
    offsets across a KiB inside a guarded buffer: outputs match the oracle and
    no byte outside [start, start + n*W) changes."""
    import torch

    g = np.random.Generator(np.random.PCG64(100 + kind))
    W, A = KIND_BYTES[kind], KIND_ALIGN[kind]
    buf = torch.empty(5000 * 8 + 2048, dtype=torch.uint8, device="cuda")
    for trial in range(60):
        n = int(g.integers(0, 5001)) if trial > 3 else [0, 1, 2, 3][trial]
        # start offsets across a whole KiB: the kernel writes a head of up to
        # 1024/W elements one by one before its first aligned KiB
        off = A * int(g.integers(0, 1024 // A + 2))
        key = int(g.integers(0, 2**64, dtype=np.uint64))
        ctr0 = int(g.integers(0, 2**64, dtype=np.uint64)) if trial % 3 else 2**64 - int(g.integers(1, 3000))
        log(f"fill kind={kind} trial={trial} n={n} off={off} key={key:#x} ctr0={ctr0:#x}")
        buf.fill_(0xAB)
        sq.fill_ptr(kind, key, ctr0, n, buf.data_ptr() + 64 + off)
        torch.cuda.synchronize()
        host = to_host_bytes(buf)
        got = host[64 + off: 64 + off + n * W]
        ref = oracle_bytes(oracle_mod, kind, key, ctr0, n)
        assert got.tobytes() == ref.tobytes(), first_diff(got, ref)
        assert np.all(host[: 64 + off] == 0xAB) and np.all(host[64 + off + n * W:] == 0xAB), "write outside range"


@pytest.mark.parametrize("kind", KINDS)
def test_fill_every_config(sq, oracle_mod, kind):
    """Every launch configuration the tuner may choose gives identical bits on
    a ragged size spanning many chunks (and a partial last chunk)."""
    n = 3 * (1 << 18) + 7
    key, ctr0 = 0xE3B0C44298FC1C14, 2**64 - 100000
    ref = oracle_bytes(oracle_mod, kind, key, ctr0, n)
    cfgs = [sq.cfg(b, u, 1, 2) for b in (64, 128, 256, 512, 1024) for u in (1, 2, 4, 8)]
    cfgs += [sq.cfg(b, u, g, x) for b in (64, 256, 1024) for u in (1, 4, 8) for g in (1, 4, 16, 64) for x in (0, 1)]
    for c in cfgs:
        log(f"fill kind={kind} cfg={c.as_dict()} n={n}")
        out = sq.fill(kind, key, ctr0, n, launch_cfg=c)
        got = to_host_bytes(out)
        assert got.tobytes() == ref.tobytes(), (c.as_dict(), first_diff(got, ref))


@pytest.mark.parametrize("kind", KINDS)
def test_fill_misaligned_every_order(sq, oracle_mod, kind):
    """Start offsets that leave a head before the first aligned KiB, under each
    chunk order and small and large workgroups: bytes equal the oracle's and
    nothing outside the range is written."""
    import torch

    W, A = KIND_BYTES[kind], KIND_ALIGN[kind]
    key, ctr0 = 0x2F8E5C1B7A3D9046, 2**64 - 40000
    buf = torch.empty(100000 * 8 + 4096, dtype=torch.uint8, device="cuda")
    cfgs = [sq.cfg(64, 4, 1, 2), sq.cfg(256, 1, 1, 2), sq.cfg(128, 8, 1, 2), sq.cfg(1024, 2, 1, 2),
            sq.cfg(256, 4, 4, 0), sq.cfg(1024, 8, 2, 1)]
    for n in (7, 1000, 70001):
        ref = oracle_bytes(oracle_mod, kind, key, ctr0, n)
        for off in (A, 1024 - A, 1024 + 3 * A):
            for c in cfgs:
                log(f"misaligned fill kind={kind} n={n} off={off} cfg={c.as_dict()}")
                buf.fill_(0x3C)
                sq.check(sq.lib().sq_fill_cfg(kind, key, ctr0, n, buf.data_ptr() + 64 + off, sq.ctypes.byref(c),
                                              sq._stream()))
                torch.cuda.synchronize()
                host = to_host_bytes(buf)
                got = host[64 + off: 64 + off + n * W]
                assert got.tobytes() == ref.tobytes(), (c.as_dict(), first_diff(got, ref))
                assert np.all(host[: 64 + off] == 0x3C) and np.all(host[64 + off + n * W:] == 0x3C)


@pytest.mark.parametrize("kind", KINDS)
def test_fill_lanes_shape_ragged_misaligned(sq, oracle_mod, kind):
    """Bodies of at least 2^22 16-byte vectors in the one-vector-per-lane
    shape (256 lanes, one chunk per workgroup) take the kernel that reads each
    lane's Weyl offset from its argument table: a ragged size (a partial last
    chunk and a tail of single elements) at start offsets that leave a head,
    with counters that wrap past 2^64, equals the oracle and writes nothing
    outside its range."""
    import torch

    W, A = KIND_BYTES[kind], KIND_ALIGN[kind]
    E = 16 // W
    n = E * ((1 << 22) + 3 * 256 + 3) + (E - 1)
    key, ctr0 = 0x7C1F4A9E3B5D2068, 2**64 - 5 * 10**6
    ref = oracle_bytes(oracle_mod, kind, key, ctr0, n)
    buf = torch.empty(n * W + 4096, dtype=torch.uint8, device="cuda")
    c = sq.cfg(256, 1, 1, 2)
    for off in (A, 1024 - A, 0):
        log(f"lanes-shape fill kind={kind} n={n} off={off}")
        buf.fill_(0x5E)
        sq.check(sq.lib().sq_fill_cfg(kind, key, ctr0, n, buf.data_ptr() + 1024 + off, sq.ctypes.byref(c),
                                      sq._stream()))
        torch.cuda.synchronize()
        host = to_host_bytes(buf)
        got = host[1024 + off: 1024 + off + n * W]
        assert got.tobytes() == ref.tobytes(), first_diff(got, ref)
        assert np.all(host[: 1024 + off] == 0x5E) and np.all(host[1024 + off + n * W:] == 0x5E)
    del buf
    torch.cuda.empty_cache()


def test_fill_and_reduce_replayed_from_a_captured_graph(sq, oracle_mod):
    """A squares32 fill large enough for the lane-table kernel (its lane
    offsets travel in the kernel arguments), a small squares64 fill and a
    fused F64 sum, captured once into a HIP graph and replayed three times
    with eager work and synchronisations in between: every replay equals the
    eager result, which equals the oracle's."""
    import torch

    key, ctr0 = 0x8F1BBCDCCA62C1D6, 2**64 - 3000
    n_big, n_small, n_sum = (1 << 24) + 5, 10007, 1 << 20
    ref_big = sq.fill(0, key, ctr0, n_big)
    ref_small = sq.fill(2, key, ctr0, n_small)
    ref_sum = sq.reduce(3, key, ctr0, n_sum)
    assert np.array_equal(ref_big.cpu().numpy().view(np.uint32),
                          oracle_mod.fill(0, key, ctr0, n_big, threads=HOST_THREADS))
    assert np.array_equal(ref_small.cpu().numpy().view(np.uint64), oracle_mod.fill(2, key, ctr0, n_small))
    big = torch.zeros_like(ref_big)
    small = torch.zeros_like(ref_small)
    res = sq.result_tensor()
    ws = sq.reduce_workspace(n_sum)
    torch.cuda.synchronize()
    g = torch.cuda.CUDAGraph()
    with torch.cuda.graph(g):
        sq.fill(0, key, ctr0, n_big, out=big)
        sq.fill(2, key, ctr0, n_small, out=small)
        sq.reduce_async(3, key, ctr0, n_sum, res, ws)
    for r in range(3):
        log(f"graph replay {r}")
        big.zero_()
        small.zero_()
        res.zero_()
        torch.cuda.synchronize()
        g.replay()
        torch.cuda.synchronize()
        assert torch.equal(big, ref_big), f"replay {r}: lane-table fill"
        assert torch.equal(small, ref_small), f"replay {r}: small fill"
        assert sq.read_result(res) == ref_sum, f"replay {r}: sum"
    del g, big, small


def test_invalid_arguments(sq):
    import torch

    buf = torch.zeros(64, dtype=torch.uint8, device="cuda")
    with pytest.raises(sq.SquaresError) as e:
        sq.fill_ptr(0, 1, 0, 4, buf.data_ptr() + 2)  # not 4-byte aligned
    assert e.value.status == -2
    with pytest.raises(sq.SquaresError) as e:
        sq.fill_ptr(2, 1, 0, 2, buf.data_ptr() + 4)  # not 8-byte aligned for u64
    assert e.value.status == -2
    with pytest.raises(sq.SquaresError) as e:
        sq.fill_ptr(4, 1, 0, 2, buf.data_ptr() + 4)  # split kinds write whole squares64 outputs
    assert e.value.status == -2
    with pytest.raises(sq.SquaresError) as e:
        sq.fill_ptr(7, 1, 0, 2, buf.data_ptr())  # unknown kind
    assert e.value.status == -1
    with pytest.raises(sq.SquaresError) as e:
        sq.fill_ptr(0, 1, 0, 2, 0)  # null with n > 0
    assert e.value.status == -1
    sq.fill_ptr(0, 1, 0, 0, 0)  # n == 0: no launch, OK
    with pytest.raises(sq.SquaresError):
        sq.fill(0, 1, 0, 16, launch_cfg=sq.cfg(block=96))
    # the binding refuses an output tensor too small for the call (the C ABI
    # takes a raw pointer and cannot check)
    with pytest.raises(ValueError):
        sq.fill(0, 1, 0, 11, out=torch.empty(10, dtype=torch.uint32, device="cuda"))
    with pytest.raises(ValueError):
        sq.sq64_fill(1, 0, 6, out=torch.empty(5, dtype=torch.uint64, device="cuda"))
    with pytest.raises(ValueError):
        sq.fill_strided(2, 1, 0, 3, 6, out=torch.empty(40, dtype=torch.uint8, device="cuda"))
    with pytest.raises(ValueError):
        sq.make_keys(1, 0, 9, out=torch.empty(8, dtype=torch.uint64, device="cuda"))


def test_argument_order_matches_paper_scalar(sq, oracle_mod):
    """The bulk calls take (key, ctr0); the paper's functions take (ctr, key):
    sq32_fill(key, ctr, 1)[0] == squares32(ctr, key)."""
    g = np.random.Generator(np.random.PCG64(7))
    for _ in range(20):
        ctr = int(g.integers(0, 2**64, dtype=np.uint64))
        key = int(g.integers(0, 2**64, dtype=np.uint64))
        a = int(sq.sq32_fill(key, ctr, 1).cpu().numpy()[0])
        b = int(sq.sq64_fill(key, ctr, 1).cpu().numpy()[0])
        assert a == oracle_mod.squares32(ctr, key)
        assert b == oracle_mod.squares64(ctr, key)


def test_named_entry_points(sq, oracle_mod):
    key, ctr0, n = 0x7A3C91E4B85D2F60, 12345, 10007
    for fn, kind in ((sq.sq32_fill, 0), (sq.uniform_f32, 1), (sq.sq64_fill, 2), (sq.uniform_f64, 3),
                     (sq.sq64x2_fill, 4), (sq.uniform_f32x2, 5)):
        out = fn(key, ctr0, n)
        assert to_host_bytes(out).tobytes() == oracle_bytes(oracle_mod, kind, key, ctr0, n).tobytes()


def test_plain_fill_64mib(sq, oracle_mod):
    """The 64 MiB squares32 fill (one distinct-digit key, counters 0..2^24-1)
    in full, plus squares64 on the same counters, the hi32 identity, and the
    split kind (the squares64 words, high words equal to squares32)."""
    from paper_2004_06278_amd import workloads as W

    c = W.plain_fill_case()
    log(f"plain fill key={c.key:#x} n={c.n}")
    u32 = sq.sq32_fill(c.key, c.ctr0, c.n).cpu().numpy()
    ref = oracle_mod.fill(0, c.key, c.ctr0, c.n, threads=HOST_THREADS)
    assert np.array_equal(u32, ref)
    u64 = sq.sq64_fill(c.key, c.ctr0, c.n).cpu().numpy()
    assert np.array_equal(u64 >> np.uint64(32), u32.astype(np.uint64))
    assert np.array_equal(u64, oracle_mod.fill(2, c.key, c.ctr0, c.n, threads=HOST_THREADS))
    x2 = sq.sq64x2_fill(c.key, c.ctr0, 2 * c.n).cpu().numpy()
    assert x2.tobytes() == u64.tobytes()
    assert np.array_equal(x2[1::2], u32)


@pytest.mark.parametrize("kind", [0, 4])
def test_fill_past_2p32_outputs(sq, oracle_mod, kind):
    """n = 2^32 + 2^17 + 3 outputs (16 GiB): output indices past 32 bits and
    byte offsets past 2^34.  The 2^16 outputs before index 2^32 and the whole
    ragged tail after it equal the oracle's, as do 2^12 random positions; the
    counter passes 2^64 - 1 -> 0 inside the tail."""
    import torch

    from paper_2004_06278_amd import workloads as W

    key = W.single_key_case().key
    n = (1 << 32) + (1 << 17) + 3
    per_ctr = 2 if kind in (4, 5) else 1            # outputs per counter
    wrap_at = (1 << 32) + 100                       # output index whose counter is 0
    ctr0 = (2**64 - wrap_at // per_ctr) % 2**64
    log(f"fill past 2^32 outputs kind={kind} key={key:#x} ctr0={ctr0:#x} n={n}")
    out = sq.fill(kind, key, ctr0, n)
    start = (1 << 32) - (1 << 16)                   # even: a split pair starts here
    got = to_host_bytes(out.view(torch.uint8)[start * 4: n * 4])
    want = oracle_bytes(oracle_mod, kind, key, (ctr0 + start // per_ctr) % 2**64, n - start)
    assert np.array_equal(got, want), first_diff(got, want)
    g = np.random.Generator(np.random.PCG64(57 + kind))
    idx = g.integers(0, n, size=1 << 12)
    iv = out.view(torch.int32)
    got = iv[torch.from_numpy(idx.astype(np.int64)).cuda()].cpu().numpy().view(np.uint8).reshape(-1, 4)
    for row, i in zip(got, idx):
        assert row.tobytes() == oracle_element(oracle_mod, kind, key, ctr0, int(i)), f"position {int(i)}"
    del out, iv
    torch.cuda.empty_cache()


@pytest.mark.parametrize("kind", KINDS)
def test_full_size_complete(sq, oracle_mod, kind):
    """Every one of the n = 2^32 outputs of the single-key workload (U32, F32
    and the split-word U32X2, F32X2: 16 GiB; U64 and F64: 32 GiB), in the
    benchmark's launch configuration, equals the oracle's: compared in chunks
    of 2^28 outputs, the oracle running on all host threads into a reused
    buffer (a split kind's chunk starts at counter ctr0 + base / 2)."""
    import torch

    from paper_2004_06278_amd import workloads as W

    c = W.single_key_case()
    n, chunk = 1 << 32, 1 << 28
    log(f"full-size complete compare kind={kind} key={c.key:#x} ctr0={c.ctr0:#x} n={n}")
    out = sq.fill(kind, c.key, c.ctr0, n)
    tdt = torch.int32 if KIND_BYTES[kind] == 4 else torch.int64
    ndt = {0: np.uint32, 1: np.float32, 2: np.uint64, 3: np.float64, 4: np.uint32, 5: np.float32}[kind]
    per_ctr = 2 if kind in (4, 5) else 1
    flat = out.view(tdt)
    host = torch.empty(chunk, dtype=tdt, pin_memory=True)
    ref = np.empty(chunk, dtype=ndt)
    for base in range(0, n, chunk):
        host.copy_(flat[base: base + chunk])
        oracle_mod.fill_into(kind, c.key, (c.ctr0 + base // per_ctr) % 2**64, ref, threads=HOST_THREADS)
        got = host.numpy()                      # compared as integers: bit equality, floats included
        want = ref.view(got.dtype)
        if not np.array_equal(got, want):
            bad = int(np.nonzero(got != want)[0][0])
            pytest.fail(f"first mismatch at output {base + bad}")
    del out, flat
    torch.cuda.empty_cache()


def test_fill_past_2p31_work_items(sq, oracle_mod):
    """n = 2^32 + 2^30 U64 outputs (40 GiB) in the default shape: one launch of
    10485760 workgroups of 256 lanes (2.7e9 work-items, past 2^31 and below
    the 2^32 a launch may hold).  The outputs around output 2^31 + 2^29, the
    first and last 2^14 and 2^12 random positions equal the oracle's."""
    import torch

    key, ctr0 = 0xC2B2AE3D27D4EB4F, 0x165667B19E3779F9
    n, k = (1 << 32) + (1 << 30), 1 << 14
    log(f"fill U64 n=2^32+2^30 key={key:#x} ctr0={ctr0:#x}")
    out = sq.fill(2, key, ctr0, n)
    mid = n // 2
    for a in (0, mid - k, n - k):
        got = out[a: a + (2 * k if a == mid - k else k)].cpu().numpy()
        ref = oracle_mod.fill(2, key, (ctr0 + a) % 2**64, got.size, threads=HOST_THREADS)
        assert np.array_equal(got, ref), f"block at {a}"
    g = np.random.Generator(np.random.PCG64(2032))
    idx = g.integers(0, n, size=1 << 12)
    got = out.view(torch.int64)[torch.from_numpy(idx.astype(np.int64)).cuda()].cpu().numpy().view(np.uint8)
    for row, i in zip(got.reshape(-1, 8), idx):
        assert row.tobytes() == oracle_element(oracle_mod, 2, key, ctr0, int(i)), f"position {int(i)}"
    del out
    torch.cuda.empty_cache()


def test_fill_2p33_u64_split_launches(sq, oracle_mod):
    """n = 2^33 U64 outputs (64 GiB) in the default shape (one 4 KiB chunk per
    256-lane workgroup) needs 2^24 workgroups, more than one launch of fewer
    than 2^32 work-items can hold, so the fill is split into two launches of
    2^23 chunks.  The 2^15 outputs around
    output 2^32, the first and last 2^14 and 2^12 random positions equal the
    oracle's."""
    import torch

    from paper_2004_06278_amd import workloads as W

    c = W.single_key_case(seed=21)
    n, k = 1 << 33, 1 << 14
    log(f"fill U64 n=2^33 key={c.key:#x} ctr0={c.ctr0:#x}")
    out = sq.fill(2, c.key, c.ctr0, n)
    for a in (0, (1 << 32) - k, n - k):
        got = out[a: a + (2 * k if a == (1 << 32) - k else k)].cpu().numpy()
        ref = oracle_mod.fill(2, c.key, (c.ctr0 + a) % 2**64, got.size, threads=HOST_THREADS)
        assert np.array_equal(got, ref), f"block at {a}"
    g = np.random.Generator(np.random.PCG64(2033))
    idx = g.integers(0, n, size=1 << 12)
    got = out.view(torch.int64)[torch.from_numpy(idx.astype(np.int64)).cuda()].cpu().numpy().view(np.uint8)
    for row, i in zip(got.reshape(-1, 8), idx):
        assert row.tobytes() == oracle_element(oracle_mod, 2, c.key, c.ctr0, int(i)), f"position {int(i)}"
    del out
    torch.cuda.empty_cache()
