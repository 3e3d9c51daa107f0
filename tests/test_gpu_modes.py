"""GPU parity of the counter modes beyond the unit-step fill: counter
increments other than one (fill and fused sum), key-counter mode (fixed
counter, one output per key) and on-device distinct-digit key generation,
each against the CPU oracle."""
from __future__ import annotations

import numpy as np
import pytest

from gpu_helpers import KIND_ALIGN, KIND_BYTES, first_diff, log, to_host_bytes

pytestmark = pytest.mark.gpu

KINDS = [0, 1, 2, 3, 4, 5]
M64 = 2**64 - 1


@pytest.fixture(scope="module")
def sq():
    import torch

    from paper_2004_06278_amd import squares

    squares.lib()
    assert torch.cuda.is_available()
    return squares


def _steps(g):
    return [0, 2, 3, 7, 2**32 + 1, M64, int(g.integers(2, 2**64, dtype=np.uint64))]


# ---------------------------------------------------------------- strided fill
@pytest.mark.parametrize("kind", KINDS)
def test_strided_fill_small_misaligned(sq, oracle_mod, kind):
    """Steps 0, 2, 3, 7, 2^32+1, 2^64-1 and a random one; lengths spanning the
    1 KiB head, several chunks and a ragged tail; start offsets across a KiB in
    a guarded buffer: bytes equal the oracle's, nothing outside is written."""
    import torch

    g = np.random.Generator(np.random.PCG64(500 + kind))
    W, A = KIND_BYTES[kind], KIND_ALIGN[kind]
    buf = torch.empty(70000 * 8 + 4096, dtype=torch.uint8, device="cuda")
    for step in _steps(g):
        for trial in range(6):
            n = [0, 1, 5, 1023, 65536 + 3, int(g.integers(0, 70000))][trial]
            off = A * int(g.integers(0, 1024 // A + 2))
            key = int(g.integers(0, 2**64, dtype=np.uint64))
            ctr0 = 2**64 - int(g.integers(1, 5000)) if trial % 2 else int(g.integers(0, 2**64, dtype=np.uint64))
            log(f"strided kind={kind} step={step:#x} n={n} off={off} key={key:#x} ctr0={ctr0:#x}")
            buf.fill_(0x5A)
            out_addr = buf.data_ptr() + 64 + off
            sq.check(sq.lib().sq_fill_strided(kind, key, ctr0, step, n, out_addr, sq._stream()))
            torch.cuda.synchronize()
            host = to_host_bytes(buf)
            got = host[64 + off: 64 + off + n * W]
            ref = oracle_mod.fill_strided(kind, key, ctr0, step, n).view(np.uint8)
            assert got.tobytes() == ref.tobytes(), first_diff(got, ref)
            assert np.all(host[: 64 + off] == 0x5A) and np.all(host[64 + off + n * W:] == 0x5A)


@pytest.mark.parametrize("kind", KINDS)
def test_strided_fill_every_config(sq, oracle_mod, kind):
    n = (1 << 19) + 13
    key, ctr0, step = 0x3C6EF372FE94F82B, 2**64 - 77777, 0x10001
    ref = oracle_mod.fill_strided(kind, key, ctr0, step, n).view(np.uint8)
    cfgs = [sq.cfg(b, u, 1, 2) for b in (64, 256, 1024) for u in (1, 2, 4, 8)]
    cfgs += [sq.cfg(b, u, g, x) for b in (256, 1024) for u in (4, 8) for g in (1, 16) for x in (0, 1)]
    for c in cfgs:
        log(f"strided kind={kind} cfg={c.as_dict()}")
        got = to_host_bytes(sq.fill_strided(kind, key, ctr0, step, n, launch_cfg=c))
        assert got.tobytes() == ref.tobytes(), (c.as_dict(), first_diff(got, ref))


@pytest.mark.parametrize("kind", KINDS)
def test_strided_step_one_is_the_fill(sq, kind):
    key, ctr0, n = 0xA54FF53A5F1D36F1, 2**64 - 1000, 100003
    a = to_host_bytes(sq.fill_strided(kind, key, ctr0, 1, n))
    b = to_host_bytes(sq.fill(kind, key, ctr0, n))
    assert a.tobytes() == b.tobytes()


@pytest.mark.parametrize("kind", [0, 1, 2, 3, 4, 5])
def test_strided_lanes_shape_complete(sq, oracle_mod, kind):
    """A strided fill of at least 2^22 16-byte vectors in the one-vector-per-
    lane shape (the lane-table kernel), ragged and with counters wrapping past
    2^64, for a small step and one above 2^32: every output equals the
    oracle's."""
    E = 16 // KIND_BYTES[kind]
    n = E * ((1 << 22) + 5 * 256 + 1) + (E - 1)
    key = 0x3D9B1F6A58C2E407
    c = sq.cfg(256, 1, 1, 2)
    for step, ctr0 in ((3, 2**64 - 7 * 10**6), (2**32 + 1, 0x9E3779B97F4A7C15)):
        log(f"strided lanes-shape kind={kind} step={step:#x} n={n}")
        got = to_host_bytes(sq.fill_strided(kind, key, ctr0, step, n, launch_cfg=c))
        ref = oracle_mod.fill_strided(kind, key, ctr0, step, n).view(np.uint8)
        assert got.tobytes() == ref.tobytes(), first_diff(got, ref)


def test_strided_large_sampled(sq, oracle_mod):
    """2^28 squares32 outputs with step 3 from a random counter: first, last and
    4096 random outputs equal the oracle's."""
    import torch

    key, ctr0, step, n = 0x9B05688C2B3E6C1F, 0xD1B54A32D192ED03, 3, 1 << 28
    log(f"strided large n={n}")
    out = sq.fill_strided(0, key, ctr0, step, n)
    g = np.random.Generator(np.random.PCG64(9))
    idx = np.unique(np.concatenate([np.arange(64), n - 1 - np.arange(64), g.integers(0, n, 4096)]))
    got = out.view(torch.int32)[torch.from_numpy(idx.astype(np.int64)).cuda()].cpu().numpy().view(np.uint32)
    ref = np.array([oracle_mod.squares32((ctr0 + int(i) * step) % 2**64, key) for i in idx], dtype=np.uint32)
    assert np.array_equal(got, ref)
    del out
    torch.cuda.empty_cache()


# ---------------------------------------------------------------- strided sum
def _strided_exact_sum(o, kind: int, key: int, ctr0: int, step: int, n: int) -> int:
    """Exact integer sum of the kind's terms over a strided range, from the
    oracle's raw outputs: U32/U64 words, shifted right by 8 (F32, F32X2) or
    11 (F64) as the kind's scale says, summed as split 32-bit halves so no
    partial sum can overflow."""
    base = {0: 0, 1: 0, 2: 2, 3: 2, 4: 4, 5: 4}[kind]
    w = o.fill_strided(base, key, ctr0, step, n).astype(np.uint64)
    w = w >> np.uint64({1: 8, 5: 8, 3: 11}.get(kind, 0))
    hi = int((w >> np.uint64(32)).sum(dtype=np.uint64))
    lo = int((w & np.uint64(0xFFFFFFFF)).sum(dtype=np.uint64))
    return (hi << 32) + lo


@pytest.mark.parametrize("kind", KINDS)
def test_strided_reduce(sq, oracle_mod, kind):
    g = np.random.Generator(np.random.PCG64(700 + kind))
    for step in _steps(g):
        for n in (0, 1, 2, 3, 255, 1000, 65536 + 5):
            key = int(g.integers(0, 2**64, dtype=np.uint64))
            ctr0 = 2**64 - int(g.integers(1, 3000)) if n % 2 else int(g.integers(0, 2**64, dtype=np.uint64))
            log(f"strided reduce kind={kind} step={step:#x} n={n} key={key:#x} ctr0={ctr0:#x}")
            s, v, nn = sq.reduce_strided(kind, key, ctr0, step, n)
            ref = _strided_exact_sum(oracle_mod, kind, key, ctr0, step, n)
            assert s == ref, (step, n, s, ref)
            assert v == oracle_mod.rounded_value(kind, ref) and nn == n


@pytest.mark.parametrize("kind", KINDS)
def test_strided_reduce_every_config_and_unit_step(sq, kind):
    """Strided sums agree across launch configurations; step 1 equals the
    plain fused sum; a sum over [a, a+b) plus one over [a+b, a+c) with the same
    step equals the one over [a, a+c)."""
    key, ctr0, step, n = 0x510E527FADE682D1, 2**64 - 123456, 5, (1 << 21) + 9
    ref = None
    for unroll in (1, 2, 4):
        for gpc in (1, 8, 64):
            c = sq.cfg(256, unroll, gpc)
            log(f"strided reduce kind={kind} cfg={c.as_dict()}")
            s, _, _ = sq.reduce_strided(kind, key, ctr0, step, n, launch_cfg=c)
            ref = s if ref is None else ref
            assert s == ref, c.as_dict()
    assert sq.reduce_strided(kind, key, ctr0, 1, n)[0] == sq.reduce(kind, key, ctr0, n)[0]
    per_ctr = 2 if kind in (4, 5) else 1
    b = 1_000_000
    left = sq.reduce_strided(kind, key, ctr0, step, b)[0]
    right = sq.reduce_strided(kind, key, (ctr0 + (b // per_ctr) * step) % 2**64, step, n - b)[0]
    assert left + right == ref


# ---------------------------------------------------------------- key-counter mode
def _keys(g, m):
    k = g.integers(0, 2**64, size=m, dtype=np.uint64)
    k[:: 13] = 0
    k[1:: 17] &= np.uint64(~1 & M64)
    return k


@pytest.mark.parametrize("kind", [0, 1, 2, 3])
def test_key_counter_mode(sq, oracle_mod, kind):
    """m from 0 to 2^20+3 keys, counters 0, 1, 2^64-1 and random: vector path
    (16-byte aligned keys and output) and element path (keys or output off by
    one element), bytes equal the oracle's; guards untouched."""
    import torch

    g = np.random.Generator(np.random.PCG64(800 + kind))
    W = KIND_BYTES[kind]
    for m in (0, 1, 2, 3, 4, 5, 7, 1000, 4099, (1 << 20) + 3):
        keys = _keys(g, m)
        for ctr in (0, 1, M64, int(g.integers(0, 2**64, dtype=np.uint64))):
            ref = oracle_mod.fill_keys(kind, ctr, keys).view(np.uint8)
            for kshift, oshift in ((0, 0), (1, 0), (0, 1)):
                kbuf = torch.zeros(m + 4, dtype=torch.int64, device="cuda")
                kbuf[kshift: kshift + m] = torch.from_numpy(keys.view(np.int64)).cuda()
                obuf = torch.full((m * W + 256,), 0x77, dtype=torch.uint8, device="cuda")
                o0 = 64 + oshift * W
                log(f"keys kind={kind} m={m} ctr={ctr:#x} kshift={kshift} oshift={oshift}")
                sq.check(sq.lib().sq_fill_keys(kind, ctr, kbuf.data_ptr() + 8 * kshift, m,
                                               obuf.data_ptr() + o0, sq._stream()))
                torch.cuda.synchronize()
                host = to_host_bytes(obuf)
                assert host[o0: o0 + m * W].tobytes() == ref.tobytes(), first_diff(host[o0: o0 + m * W], ref)
                assert np.all(host[:o0] == 0x77) and np.all(host[o0 + m * W:] == 0x77)
            if m > 100000:
                break


@pytest.mark.parametrize("kind", [0, 3])
def test_key_counter_every_config(sq, oracle_mod, kind):
    import torch

    g = np.random.Generator(np.random.PCG64(900 + kind))
    m = 3 * (1 << 18) + 5
    keys = _keys(g, m)
    kd = torch.from_numpy(keys.view(np.int64)).cuda()
    ref = oracle_mod.fill_keys(kind, 0, keys).view(np.uint8)
    cfgs = [sq.cfg(b, 4, g) for b in (64, 256, 512, 1024) for g in (1, 8, 64)]
    cfgs += [sq.cfg(b, 4, 1, 2) for b in (64, 128, 256, 1024)]
    for c in cfgs:
        log(f"keys kind={kind} cfg={c.as_dict()}")
        got = to_host_bytes(sq.fill_keys(kind, 0, kd, launch_cfg=c))
        assert got.tobytes() == ref.tobytes(), c.as_dict()


def test_key_counter_equals_batch_of_single_outputs(sq):
    """Key-counter mode is a ragged batch of length-1 streams all at one counter."""
    import torch

    g = np.random.Generator(np.random.PCG64(31))
    m, ctr = 5000, 0x0123456789ABCDEF
    keys = _keys(g, m)
    a = to_host_bytes(sq.fill_keys(2, ctr, torch.from_numpy(keys.view(np.int64)).cuda()))
    db = sq.batch_to_device(keys, np.full(m, ctr, dtype=np.uint64), np.ones(m, dtype=np.uint64),
                            8 * np.arange(m, dtype=np.uint64), np.full(m, 2, dtype=np.uint8), 8 * m)
    sq.fill_batch(db)
    assert a.tobytes() == to_host_bytes(db.out)[: 8 * m].tobytes()


def test_key_counter_invalid(sq):
    import torch

    kb = torch.zeros(16, dtype=torch.int64, device="cuda")
    ob = torch.zeros(16, dtype=torch.int64, device="cuda")
    for kind, kaddr, oaddr, status in ((4, 0, 0, -1), (9, 0, 0, -1), (0, 4, 0, -2), (2, 0, 4, -2)):
        with pytest.raises(sq.SquaresError) as e:
            sq.check(sq.lib().sq_fill_keys(kind, 0, kb.data_ptr() + kaddr, 4, ob.data_ptr() + oaddr, sq._stream()))
        assert e.value.status == status


# ---------------------------------------------------------------- key generation
def _distinct_halves(keys: np.ndarray) -> bool:
    for shift in (0, 32):
        half = (keys >> np.uint64(shift)) & np.uint64(0xFFFFFFFF)
        digits = np.stack([(half >> np.uint64(4 * i)) & np.uint64(15) for i in range(8)], axis=1)
        s = np.sort(digits, axis=1)
        if np.any(s[:, 1:] == s[:, :-1]):
            return False
    return True


def test_make_keys_parity(sq, oracle_mod):
    """Device keys equal the oracle's bit for bit (counters across the wrap,
    several grid sizes), every key has distinct-digit halves, and windows
    compose."""
    import torch

    for gk, c0, m in ((0x9E3779B97F4A7C15, 0, 1), (0x9E3779B97F4A7C15, 2**64 - 9, 1000),
                      (0x7C2B5E19A4D3F680, 12345, (1 << 20) + 5)):
        log(f"make_keys gk={gk:#x} c0={c0:#x} m={m}")
        got = sq.make_keys(gk, c0, m).cpu().numpy().view(np.uint64)
        ref = oracle_mod.make_keys(gk, c0, m)
        assert np.array_equal(got, ref), int(np.nonzero(got != ref)[0][0])
        assert _distinct_halves(got) and np.all(got & np.uint64(1) == 1)
    win = sq.make_keys(0x9E3779B97F4A7C15, 20, 10).cpu().numpy().view(np.uint64)
    whole = sq.make_keys(0x9E3779B97F4A7C15, 0, 20).cpu().numpy().view(np.uint64)
    assert np.array_equal(win, whole[10:20])
    torch.cuda.synchronize()


def test_make_keys_feed_key_counter_mode(sq, oracle_mod):
    """Section 4's key-counter test: keys from the key generator, counter 0."""
    keys = sq.make_keys(0x6A09E667F3BCC909, 0, 4096)
    got = sq.fill_keys(0, 0, keys).cpu().numpy().view(np.uint32)
    ref = oracle_mod.fill_keys(0, 0, oracle_mod.make_keys(0x6A09E667F3BCC909, 0, 4096))
    assert np.array_equal(got, ref)


# ---------------------------------------------------------------- scalar entry points
def test_make_keys_and_key_counter_past_2p32(sq, oracle_mod):
    """2^32 + 5 keys generated on the device (32 GiB; key indices past 32 bits,
    the generator's counter wrapping 500 keys before the end) and a U32
    key-counter fill over all of them (16 GiB): the last 2^12 keys and
    outputs and 2^12 random ones equal the oracle's."""
    import torch

    gk, c0, ctr = 0x243F6A8885A308D3, 2**64 - 2**33 + 1000, 7
    m = (1 << 32) + 5
    log(f"make_keys + key-counter past 2^32 gk={gk:#x} c0={c0:#x} m={m}")
    keys = sq.make_keys(gk, c0, m)
    out = sq.fill_keys(0, ctr, keys)
    g = np.random.Generator(np.random.PCG64(77))
    idx = np.unique(np.concatenate([m - 1 - np.arange(1 << 12), g.integers(0, m, size=1 << 12)])).astype(np.int64)
    ti = torch.from_numpy(idx).cuda()
    got_k = keys.view(torch.int64)[ti].cpu().numpy().view(np.uint64)
    got_o = out.view(torch.int32)[ti].cpu().numpy().view(np.uint32)
    for j, kj in zip(idx, got_k):
        assert kj == oracle_mod.make_keys(gk, (c0 + 2 * int(j)) % 2**64, 1)[0], f"key {int(j)}"
    assert np.array_equal(got_o, oracle_mod.fill_keys(0, ctr, got_k))
    del keys, out
    torch.cuda.empty_cache()


def test_key_counter_grid_cap(sq, oracle_mod):
    """2^33 + 3 squares64 keys generated on the device (2^32 + 1 vectors of two
    outputs, 64 GiB of keys and 64 GiB of output) with one vector per lane
    asked for: one workgroup per 256 vectors would be 2^32 + 256 work-items,
    more than a launch may hold, so the grid is capped (16777215 workgroups)
    and the kernel strides over the rest.  At the last 2^12 and 2^12 random positions the
    keys equal the oracle's key generation and the outputs the oracle's
    key-counter mode."""
    import torch

    gk, c0, ctr = 0x13198A2E03707344, 0xA4093822299F31D0, 0x5851F42D4C957F2D
    m = (1 << 33) + 3
    log(f"key-counter grid cap m={m}")
    keys = sq.make_keys(gk, c0, m)
    out = sq.fill_keys(2, ctr, keys, launch_cfg=sq.cfg(256, 1, 1, 2))
    g = np.random.Generator(np.random.PCG64(78))
    idx = np.unique(np.concatenate([m - 1 - np.arange(1 << 12), g.integers(0, m, size=1 << 12)])).astype(np.int64)
    ti = torch.from_numpy(idx).cuda()
    got_k = keys.view(torch.int64)[ti].cpu().numpy().view(np.uint64)
    got_o = out.view(torch.int64)[ti].cpu().numpy().view(np.uint64)
    for j in (int(idx[0]), int(idx[len(idx) // 2]), int(idx[-1])):
        k = got_k[np.searchsorted(idx, j)]
        assert k == oracle_mod.make_keys(gk, (c0 + 2 * j) % 2**64, 1)[0], f"key {j}"
    assert np.array_equal(got_o, oracle_mod.fill_keys(2, ctr, got_k))
    del keys, out
    torch.cuda.empty_cache()


def test_scalar_entry_points_paper_argument_order(sq, oracle_mod):
    """sq32_at / sq64_at take (ctr, key) like the paper's functions and agree
    with the oracle and with element 0 of a bulk fill called as (key, ctr0)."""
    g = np.random.Generator(np.random.PCG64(61))
    pairs = [(0, 0), (1, 2**32 + 1), (1, 2**63), (2**64 - 1, 1), (5, 2**32)]
    pairs += [(int(a), int(b)) for a, b in g.integers(0, 2**64, size=(40, 2), dtype=np.uint64)]
    for ctr, key in pairs:
        assert sq.sq32_at(ctr, key) == oracle_mod.squares32(ctr, key)
        assert sq.sq64_at(ctr, key) == oracle_mod.squares64(ctr, key)
    ctr, key = pairs[-1]
    assert int(sq.sq32_fill(key, ctr, 1).cpu().numpy().view(np.uint32)[0]) == sq.sq32_at(ctr, key)
    assert int(sq.sq64_fill(key, ctr, 1).cpu().numpy().view(np.uint64)[0]) == sq.sq64_at(ctr, key)


def test_debug_validate_rejects_overlap(sq, monkeypatch):
    """With SQ_DEBUG_VALIDATE set, overlapping streams and streams the kernels
    would skip are errors at the call; a valid batch still runs."""
    keys = np.array([1, 2, 3], dtype=np.uint64)
    ctrs = np.zeros(3, dtype=np.uint64)
    lens = np.array([100, 100, 100], dtype=np.uint64)
    kinds = np.zeros(3, dtype=np.uint8)
    db = sq.batch_to_device(keys, ctrs, lens, np.array([0, 200, 800], dtype=np.uint64), kinds, 4096)
    monkeypatch.setenv("SQ_DEBUG_VALIDATE", "1")
    with pytest.raises(sq.SquaresError) as e:
        sq.fill_batch(db)
    assert e.value.status == -1 and "overlap" in str(e.value)
    ok = sq.batch_to_device(keys, ctrs, lens, np.array([0, 400, 800], dtype=np.uint64), kinds, 4096)
    sq.fill_batch(ok)
    assert sq.batch_errors(ok) == 0
    bad = sq.batch_to_device(keys, ctrs, lens, np.array([0, 400, 4000], dtype=np.uint64), kinds, 4096)
    with pytest.raises(sq.SquaresError) as e:
        sq.fill_batch(bad)
    assert e.value.status == -1 and "past the arena" in str(e.value)
