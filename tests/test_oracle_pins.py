"""CPU tests of the oracle against what the paper and the mathematics fix.

The oracle is checked against the pin battery in ``pins.py`` (closed forms,
hand-worked examples, the squares64/squares32 identity, a balance screen),
plus bulk properties: counter order and wrap, the Weyl identity the paper
relies on, the exact uniform conversions and the exact sum.  A mutation
battery shows that each plausible transcription mistake fails at least one
pin, so the pins are not vacuous.
"""
from __future__ import annotations

import time
from fractions import Fraction

import numpy as np
import pytest

from pins import ALL_PINS, EDGE_WORDS, M64, OracleImpl, balance_screen, load_worked_examples, pin_balance

U64_ = np.uint64


# ---------------------------------------------------------------- oracle pins
@pytest.mark.parametrize("name", sorted(ALL_PINS))
def test_oracle_passes_pin(oracle_mod, name):
    impl = OracleImpl(oracle_mod)
    if name == "balance":
        bad = pin_balance(impl, n=1 << 24)  # 2^24 outputs, as on the 64 MiB fill
    else:
        bad = ALL_PINS[name](impl)
    assert not bad, bad


def test_worked_examples_nontrivial():
    rows = load_worked_examples()
    assert len(rows) >= 10
    assert len({r[1] for r in rows}) >= 4  # several keys


# ---------------------------------------------------------------- mutation battery
def _model(ctr, key, out64, *, swap_args=False, z_plus_one=False, z_minus=False, skip_rot=(),
           rot_amt=32, shift_not_rot=False, addends="yzyzy", low_out=False, no_cross=False,
           t_after_rot=False, r5_no_shift=False, xor_to_add=False, y32=False, rounds=4):
    """Numpy model of the rounds with switches for plausible mistakes.  Only
    used to show the pins catch each mistake; never a reference for anything."""
    ctr = ctr.astype(U64_)
    key = key.astype(U64_)
    s32, lo = U64_(32), U64_(0xFFFFFFFF)
    if y32:
        y = ((ctr & lo) * (key & lo)) & lo
    else:
        y = ctr * key
    if swap_args:
        z = y + ctr
    elif z_plus_one:
        z = y + U64_(1)
    elif z_minus:
        z = y - key
    else:
        z = y + key
    add = {"y": y, "z": z}

    def sq(x):
        return (x & lo) * (x & lo) if no_cross else x * x

    def rot(x):
        if shift_not_rot:
            return x >> s32
        a = U64_(rot_amt)
        return (x >> a) | (x << (U64_(64) - a))

    x = y
    for r in range(1, rounds):
        x = sq(x) + add[addends[r - 1]]
        if r not in skip_rot:
            x = rot(x)
    t = sq(x) + add[addends[rounds - 1]]
    if not out64:
        return (t & lo) if low_out else (t >> s32)
    x5 = t if t_after_rot else rot(t)
    if t_after_rot:
        t = rot(t)
    r5 = sq(x5) + add[addends[rounds]]
    r5 = r5 if r5_no_shift else (r5 >> s32)
    return (t + r5) if xor_to_add else (t ^ r5)


class ModelImpl:
    def __init__(self, kw32=None, kw64=None):
        self.kw32 = kw32 or {}
        self.kw64 = kw64 or {}

    def sq32(self, c, k):
        return _model(c, k, False, **self.kw32)

    def sq64(self, c, k):
        return _model(c, k, True, **self.kw64)

    def range32(self, key, ctr0, n):
        c = (U64_(ctr0) + np.arange(n, dtype=U64_)).astype(U64_)
        return self.sq32(c, np.full(n, key, dtype=U64_))

    def range64(self, key, ctr0, n):
        c = (U64_(ctr0) + np.arange(n, dtype=U64_)).astype(U64_)
        return self.sq64(c, np.full(n, key, dtype=U64_))


def _both(**kw):
    return ModelImpl(kw, kw)


MUTANTS = {
    "ctr_key_roles_swapped": _both(swap_args=True),
    "z_is_y_plus_1": _both(z_plus_one=True),
    "z_is_ctr_minus_1_times_key": _both(z_minus=True),
    "no_rotate_round1": _both(skip_rot=(1,)),
    "no_rotate_round2": _both(skip_rot=(2,)),
    "no_rotate_round3": _both(skip_rot=(3,)),
    "rotate_by_16": _both(rot_amt=16),
    "rotate_by_31": _both(rot_amt=31),
    "shift_instead_of_rotate": _both(shift_not_rot=True),
    "addends_zyzyz": _both(addends="zyzyz"),
    "addends_all_y": _both(addends="yyyyy"),
    "addends_yzyyy": _both(addends="yzyyy"),
    "cross_term_dropped": _both(no_cross=True),
    "ctr_key_product_32bit": _both(y32=True),
    "three_rounds": ModelImpl({"rounds": 3}, {"rounds": 3}),
    "five_rounds_32": ModelImpl({"rounds": 5, "addends": "yzyzyz"}, {}),
    "sq32_low_half": ModelImpl({"low_out": True}, {}),
    "sq64_t_after_rotate": ModelImpl({}, {"t_after_rot": True}),
    "sq64_round5_adds_z": ModelImpl({}, {"addends": "yzyzz"}),
    "sq64_round5_unshifted": ModelImpl({}, {"r5_no_shift": True}),
    "sq64_add_not_xor": ModelImpl({}, {"xor_to_add": True}),
}


def test_unmutated_model_passes_all_pins():
    impl = ModelImpl()
    for name, pin in ALL_PINS.items():
        assert not pin(impl), name


@pytest.mark.parametrize("mutant", sorted(MUTANTS))
def test_each_mutant_fails_a_pin(mutant):
    impl = MUTANTS[mutant]
    failed = [name for name, pin in ALL_PINS.items() if pin(impl)]
    assert failed, f"mutant {mutant} passes every pin"


# ---------------------------------------------------------------- transcription cross-check
def _bigint_sq(ctr, key, out64):
    """Arbitrary-precision re-evaluation.  A second transcription, kept as a
    consistency check of the C build; not counted as a pin."""
    y = (ctr * key) % 2**64
    z = ((ctr + 1) * key) % 2**64
    x = y
    for a in (y, z, y):
        x = (x * x + a) % 2**64
        x = ((x >> 32) | (x << 32)) % 2**64
    t = (x * x + z) % 2**64
    if not out64:
        return t >> 32
    x = ((t >> 32) | (t << 32)) % 2**64
    return t ^ (((x * x + y) % 2**64) >> 32)


def test_transcription_bigint_and_trace(oracle_mod):
    g = np.random.Generator(np.random.PCG64(21))
    pairs = [(a, b) for a in EDGE_WORDS for b in EDGE_WORDS]
    pairs += [(int(a), int(b)) for a, b in g.integers(0, 1 << 64, size=(5000, 2), dtype=np.uint64, endpoint=False)]
    for c, k in pairs:
        assert oracle_mod.squares32(c, k) == _bigint_sq(c, k, False)
        assert oracle_mod.squares64(c, k) == _bigint_sq(c, k, True)
    # the trace's round-4 value is t; its high half is squares32
    for c, k in pairs[:500]:
        tr = oracle_mod.trace(c, k)
        assert tr[3] >> 32 == oracle_mod.squares32(c, k)
        assert tr[3] ^ (tr[4] >> 32) == oracle_mod.squares64(c, k)


def test_transcription_int128_every_round(oracle_mod, tmp_path):
    """The oracle's per-round values against a second transcription with full
    128-bit products and explicit truncation (tests/xcheck_int128.c, built
    here with gcc), on 2^20 random pairs plus all pairs of edge words.  A
    consistency check of the build, not counted as a pin."""
    import ctypes
    import os
    import subprocess

    src = os.path.join(os.path.dirname(os.path.abspath(__file__)), "xcheck_int128.c")
    so = str(tmp_path / "libxcheck.so")
    subprocess.run(["gcc", "-O2", "-shared", "-fPIC", "-o", so, src], check=True)
    X = ctypes.CDLL(so)
    vp = ctypes.c_void_p
    X.xcheck_trace_batch.argtypes = [vp, vp, ctypes.c_uint64, vp]
    g = np.random.Generator(np.random.PCG64(23))
    ctrs = g.integers(0, 1 << 64, size=1 << 20, dtype=np.uint64, endpoint=False)
    keys = g.integers(0, 1 << 64, size=1 << 20, dtype=np.uint64, endpoint=False)
    edge = np.array(EDGE_WORDS, dtype=np.uint64)
    ctrs = np.concatenate([ctrs, np.repeat(edge, edge.size)])
    keys = np.concatenate([keys, np.tile(edge, edge.size)])
    want = np.empty((ctrs.size, 5), dtype=np.uint64)
    X.xcheck_trace_batch(ctrs.ctypes.data, keys.ctypes.data, ctrs.size, want.ctypes.data)
    got = oracle_mod.trace_batch(ctrs, keys)
    assert np.array_equal(got, want)


def test_oracle_under_host_sanitizers(tmp_path):
    """Every oracle entry point on edge cases with buffers of exactly the size
    each call may write, built with gcc's address and undefined-behaviour
    sanitizers (tests/oracle_sanitize.c): no out-of-range access, no
    undefined shift or overflow, no leak, and the entry points agree with
    each other.  Skipped where the host compiler has no sanitizer runtime."""
    import os
    import subprocess

    here = os.path.dirname(os.path.abspath(__file__))
    exe = str(tmp_path / "oracle_sanitize")
    cmd = ["gcc", "-std=c11", "-O1", "-g", "-Wall", "-Wextra", "-fsanitize=address,undefined",
           "-fno-sanitize-recover=all", "-fno-omit-frame-pointer", os.path.join(here, "oracle_sanitize.c"),
           os.path.join(here, "..", "oracle", "squares_oracle.c"), "-o", exe]
    r = subprocess.run(cmd, capture_output=True, text=True)
    if r.returncode != 0:
        if "asan" in r.stderr or "ubsan" in r.stderr:
            pytest.skip("no sanitizer runtime for the host compiler")
        pytest.fail(r.stderr)
    run = subprocess.run([exe], capture_output=True, text=True, timeout=300,
                         env=dict(os.environ, ASAN_OPTIONS="detect_leaks=1:abort_on_error=0"))
    assert run.returncode == 0 and run.stdout.strip().endswith("ok"), run.stdout[-2000:] + run.stderr[-2000:]


# ---------------------------------------------------------------- bulk: counters
def test_fill_is_counter_order(oracle_mod):
    o = oracle_mod
    key, ctr0 = 0xC8E3A1F7D49B2650, 0x123456789ABCDEF0
    a = o.fill(o.U32, key, ctr0, 300)
    b = o.fill(o.U64, key, ctr0, 300)
    for i in range(300):
        assert int(a[i]) == o.squares32(ctr0 + i, key)
        assert int(b[i]) == o.squares64(ctr0 + i, key)


@pytest.mark.parametrize("kind", [0, 1, 2, 3])
def test_counter_wrap(oracle_mod, kind):
    """The counter is a 64-bit integer (Section 3): a range that passes 2^64-1
    continues at 0 with the same key."""
    o = oracle_mod
    key = 0x5F0E9D8C7B6A4132
    for d in (1, 2, 7, 100):
        n = 257
        whole = o.fill(kind, key, 2**64 - d, n)
        parts = np.concatenate([o.fill(kind, key, 2**64 - d, d), o.fill(kind, key, 0, n - d)])
        assert whole.tobytes() == parts.tobytes()


def test_weyl_identity():
    """Section 2: repeating w += s i times gives i*s mod 2^64, the identity that
    lets counter*key stand in for a Weyl sequence (and that a kernel stepping
    y by key, or by a multiple of key, relies on)."""
    g = np.random.Generator(np.random.PCG64(22))
    for s in [int(v) for v in g.integers(0, 1 << 64, size=4, dtype=np.uint64, endpoint=False)] + [M64, 1 << 63]:
        w = 0
        for i in range(1 << 16):
            assert w == (i * s) % 2**64
            w = (w + s) % 2**64
    # jumps: y(c0 + j) == y(c0) + j*key for strides used by bulk stepping
    for key in (0x9E3779B97F4A7C15, M64):
        for c0 in (0, M64 - 5, 1 << 63):
            for j in (1, 4, 2, 65536, 1 << 32, (1 << 64) - 3):
                assert ((c0 + j) * key) % 2**64 == ((c0 * key) + j * key) % 2**64
    # (ctr+1)*key == ctr*key + key: the second addend of one counter is the
    # first addend of the next
    for c in EDGE_WORDS:
        assert ((c + 1) * 0x6A09E667F3BCC909) % 2**64 == (c * 0x6A09E667F3BCC909 + 0x6A09E667F3BCC909) % 2**64


def test_threads_equal_single(oracle_mod):
    o = oracle_mod
    key, ctr0 = 0xA3B1C2D4E5F60789, 2**64 - 5000
    for kind in (0, 1, 2, 3):
        a = o.fill(kind, key, ctr0, 100003, threads=1)
        b = o.fill(kind, key, ctr0, 100003, threads=7)
        assert a.tobytes() == b.tobytes()


# ---------------------------------------------------------------- uniform conversions
def test_uniform_f32_is_top_24_bits(oracle_mod):
    """f32 = top 24 bits of the 32-bit output scaled into [0,1): an integer
    multiple of 2^-24 with 0 <= u*2^-32 - f < 2^-24."""
    o = oracle_mod
    key, ctr0, n = 0x2B7E151628AED2A6, 99, 1 << 16
    u = o.fill(o.U32, key, ctr0, n).astype(np.int64)
    f = o.fill(o.F32, key, ctr0, n)
    m = f.astype(np.float64) * 2.0**24
    assert np.all(m == np.floor(m))
    d = u.astype(np.float64) * 2.0**-32 - f.astype(np.float64)
    assert np.all(d >= 0) and np.all(d < 2.0**-24)
    assert np.all(f >= 0) and np.all(f < 1)
    lib = o.lib()
    assert lib.oracle_to_f32(0) == 0.0
    assert lib.oracle_to_f32(0xFFFFFFFF) == 1.0 - 2.0**-24
    assert lib.oracle_to_f32(0x80000000) == 0.5
    assert lib.oracle_to_f32(0xFF) == 0.0 and lib.oracle_to_f32(0x100) == 2.0**-24


def test_uniform_f64_is_top_53_bits(oracle_mod):
    """f64 = top 53 bits of the 64-bit output scaled into [0,1), exactly."""
    o = oracle_mod
    key, ctr0, n = 0x2B7E151628AED2A6, 2**64 - 1000, 1 << 14
    u = o.fill(o.U64, key, ctr0, n)
    f = o.fill(o.F64, key, ctr0, n)
    for i in range(0, n, 7):
        exact = Fraction(int(u[i]), 2**64)
        fi = Fraction(float(f[i]))
        assert (fi * 2**53).denominator == 1
        assert 0 <= exact - fi < Fraction(1, 2**53)
    lib = o.lib()
    assert lib.oracle_to_f64(0) == 0.0
    assert lib.oracle_to_f64(M64) == 1.0 - 2.0**-53
    assert lib.oracle_to_f64(1 << 63) == 0.5
    assert lib.oracle_to_f64(2047) == 0.0 and lib.oracle_to_f64(2048) == 2.0**-53


# ---------------------------------------------------------------- exact sum
@pytest.mark.parametrize("kind", [0, 1, 2, 3])
def test_exact_sum(oracle_mod, kind):
    o = oracle_mod
    key, ctr0 = 0x3C6EF372FE94F82B, 2**64 - 12345
    n = 1 << 17
    vals = o.fill({0: o.U32, 1: o.U32, 2: o.U64, 3: o.U64}[kind], key, ctr0, n)
    shift = {0: 0, 1: 8, 2: 0, 3: 11}[kind]
    expect = sum(int(v) >> shift for v in vals)
    assert o.exact_sum(kind, key, ctr0, n) == expect
    assert o.exact_sum(kind, key, ctr0, n, threads=5) == expect
    # additivity over a split point, including across the wrap
    for b in (0, 1, 12345, 77777, n):
        left = o.exact_sum(kind, key, ctr0, b)
        right = o.exact_sum(kind, key, (ctr0 + b) % 2**64, n - b)
        assert left + right == expect
    # the scaled value of a uniform kind equals the float sum done exactly
    if kind in (1, 3):
        fv = o.fill(kind, key, ctr0, 4096)
        exact = sum(Fraction(float(v)) for v in fv)
        assert Fraction(o.exact_sum(kind, key, ctr0, 4096)) * Fraction(2) ** o.KIND_SUM_SCALE[kind] == exact
    assert o.exact_sum(kind, key, ctr0, 0) == 0


def test_rounded_value_is_nearest_even(oracle_mod):
    o = oracle_mod
    # ties to even on a 54-bit integer
    assert o.rounded_value(o.U64, 2**53 + 1) == float(2**53)
    assert o.rounded_value(o.U64, 2**53 + 3) == float(2**53 + 4)
    big = (1 << 127) + (1 << 74) + 1  # just above a tie: rounds up
    assert o.rounded_value(o.U64, big) == float((1 << 127) + (1 << 75))
    assert o.rounded_value(o.F64, 2**53) == 1.0


def test_sum_near_u128_limit(oracle_mod):
    """The 128-bit accumulator carries: a sum of 2^20 values near 2^64 exceeds
    2^64 and must keep its high word."""
    o = oracle_mod
    s = o.exact_sum(o.U64, 0x8F1BBCDCCA62C1D6, 7, 1 << 20)
    assert s > 2**64 and s < (1 << 20) * 2**64


# ---------------------------------------------------------------- batch
def test_batch_matches_per_stream(oracle_mod):
    from paper_2004_06278_amd import workloads as W

    o = oracle_mod
    b = W.small_random_batch(seed=31, m=60, max_len=700)
    arena = o.fill_batch(b.keys, b.ctr0s, b.lens, b.offs, b.kinds, b.arena_bytes)
    for s in range(b.m):
        k, L, off = int(b.kinds[s]), int(b.lens[s]), int(b.offs[s])
        ref = o.fill(k, int(b.keys[s]), int(b.ctr0s[s]), L).view(np.uint8)
        assert arena[off: off + ref.size].tobytes() == ref.tobytes()


def test_config1_oracle_under_one_second(oracle_mod):
    """The 2^24-output squares32 fill runs on one core in well under a second."""
    o = oracle_mod
    from paper_2004_06278_amd import workloads as W

    c = W.plain_fill_case()
    u = np.ones(c.n, dtype=np.uint32)  # pages touched before timing
    dt = []
    for _ in range(2):
        t0 = time.perf_counter()
        o.fill_into(o.U32, c.key, c.ctr0, u)
        dt.append(time.perf_counter() - t0)
    assert min(dt) < 1.0, dt
    assert not balance_screen(u, 32)


# ---------------------------------------------------------------- split squares64 (two 32-bit outputs per call)
def test_split_halves_are_squares64_words(oracle_mod):
    """Split element 2j is the low word and 2j+1 the high word of squares64 at
    ctr0+j (Section 5's split into two 32-bit halves, read in little-endian
    order): the split fill is the 64-bit fill's memory viewed as 32-bit words."""
    o = oracle_mod
    key, ctr0 = 0x9D2C5680A1B3E7F4, 2**64 - 37
    for n in (0, 1, 2, 77, 1000):
        a = o.fill(o.U32X2, key, ctr0, n)
        b = o.fill(o.U64, key, ctr0, (n + 1) // 2).view(np.uint32)[:n]
        assert a.tobytes() == b.tobytes()


def test_split_high_words_are_squares32(oracle_mod):
    """The odd (high-word) split outputs equal squares32 at the same counter,
    because squares64 keeps round 4 whole and only XORs below 2^32."""
    o = oracle_mod
    key, ctr0, n = 0x0F7E6D5C4B3A2918, 123456789, 4096
    a = o.fill(o.U32X2, key, ctr0, 2 * n)
    assert np.array_equal(a[1::2], o.fill(o.U32, key, ctr0, n))


def test_split_floats_top_24_bits(oracle_mod):
    o = oracle_mod
    key, ctr0, n = 0x7C3B9A1E5D2F4068, 5, 1 << 14
    u = o.fill(o.U32X2, key, ctr0, n).astype(np.float64)
    f = o.fill(o.F32X2, key, ctr0, n).astype(np.float64)
    assert np.all(f * 2**24 == np.floor(f * 2**24))
    d = u * 2.0**-32 - f
    assert np.all(d >= 0) and np.all(d < 2.0**-24)


@pytest.mark.parametrize("kind", [4, 5])
def test_split_sums_and_wrap(oracle_mod, kind):
    o = oracle_mod
    key, ctr0 = 0x2E4A6C8E0B1D3F57, 2**64 - 1000
    n = 20001
    vals = o.fill(o.U32X2, key, ctr0, n).astype(object)
    shift = 8 if kind == 5 else 0
    expect = sum(int(v) >> shift for v in vals)
    assert o.exact_sum(kind, key, ctr0, n) == expect
    assert o.exact_sum(kind, key, ctr0, n, threads=7) == expect
    for b in (0, 2, 1998, 2000, 20000):  # even split points: the second part starts at a low word
        left = o.exact_sum(kind, key, ctr0, b)
        right = o.exact_sum(kind, key, (ctr0 + b // 2) % 2**64, n - b)
        assert left + right == expect
    # the counter wraps after 1000 calls = 2000 split outputs
    whole = o.fill(kind, key, ctr0, n)
    parts = np.concatenate([o.fill(kind, key, ctr0, 2000), o.fill(kind, key, 0, n - 2000)])
    assert whole.tobytes() == parts.tobytes()


# ---------------------------------------------------------------- counter increments other than one
@pytest.mark.parametrize("kind", [0, 1, 2, 3, 4, 5])
def test_strided_is_a_subsample_of_the_unit_fill(oracle_mod, kind):
    """Visiting counters ctr0, ctr0+s, ctr0+2s, ... gives the outputs a unit-step
    fill has at those counters (the step selects counters; Section 4 tests such
    increments)."""
    o = oracle_mod
    key, ctr0 = 0xB4C3D2E1F0A19283, 2**64 - 500
    split = kind in (4, 5)
    for step in (1, 2, 3, 7, 64):
        n = 600
        a = o.fill_strided(kind, key, ctr0, step, n)
        calls = (n + 1) // 2 if split else n
        unit = o.fill(kind, key, ctr0, (2 if split else 1) * calls * step)
        if split:
            ref = unit.reshape(-1, 2)[::step].reshape(-1)[:n]
        else:
            ref = unit[::step][:n]
        assert a.tobytes() == ref.tobytes()


def test_strided_special_steps(oracle_mod):
    o = oracle_mod
    key, c = 0x1A2B3C4D5E6F7081, 12345
    z = o.fill_strided(0, key, c, 0, 50)          # step 0: the same counter every time
    assert np.all(z == o.squares32(c, key))
    m = o.fill_strided(2, key, c, 2**64 - 1, 50)  # step -1 mod 2^64: counters run backwards
    assert [int(v) for v in m] == [o.squares64((c - i) % 2**64, key) for i in range(50)]
    big = o.fill_strided(0, key, 2**64 - 3, 2**63 + 1, 6)  # wraps on every step
    assert [int(v) for v in big] == [o.squares32((2**64 - 3 + i * (2**63 + 1)) % 2**64, key) for i in range(6)]


# ---------------------------------------------------------------- key-counter mode
@pytest.mark.parametrize("kind", [0, 1, 2, 3])
def test_key_counter_mode(oracle_mod, kind):
    """Counter fixed, key varying (Section 4's key-counter test mode): output j
    is the fill of keys[j] at that counter; key 0 gives 0 (closed form) and the
    hand-worked sparse keys give their worked values."""
    from pins import load_worked_examples

    o = oracle_mod
    g = np.random.Generator(np.random.PCG64(31))
    keys = g.integers(0, 2**64, size=300, dtype=np.uint64)
    keys[::17] = 0
    for ctr in (0, 1, 2**64 - 1, 0x0123456789ABCDEF):
        out = o.fill_keys(kind, ctr, keys)
        for j in range(0, 300, 7):
            assert out[j: j + 1].tobytes() == o.fill(kind, int(keys[j]), ctr, 1).tobytes()
        if kind in (0, 2):
            assert np.all(out[::17] == 0)
    rows = load_worked_examples()
    out32 = o.fill_keys(0, 1, np.array([r[1] for r in rows if r[0] == 1], dtype=np.uint64))
    assert [int(v) for v in out32] == [r[2] for r in rows if r[0] == 1]


# ---------------------------------------------------------------- distinct-digit keys
def _hex_digits(half: int) -> list[int]:
    return [(half >> (28 - 4 * i)) & 15 for i in range(8)]


def _index_of_upper(half: int) -> int:
    """Inverse of the upper-half decode, written from the shuffle's definition
    in the other direction: replay the partial Fisher-Yates shuffle and read
    each step's choice (position in the remaining list) as a mixed-radix
    digit."""
    pool = list(range(16))
    u, scale = 0, 1
    for i, d in enumerate(_hex_digits(half)):
        q = pool.index(d)
        assert q >= i
        u += (q - i) * scale
        scale *= 16 - i
        pool[q], pool[i] = pool[i], pool[q]
    return u


def _index_of_lower(half: int) -> int:
    """Inverse of the lower-half decode: the odd last digit is the first,
    radix-8 choice; the other seven digits are the shuffle's steps 1..7."""
    digits = _hex_digits(half)
    odd = digits[7]
    assert odd % 2 == 1
    pool = list(range(16))
    pool[0], pool[odd] = pool[odd], pool[0]
    u, scale = (odd - 1) // 2, 8
    for i, d in enumerate(digits[:7], start=1):
        q = pool.index(d)
        assert q >= i
        u += (q - i) * scale
        scale *= 16 - i
        pool[q], pool[i] = pool[i], pool[q]
    return u


def test_key_half_hand_values(oracle_mod):
    """Worked by hand.  Upper half: index 0 takes the digits in order; index 1
    first takes digit 1 (then 0, which the swap moved to position 1); the last
    index takes the last remaining digit at every step: 15, then 0 (moved to
    position 15 by the first swap), then 1, 2, ...  Lower half: index 0 puts
    odd digit 1 last and takes 0, 2, 3, ... in front; index 1 chooses odd
    digit 3; the last index chooses 15 and then the last remaining digit at
    every step: 0 (moved to position 15), 1, 2, ..."""
    o = oracle_mod
    assert o.KEY_CHOICES_HI == 518918400 and o.KEY_CHOICES_LO == 259459200
    assert o.key_upper(0) == 0x01234567
    assert o.key_upper(1) == 0x10234567
    assert o.key_upper(16) == 0x02134567  # second step's choice 1: position 2 after the first step
    assert o.key_upper(o.KEY_CHOICES_HI - 1) == 0xF0123456
    assert o.key_lower(0) == 0x02345671
    assert o.key_lower(1) == 0x12045673   # odd digit 3 swapped with 0: list 3,1,2,0,4,..., then 1,2,0,4,5,6,7
    assert o.key_lower(8) == 0x20345671   # first shuffle step's choice 1
    assert o.key_lower(o.KEY_CHOICES_LO - 1) == 0x0123456F


def test_key_half_is_a_bijection_sample(oracle_mod):
    """Decoding then re-encoding returns the index (so distinct indices give
    distinct halves); every half has 8 different digits and every lower half
    ends in an odd digit."""
    o = oracle_mod
    g = np.random.Generator(np.random.PCG64(41))
    for N, dec, enc in ((o.KEY_CHOICES_HI, o.key_upper, _index_of_upper),
                        (o.KEY_CHOICES_LO, o.key_lower, _index_of_lower)):
        us = [0, 1, 7, 8, 15, 16, 239, 240, N - 1] + [int(v) for v in g.integers(0, N, 3000)]
        for u in us:
            h = dec(u)
            assert len(set(_hex_digits(h))) == 8
            assert enc(h) == u
            if dec is o.key_lower:
                assert h & 1


def test_key_index_end_points(oracle_mod):
    o = oracle_mod
    for N in (o.KEY_CHOICES_HI, o.KEY_CHOICES_LO):
        assert o.key_index(0, N) == 0
        assert o.key_index(2**64 - 1, N) == N - 1
        assert o.key_index(2**63, N) == N // 2
        g = np.random.Generator(np.random.PCG64(43))
        for r in g.integers(0, 2**64, size=200, dtype=np.uint64):
            assert o.key_index(int(r), N) == (int(r) * N) >> 64


def test_make_keys_property_and_source(oracle_mod):
    """Each key has distinct-digit halves (Section 3, Discussion) and an odd
    last digit; its halves come from squares64 at counters ctr0 + 2j and
    ctr0 + 2j + 1; counters wrap."""
    o = oracle_mod
    gk, c0 = 0x9E3779B97F4A7C15, 2**64 - 7
    keys = o.make_keys(gk, c0, 64)
    for j, k in enumerate(int(v) for v in keys):
        up, lo = k >> 32, k & 0xFFFFFFFF
        assert len(set(_hex_digits(up))) == 8 and len(set(_hex_digits(lo))) == 8 and k & 1
        r_up = o.squares64((c0 + 2 * j) % 2**64, gk)
        r_lo = o.squares64((c0 + 2 * j + 1) % 2**64, gk)
        assert _index_of_upper(up) == (r_up * o.KEY_CHOICES_HI) >> 64
        assert _index_of_lower(lo) == (r_lo * o.KEY_CHOICES_LO) >> 64
    # a later window of the same range is the same keys
    assert o.make_keys(gk, (c0 + 10) % 2**64, 5).tolist() == keys[5:10].tolist()


def test_make_keys_digit_frequencies(oracle_mod):
    """Digit frequencies per position match the procedure's exact
    distribution (loose chi-square screens over 40000 keys): 1/16 each in the
    upper half; 1/8 for each odd digit in the last position; in the other
    lower positions 1/15 for an even digit and 7/120 for an odd one (the odd
    last digit is drawn first and excluded).  No two keys collide."""
    o = oracle_mod
    keys = o.make_keys(0x7C2B5E19A4D3F680, 0, 40000)
    assert np.unique(keys).size == keys.size
    odd = np.arange(16) % 2 == 1
    for pos in range(16):
        d = ((keys >> np.uint64(60 - 4 * pos)) & np.uint64(15)).astype(np.int64)
        cnt = np.bincount(d, minlength=16).astype(float)
        if pos < 8:
            p = np.full(16, 1 / 16)
        elif pos == 15:
            p = np.where(odd, 1 / 8, 0.0)
            assert cnt[~odd].sum() == 0
        else:
            p = np.where(odd, 7 / 120, 1 / 15)
        assert abs(p.sum() - 1) < 1e-12
        m = p > 0
        exp = keys.size * p[m]
        chi2 = float(((cnt[m] - exp) ** 2 / exp).sum())
        assert chi2 < 60, (pos, chi2)  # at most 15 dof: p ~ 1e-7
