"""Pin battery: properties the paper and the mathematics fix for squares32 /
squares64, written so they can be applied to any implementation (the CPU
oracle, and deliberately broken variants that show each pin has teeth).

An implementation is an object with
    sq32(ctr, key) -> uint64 ndarray   (elementwise over uint64 ndarrays)
    sq64(ctr, key) -> uint64 ndarray
    range32(key, ctr0, n) / range64(key, ctr0, n) -> uint64 ndarray
Each pin returns a list of failure descriptions (empty when it holds).
"""
from __future__ import annotations

import os

import numpy as np
from scipy import stats

M64 = (1 << 64) - 1
EDGE_WORDS = [0, 1, 2, 3, (1 << 32) - 1, 1 << 32, (1 << 32) + 1, 1 << 63, M64, M64 - 1,
              0x5555555555555555, 0xAAAAAAAAAAAAAAAA, 0x0123456789ABCDEF, 0xFEDCBA9876543210]
GOLDEN = os.path.join(os.path.dirname(os.path.abspath(__file__)), "golden", "worked_examples.txt")


def load_worked_examples():
    rows = []
    with open(GOLDEN) as f:
        for line in f:
            line = line.strip()
            if not line or line.startswith("#"):
                continue
            c, k, a, b = (int(t, 16) for t in line.split())
            rows.append((c, k, a, b))
    return rows


def _u64(vals) -> np.ndarray:
    return np.array([v & M64 for v in vals], dtype=np.uint64)


def _rand_pairs(seed: int, n: int):
    g = np.random.Generator(np.random.PCG64(seed))
    c = g.integers(0, 1 << 64, size=n, dtype=np.uint64, endpoint=False)
    k = g.integers(0, 1 << 64, size=n, dtype=np.uint64, endpoint=False)
    ce = _u64([a for a in EDGE_WORDS for _ in EDGE_WORDS])
    ke = _u64([b for _ in EDGE_WORDS for b in EDGE_WORDS])
    return np.concatenate([c, ce]), np.concatenate([k, ke])


# ----------------------------------------------------------------------------
def pin_key_zero(impl) -> list[str]:
    """key = 0 makes y = z = 0, so every round squares 0: both outputs are 0
    for every counter (Section 2: the only inputs are ctr*key and (ctr+1)*key)."""
    g = np.random.Generator(np.random.PCG64(11))
    ctr = np.concatenate([_u64(EDGE_WORDS), g.integers(0, 1 << 64, size=500, dtype=np.uint64, endpoint=False)])
    key = np.zeros_like(ctr)
    bad = []
    if np.any(impl.sq32(ctr, key) != 0):
        bad.append("squares32(ctr, 0) != 0")
    if np.any(impl.sq64(ctr, key) != 0):
        bad.append("squares64(ctr, 0) != 0")
    return bad


def pin_worked_examples(impl) -> list[str]:
    """Hand-derived values for sparse keys (tests/golden/worked_examples.txt)."""
    rows = load_worked_examples()
    c = _u64([r[0] for r in rows])
    k = _u64([r[1] for r in rows])
    a = impl.sq32(c, k)
    b = impl.sq64(c, k)
    bad = []
    for i, (cc, kk, e32, e64) in enumerate(rows):
        if int(a[i]) != e32:
            bad.append(f"squares32({cc:#x},{kk:#x}) = {int(a[i]):#x}, expected {e32:#x}")
        if int(b[i]) != e64:
            bad.append(f"squares64({cc:#x},{kk:#x}) = {int(b[i]):#x}, expected {e64:#x}")
    return bad


def pin_key_one(impl) -> list[str]:
    """Closed form for key = 1 and 0 <= c <= 65535 (worked example E):
    squares32 = 0 and squares64 = c + 1."""
    n = 65536
    a = impl.range32(1, 0, n)
    b = impl.range64(1, 0, n)
    bad = []
    if np.any(a != 0):
        bad.append("key=1: squares32 != 0 for some c <= 65535")
    if np.any(b != np.arange(1, n + 1, dtype=np.uint64)):
        bad.append("key=1: squares64 != c+1 for some c <= 65535")
    return bad


def _rot(x: int) -> int:
    return ((x >> 32) | (x << 32)) & M64


def ctr_zero_closed_form(key: int) -> tuple[int, int]:
    """At ctr = 0: y = 0 and z = key, so round 1 gives 0, round 2 gives key, and
    with X = rot(rot(key)^2) the outputs are hi32(X^2 + key) (squares32) and
    t ^ hi32(rot(t)^2) with t = X^2 + key (squares64; round 5 adds y = 0)."""
    X = _rot((_rot(key) ** 2) & M64)
    t = (X * X + key) & M64
    return t >> 32, t ^ (((_rot(t) ** 2) & M64) >> 32)


def pin_ctr_zero(impl) -> list[str]:
    g = np.random.Generator(np.random.PCG64(12))
    keys = [int(v) for v in g.integers(0, 1 << 64, size=300, dtype=np.uint64, endpoint=False)] + EDGE_WORDS
    k = _u64(keys)
    c = np.zeros_like(k)
    a = impl.sq32(c, k)
    b = impl.sq64(c, k)
    bad = []
    for i, kk in enumerate(keys):
        e32, e64 = ctr_zero_closed_form(kk)
        if int(a[i]) != e32 or int(b[i]) != e64:
            bad.append(f"ctr=0 closed form fails at key {kk:#x}")
            break
    return bad


def pin_hi32(impl) -> list[str]:
    """hi32(squares64(c,k)) == squares32(c,k): squares64 keeps round 4's full
    half square t (Section 5) whose upper half is squares32's output, and the
    round-5 term is shifted right by 32 so it only touches the low half."""
    c, k = _rand_pairs(13, 3000)
    a = impl.sq32(c, k)
    b = impl.sq64(c, k)
    if np.any((b >> np.uint64(32)) != a):
        return ["hi32(squares64) != squares32"]
    return []


def balance_screen(u: np.ndarray, bits: int, p_min: float = 1e-6) -> list[str]:
    """Gross-error screen on outputs: monobit count, per-bit-position balance
    (chi-square, df = bits) and byte-value histogram (chi-square, df = 255)."""
    bad = []
    n = u.size
    dtype = np.uint32 if bits == 32 else np.uint64
    by = np.ascontiguousarray(u.astype(dtype)).view(np.uint8)
    bitmat = np.unpackbits(by.reshape(n, bits // 8), axis=1, bitorder="little")
    ones_per_pos = bitmat.sum(axis=0, dtype=np.int64)
    total = int(ones_per_pos.sum())
    z = (total - n * bits / 2) / np.sqrt(n * bits / 4)
    p_mono = 2 * stats.norm.sf(abs(z))
    chi_pos = float((((ones_per_pos - n / 2) ** 2) / (n / 4)).sum())
    p_pos = stats.chi2.sf(chi_pos, bits)
    hist = np.bincount(by, minlength=256)
    exp = by.size / 256
    chi_byte = float((((hist - exp) ** 2) / exp).sum())
    p_byte = stats.chi2.sf(chi_byte, 255)
    for name, p in (("monobit", p_mono), ("bit-position", p_pos), ("byte", p_byte)):
        if p < p_min:
            bad.append(f"{name} balance p={p:.3g} (bits={bits})")
    return bad


SCREEN_KEY = 0x8B5AD4CEF3C97A61  # distinct-digit key (upper 8B5AD4CE, lower F3C97A61)


def pin_balance(impl, n: int = 1 << 20) -> list[str]:
    return (balance_screen(impl.range32(SCREEN_KEY, 0, n), 32)
            + balance_screen(impl.range64(SCREEN_KEY, 0, n), 64))


ALL_PINS = {
    "key_zero": pin_key_zero,
    "worked_examples": pin_worked_examples,
    "key_one": pin_key_one,
    "ctr_zero": pin_ctr_zero,
    "hi32": pin_hi32,
    "balance": pin_balance,
}


# ----------------------------------------------------------------------------
class OracleImpl:
    """The CPU oracle seen through the pin interface."""

    def __init__(self, oracle):
        self.o = oracle

    def sq32(self, ctr, key):
        return np.array([self.o.squares32(int(c), int(k)) for c, k in zip(ctr, key)], dtype=np.uint64)

    def sq64(self, ctr, key):
        return np.array([self.o.squares64(int(c), int(k)) for c, k in zip(ctr, key)], dtype=np.uint64)

    def range32(self, key, ctr0, n):
        return self.o.fill(self.o.U32, key, ctr0, n).astype(np.uint64)

    def range64(self, key, ctr0, n):
        return self.o.fill(self.o.U64, key, ctr0, n)
