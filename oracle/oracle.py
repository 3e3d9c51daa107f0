"""CPU oracle for the Squares counter-based RNG (arXiv 2004.06278).

TEST INFRASTRUCTURE ONLY.  Python wrapper around the plain C oracle in
``squares_oracle.c``.  Only the test suite, the smoke check and the
benchmark's CPU-baseline leg may import this module.  It shares nothing with
the GPU library: it neither imports the package nor loads ``libsquares.so``.

Every function here either forwards to the C oracle or is a plain definition
written out (the correctly rounded double of an exact sum uses Python's
``fractions.Fraction``, whose conversion to float rounds to nearest-even).
"""
from __future__ import annotations

import ctypes
import os
import subprocess
import threading
from fractions import Fraction

import numpy as np

HERE = os.path.dirname(os.path.abspath(__file__))
SRC = os.path.join(HERE, "squares_oracle.c")
LIB = os.path.join(HERE, "liboracle.so")

# Output kinds (must match the enum in squares_oracle.c).
U32, F32, U64, F64, U32X2, F32X2 = 0, 1, 2, 3, 4, 5
KIND_BYTES = {U32: 4, F32: 4, U64: 8, F64: 8, U32X2: 4, F32X2: 4}
KIND_DTYPE = {U32: np.uint32, F32: np.float32, U64: np.uint64, F64: np.float64, U32X2: np.uint32,
              F32X2: np.float32}
# Power-of-two scale of the integer sum of each kind: value = sum * 2^scale.
KIND_SUM_SCALE = {U32: 0, F32: -24, U64: 0, F64: -53, U32X2: 0, F32X2: -24}


def build(force: bool = False) -> str:
    """Compile the C oracle with gcc into ``liboracle.so`` next to it."""
    if force or not os.path.exists(LIB) or os.path.getmtime(LIB) < os.path.getmtime(SRC):
        tmp = LIB + ".tmp"
        subprocess.check_call(
            ["gcc", "-O2", "-std=c11", "-Wall", "-Wextra", "-fPIC", "-shared", SRC, "-o", tmp]
        )
        os.replace(tmp, LIB)
    return LIB


_lib = None
_lib_lock = threading.Lock()


def lib() -> ctypes.CDLL:
    global _lib
    with _lib_lock:
        if _lib is None:
            path = LIB if os.path.exists(LIB) else build()
            L = ctypes.CDLL(path)
            u64, u32, vp = ctypes.c_uint64, ctypes.c_uint32, ctypes.c_void_p
            L.oracle_squares32.argtypes = [u64, u64]
            L.oracle_squares32.restype = u32
            L.oracle_squares64.argtypes = [u64, u64]
            L.oracle_squares64.restype = u64
            L.oracle_trace.argtypes = [u64, u64, vp]
            L.oracle_trace.restype = None
            L.oracle_to_f32.argtypes = [u32]
            L.oracle_to_f32.restype = ctypes.c_float
            L.oracle_to_f64.argtypes = [u64]
            L.oracle_to_f64.restype = ctypes.c_double
            for name in ("oracle_fill_u32", "oracle_fill_u64", "oracle_fill_f32", "oracle_fill_f64",
                         "oracle_fill_u32x2", "oracle_fill_f32x2"):
                fn = getattr(L, name)
                fn.argtypes = [u64, u64, u64, vp]
                fn.restype = None
            L.oracle_kind_bytes.argtypes = [ctypes.c_int]
            L.oracle_kind_bytes.restype = ctypes.c_int
            L.oracle_fill_batch.argtypes = [u32, vp, vp, vp, vp, vp, vp]
            L.oracle_fill_batch.restype = ctypes.c_int
            L.oracle_sum.argtypes = [ctypes.c_int, u64, u64, u64, vp]
            L.oracle_sum.restype = ctypes.c_int
            L.oracle_trace_batch.argtypes = [vp, vp, u64, vp]
            L.oracle_trace_batch.restype = None
            L.oracle_fill_strided.argtypes = [ctypes.c_int, u64, u64, u64, u64, vp]
            L.oracle_fill_strided.restype = ctypes.c_int
            L.oracle_fill_keys.argtypes = [ctypes.c_int, u64, vp, u64, vp]
            L.oracle_fill_keys.restype = ctypes.c_int
            L.oracle_key_index.argtypes = [u64, u64]
            L.oracle_key_index.restype = u64
            L.oracle_key_upper.argtypes = [u64]
            L.oracle_key_upper.restype = ctypes.c_uint32
            L.oracle_key_lower.argtypes = [u64]
            L.oracle_key_lower.restype = ctypes.c_uint32
            L.oracle_make_keys.argtypes = [u64, u64, u64, vp]
            L.oracle_make_keys.restype = ctypes.c_int
            _lib = L
    return _lib


def _ptr(a: np.ndarray) -> int:
    assert a.flags["C_CONTIGUOUS"]
    return a.ctypes.data


# ---------------------------------------------------------------- scalars
def squares32(ctr: int, key: int) -> int:
    """squares32(ctr, key), Section 2."""
    return int(lib().oracle_squares32(ctr & (2**64 - 1), key & (2**64 - 1)))


def squares64(ctr: int, key: int) -> int:
    """squares64(ctr, key), Section 5."""
    return int(lib().oracle_squares64(ctr & (2**64 - 1), key & (2**64 - 1)))


def trace(ctr: int, key: int) -> list[int]:
    """x after each of the five half squares (before rotation)."""
    t = np.zeros(5, dtype=np.uint64)
    lib().oracle_trace(ctr & (2**64 - 1), key & (2**64 - 1), _ptr(t))
    return [int(v) for v in t]


# ---------------------------------------------------------------- bulk
_FILL = {U32: "oracle_fill_u32", F32: "oracle_fill_f32", U64: "oracle_fill_u64", F64: "oracle_fill_f64",
         U32X2: "oracle_fill_u32x2", F32X2: "oracle_fill_f32x2"}


def fill(kind: int, key: int, ctr0: int, n: int, threads: int = 1) -> np.ndarray:
    """out[i] = kind's value at counter ctr0 + i (mod 2^64), i in [0, n).

    ``threads`` > 1 splits [0, n) into contiguous chunks, each a separate call
    of the same C routine (ctypes releases the GIL during the call)."""
    out = np.empty(n, dtype=KIND_DTYPE[kind])
    fill_into(kind, key, ctr0, out, threads)
    return out


def fill_into(kind: int, key: int, ctr0: int, out: np.ndarray, threads: int = 1) -> None:
    fn = getattr(lib(), _FILL[kind])
    n = out.size
    key &= 2**64 - 1
    ctr0 &= 2**64 - 1
    if threads <= 1 or n < 4096:
        fn(key, ctr0, n, _ptr(out))
        return
    # chunks start at even elements so a split kind's chunk starts at a low half
    bounds = [(n * t // threads) & ~1 for t in range(threads)] + [n]
    width = out.itemsize
    base = _ptr(out)
    per_ctr = 2 if kind in (U32X2, F32X2) else 1

    def work(t: int) -> None:
        a, b = bounds[t], bounds[t + 1]
        fn(key, (ctr0 + a // per_ctr) & (2**64 - 1), b - a, base + a * width)

    ts = [threading.Thread(target=work, args=(t,)) for t in range(threads)]
    for th in ts:
        th.start()
    for th in ts:
        th.join()


def trace_batch(ctrs, keys) -> np.ndarray:
    """Per-round values (m x 5) of each (ctr, key) pair, as oracle_trace."""
    ctrs = np.ascontiguousarray(ctrs, dtype=np.uint64)
    keys = np.ascontiguousarray(keys, dtype=np.uint64)
    out = np.empty((ctrs.size, 5), dtype=np.uint64)
    lib().oracle_trace_batch(_ptr(ctrs), _ptr(keys), ctrs.size, _ptr(out))
    return out


def fill_strided(kind: int, key: int, ctr0: int, step: int, n: int) -> np.ndarray:
    """out[i] = kind's value at counter ctr0 + i*step (split kinds: word i%2 at
    ctr0 + (i//2)*step)."""
    out = np.empty(n, dtype=KIND_DTYPE[kind])
    if lib().oracle_fill_strided(kind, key & (2**64 - 1), ctr0 & (2**64 - 1), step & (2**64 - 1), n,
                                 _ptr(out)) != 0:
        raise ValueError("unknown kind")
    return out


def fill_keys(kind: int, ctr: int, keys) -> np.ndarray:
    """Key-counter mode: out[j] = kind's value at counter ctr under keys[j]."""
    keys = np.ascontiguousarray(keys, dtype=np.uint64)
    out = np.empty(keys.size, dtype=KIND_DTYPE[kind])
    if lib().oracle_fill_keys(kind, ctr & (2**64 - 1), _ptr(keys), keys.size, _ptr(out)) != 0:
        raise ValueError("kind not available in key-counter mode")
    return out


KEY_CHOICES_HI = 16 * 15 * 14 * 13 * 12 * 11 * 10 * 9
KEY_CHOICES_LO = 8 * 15 * 14 * 13 * 12 * 11 * 10 * 9


def key_index(r: int, choices: int) -> int:
    return int(lib().oracle_key_index(r & (2**64 - 1), choices))


def key_upper(u: int) -> int:
    return int(lib().oracle_key_upper(u))


def key_lower(u: int) -> int:
    return int(lib().oracle_key_lower(u))


def make_keys(gen_key: int, ctr0: int, m: int) -> np.ndarray:
    """Distinct-digit keys: key j from squares64 at counters ctr0 + 2j and
    ctr0 + 2j + 1 under gen_key."""
    out = np.empty(m, dtype=np.uint64)
    lib().oracle_make_keys(gen_key & (2**64 - 1), ctr0 & (2**64 - 1), m, _ptr(out))
    return out


def fill_batch(keys, ctr0s, lens, offs, kinds, out_bytes: int) -> np.ndarray:
    """Ragged batch into one byte arena of ``out_bytes`` (zero where no stream writes)."""
    keys = np.ascontiguousarray(keys, dtype=np.uint64)
    ctr0s = np.ascontiguousarray(ctr0s, dtype=np.uint64)
    lens = np.ascontiguousarray(lens, dtype=np.uint64)
    offs = np.ascontiguousarray(offs, dtype=np.uint64)
    kinds = np.ascontiguousarray(kinds, dtype=np.uint8)
    m = keys.size
    assert ctr0s.size == lens.size == offs.size == kinds.size == m
    out = np.zeros(out_bytes, dtype=np.uint8)
    for s in range(m):
        if int(offs[s]) + int(lens[s]) * KIND_BYTES[int(kinds[s])] > out_bytes:
            raise ValueError(f"stream {s} runs past the arena")
    rc = lib().oracle_fill_batch(m, _ptr(keys), _ptr(ctr0s), _ptr(lens), _ptr(offs), _ptr(kinds), _ptr(out))
    if rc != 0:
        raise ValueError("unknown kind")
    return out


def exact_sum(kind: int, key: int, ctr0: int, n: int, threads: int = 1) -> int:
    """Exact integer sum of the kind's integers over [ctr0, ctr0+n) (an int < 2^128)."""
    key &= 2**64 - 1
    ctr0 &= 2**64 - 1
    if threads <= 1 or n < 65536:
        o = np.zeros(2, dtype=np.uint64)
        if lib().oracle_sum(kind, key, ctr0, n, _ptr(o)) != 0:
            raise ValueError("unknown kind")
        return int(o[0]) | (int(o[1]) << 64)
    bounds = [(n * t // threads) & ~1 for t in range(threads)] + [n]
    parts = [np.zeros(2, dtype=np.uint64) for _ in range(threads)]
    per_ctr = 2 if kind in (U32X2, F32X2) else 1

    def work(t: int) -> None:
        a, b = bounds[t], bounds[t + 1]
        lib().oracle_sum(kind, key, (ctr0 + a // per_ctr) & (2**64 - 1), b - a, _ptr(parts[t]))

    ts = [threading.Thread(target=work, args=(t,)) for t in range(threads)]
    for th in ts:
        th.start()
    for th in ts:
        th.join()
    return sum(int(p[0]) | (int(p[1]) << 64) for p in parts)


def rounded_value(kind: int, s: int) -> float:
    """The double nearest (ties to even) to s * 2^scale(kind)."""
    return float(Fraction(s) * Fraction(2) ** KIND_SUM_SCALE[kind])
