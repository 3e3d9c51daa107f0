"""Seeded synthetic inputs for the Squares RNG workloads.

This module only draws inputs (keys, starting counters, stream lengths,
kinds, byte offsets, arrival times).  It holds none of the generator's
arithmetic, imports neither the GPU binding nor the CPU oracle, and is the
one module both sides receive their inputs from.

Keys follow the paper's advice (Section 3, Discussion): an irregular bit
pattern whose upper 8 hex digits are mutually different and whose lower 8
hex digits are mutually different, the digits chosen at random.  The least
significant digit is drawn first from the odd digits (a reading where the
paper is silent: an odd key makes ctr -> ctr*key a bijection mod 2^64).
"""
from __future__ import annotations

import math
from dataclasses import dataclass

import numpy as np

# Output kinds: U32/F32 come from squares32, U64/F64 from squares64, and
# U32X2/F32X2 split each squares64 output into two 32-bit outputs.
U32, F32, U64, F64, U32X2, F32X2 = 0, 1, 2, 3, 4, 5
KIND_BYTES = {U32: 4, F32: 4, U64: 8, F64: 8, U32X2: 4, F32X2: 4}
KIND_ALIGN = {U32: 4, F32: 4, U64: 8, F64: 8, U32X2: 8, F32X2: 8}
KIND_NAMES = {U32: "u32", F32: "f32", U64: "u64", F64: "f64", U32X2: "u32x2", F32X2: "f32x2"}

MASK64 = (1 << 64) - 1


def rng(seed: int) -> np.random.Generator:
    return np.random.Generator(np.random.PCG64(seed))


def distinct_digit_key(g: np.random.Generator) -> int:
    """One key: each 8-digit half is 8 different hex digits in random order,
    the last digit odd."""
    hi = [int(d) for d in g.permutation(16)[:8]]
    odd = 2 * int(g.integers(0, 8)) + 1
    lo = [int(d) for d in g.permutation(16) if d != odd][:7] + [odd]
    key = 0
    for d in hi + lo:
        key = (key << 4) | d
    return key


def distinct_digit_keys(g: np.random.Generator, m: int) -> np.ndarray:
    return np.array([distinct_digit_key(g) for _ in range(m)], dtype=np.uint64)


def uniform_u64(g: np.random.Generator, size=None):
    v = g.integers(0, 1 << 64, size=size, dtype=np.uint64, endpoint=False)
    return int(v) if size is None else v


def log_uniform_lengths(g: np.random.Generator, m: int, lo_exp: float, hi_exp: float) -> np.ndarray:
    """floor(2^U) with U ~ Uniform[lo_exp, hi_exp), clipped to [2^lo_exp, 2^hi_exp]."""
    u = g.uniform(lo_exp, hi_exp, size=m)
    n = np.floor(np.exp2(u)).astype(np.uint64)
    return np.clip(n, np.uint64(2**lo_exp), np.uint64(2**hi_exp)).astype(np.uint64)


# --------------------------------------------------------------------------
# Single key (plain fill; single-key throughput)
# --------------------------------------------------------------------------
@dataclass
class SingleKey:
    key: int
    ctr0: int
    n: int


def plain_fill_case(seed: int = 1, n: int = 1 << 24) -> SingleKey:
    """One distinct-digit key, counters 0 .. n-1 (the 64 MiB squares32 fill)."""
    g = rng(seed)
    return SingleKey(key=distinct_digit_key(g), ctr0=0, n=n)


def single_key_case(seed: int = 2, n: int = 1 << 32) -> SingleKey:
    """One distinct-digit key, a uniformly random 64-bit starting counter."""
    g = rng(seed)
    key = distinct_digit_key(g)
    return SingleKey(key=key, ctr0=uniform_u64(g), n=n)


# --------------------------------------------------------------------------
# Ragged batches
# --------------------------------------------------------------------------
@dataclass
class Batch:
    keys: np.ndarray   # uint64[m]
    ctr0s: np.ndarray  # uint64[m]
    lens: np.ndarray   # uint64[m]
    offs: np.ndarray   # uint64[m], byte offsets into one arena
    kinds: np.ndarray  # uint8[m]
    arena_bytes: int

    @property
    def m(self) -> int:
        return int(self.keys.size)

    @property
    def total_outputs(self) -> int:
        return int(self.lens.sum(dtype=np.uint64))


def pack_offsets(lens: np.ndarray, kinds: np.ndarray, g: np.random.Generator | None = None,
                 max_pad_words: int = 0, align: int = 4) -> tuple[np.ndarray, int]:
    """Exclusive prefix of the byte sizes; with ``max_pad_words`` > 0 each stream
    is preceded by a random gap of 0..max_pad_words ``align``-byte words, so
    streams start at arbitrary ``align``-byte offsets."""
    sizes = [int(l) * KIND_BYTES[int(k)] for l, k in zip(lens, kinds)]
    offs = np.zeros(len(sizes), dtype=np.uint64)
    pos = 0
    for s, sz in enumerate(sizes):
        a = max(KIND_ALIGN[int(kinds[s])], align)
        if g is not None and max_pad_words > 0:
            pos += a * int(g.integers(0, max_pad_words + 1))
        pos = (pos + a - 1) // a * a
        offs[s] = pos
        pos += sz
    return offs, pos


def ragged_batch(seed: int = 3, m: int = 4096, lo_exp: float = 10, hi_exp: float = 24,
                 kinds=(U32, F32), misalign: bool = False) -> Batch:
    """Many keys with log-uniform stream lengths in [2^lo_exp, 2^hi_exp],
    uniform 64-bit starting counters and kinds drawn evenly from ``kinds``."""
    g = rng(seed)
    keys = distinct_digit_keys(g, m)
    ctr0s = uniform_u64(g, m)
    lens = log_uniform_lengths(g, m, lo_exp, hi_exp)
    kk = np.array(kinds, dtype=np.uint8)[g.integers(0, len(kinds), size=m)]
    offs, total = pack_offsets(lens, kk, g if misalign else None, 3 if misalign else 0)
    return Batch(keys, ctr0s, lens, offs, kk, total)


def wrap_batch(seed: int = 4, m: int = 65536, max_len: int = 65536, near: int = 1 << 16) -> Batch:
    """squares64 streams whose counters start within ``near`` of 2^64, so about
    half of them pass 2^64 - 1 and continue at 0; lengths uniform in [1, max_len];
    kinds U64 / F64 evenly."""
    g = rng(seed)
    keys = distinct_digit_keys(g, m)
    d = g.integers(1, near + 1, size=m, dtype=np.uint64)
    ctr0s = (np.uint64(0) - d).astype(np.uint64)  # 2^64 - d
    lens = g.integers(1, max_len + 1, size=m, dtype=np.uint64)
    kk = np.array([U64, F64], dtype=np.uint8)[g.integers(0, 2, size=m)]
    offs, total = pack_offsets(lens, kk)
    return Batch(keys, ctr0s, lens, offs, kk, total)


def small_random_batch(seed: int, m: int, max_len: int, kinds=(U32, F32, U64, F64),
                       misalign: bool = True, zero_frac: float = 0.1) -> Batch:
    """Small mixed batch for parity tests: random lengths (some empty), random
    kinds, keys of every kind (distinct-digit, zero, even), counters anywhere."""
    g = rng(seed)
    keys = distinct_digit_keys(g, m)
    special = g.integers(0, 8, size=m)
    keys[special == 0] = 0
    keys[special == 1] = uniform_u64(g, int((special == 1).sum())) & np.uint64(~1 & MASK64)
    ctr0s = uniform_u64(g, m)
    near_wrap = g.integers(0, 4, size=m) == 0
    ctr0s[near_wrap] = (np.uint64(0) - g.integers(1, max_len + 2, size=int(near_wrap.sum()), dtype=np.uint64))
    lens = g.integers(0, max_len + 1, size=m, dtype=np.uint64)
    lens[g.random(m) < zero_frac] = 0
    kk = np.array(kinds, dtype=np.uint8)[g.integers(0, len(kinds), size=m)]
    offs, total = pack_offsets(lens, kk, g if misalign else None, 5 if misalign else 0)
    return Batch(keys, ctr0s, lens, offs, kk, total)


# --------------------------------------------------------------------------
# Serving trace
# --------------------------------------------------------------------------
@dataclass
class ServeTrace:
    arrival_s: np.ndarray  # float64[r], seconds from start
    kinds: np.ndarray      # uint8[r]
    keys: np.ndarray       # uint64[r]
    ctr0s: np.ndarray      # uint64[r]
    sizes: np.ndarray      # uint64[r], outputs per request

    @property
    def r(self) -> int:
        return int(self.sizes.size)


def serve_trace(seed: int = 5, r: int = 21000, qps: float = 1000.0, lo_exp: float = 10,
                hi_exp: float = 28, frac32: float = 0.7) -> ServeTrace:
    """Poisson arrivals at ``qps``; sizes log-uniform in [2^lo_exp, 2^hi_exp];
    ``frac32`` of requests are 32-bit (U32/F32 evenly), the rest 64-bit
    (U64/F64 evenly); per-request distinct-digit key and uniform counter."""
    g = rng(seed)
    gaps = g.exponential(1.0 / qps, size=r)
    arrival = np.cumsum(gaps) - gaps[0]
    is32 = g.random(r) < frac32
    half = g.integers(0, 2, size=r)
    kinds = np.where(is32, np.where(half == 0, U32, F32), np.where(half == 0, U64, F64)).astype(np.uint8)
    keys = distinct_digit_keys(g, r)
    ctr0s = uniform_u64(g, r)
    sizes = log_uniform_lengths(g, r, lo_exp, hi_exp)
    return ServeTrace(arrival, kinds, keys, ctr0s, sizes)


def expected_log_uniform_mean(lo_exp: float, hi_exp: float) -> float:
    """E[2^U] for U ~ Uniform[lo_exp, hi_exp) (ignoring the floor)."""
    return (2.0**hi_exp - 2.0**lo_exp) / ((hi_exp - lo_exp) * math.log(2.0))
