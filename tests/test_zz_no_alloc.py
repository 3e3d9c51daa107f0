"""The no-allocation reduce (sq_reduce_noalloc, for callers that cannot
allocate) against sq_reduce, called through the C ABI: two calls in a row on
the library's shared device scratch, the second over fewer counters, each
equal to sq_reduce's result (exact 128-bit sum, rounded value, count)."""
from __future__ import annotations

import pytest

from gpu_helpers import log

pytestmark = pytest.mark.gpu

# (kind, key, ctr0, n): the first call spans many queue chunks and wraps the
# counter; the second is smaller, so a stale partial or queue count from the
# first would change its result
CASES = [
    [(1, 0xA76E20DFEB35F7D9, 2**64 - 5000, (1 << 26) + 12345), (1, 0xA76E20DFEB35F7D9, 7, 100003)],
    [(3, 0x5D3F2A1B9C8E7641, 0x82D5383A946972CA, 1 << 27), (0, 0x5D3F2A1B9C8E7641, 1, 777)],
    [(2, 0x1F2E3D4C5B6A7989, 0, (1 << 25) + 1), (5, 0x1F2E3D4C5B6A7989, 2**63, 4097)],
]


@pytest.mark.parametrize("calls", CASES, ids=["f32-then-f32", "f64-then-u32", "u64-then-f32x2"])
def test_noalloc_reduce_matches_reduce_twice(calls, oracle_mod):
    from paper_2004_06278_amd import squares as sq

    sq.lib().sq_init()
    for kind, key, ctr0, n in calls:
        log(f"sq_reduce_noalloc kind={kind} key={key:#x} ctr0={ctr0:#x} n={n}")
        got = sq.result_tensor()
        sq.reduce_noalloc_async(kind, key, ctr0, n, got)
        got_sum = sq.read_result(got)
        want = sq.reduce(kind, key, ctr0, n)
        assert got_sum == want, (kind, n, got_sum, want)
        if n < (1 << 20):  # small enough for the oracle as well
            assert got_sum[0] == oracle_mod.exact_sum(kind, key, ctr0, n)


def test_noalloc_reduce_zero_and_errors():
    from paper_2004_06278_amd import squares as sq

    got = sq.result_tensor()
    got.fill_(0xFF)
    sq.reduce_noalloc_async(1, 0x1234567, 99, 0, got)
    assert sq.read_result(got) == (0, 0.0, 0)
    with pytest.raises(sq.SquaresError):
        sq.reduce_noalloc_async(9, 1, 0, 10, got)  # unknown kind
