"""GPU tests of the continuous-batching server: every request's output equals
the oracle and the same request served alone; admission by HBM budget,
cancellation, error paths and draining."""
from __future__ import annotations

import time

import numpy as np
import pytest

from gpu_helpers import HOST_THREADS, KIND_BYTES, first_diff, log, oracle_element, to_host_bytes

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def sq():
    from paper_2004_06278_amd import squares

    squares.lib()
    return squares


def _oracle(o, kind, key, ctr0, n):
    return o.fill(kind, key, ctr0, n).view(np.uint8)


def _mix(seed, r, max_log2):
    from paper_2004_06278_amd import workloads as W

    tr = W.serve_trace(seed=seed, r=r, qps=1e9, lo_exp=0, hi_exp=max_log2)
    return [(int(tr.kinds[i]), int(tr.keys[i]), int(tr.ctr0s[i]), int(tr.sizes[i])) for i in range(r)]


@pytest.mark.parametrize("n_streams,chunk_cap,tick_bytes",
                         [(1, 4096, 0), (2, 1 << 14, 0), (3, 1 << 20, 0), (2, 1 << 14, 100_000)])
def test_server_alone_equals_mix_equals_oracle(sq, oracle_mod, n_streams, chunk_cap, tick_bytes):
    probe = (3, 0x6C8E9CF570932BD5, 2**64 - 70000, 150001)  # F64, wraps the counter, spans many ticks
    log(f"server alone n_streams={n_streams} chunk_cap={chunk_cap} tick_bytes={tick_bytes}")
    with sq.Server(64 << 20, max_slots=64, chunk_cap=chunk_cap, n_streams=n_streams,
                   tick_bytes=tick_bytes) as srv:
        rid = srv.submit(*probe)
        srv.wait(rid)
        alone = to_host_bytes(srv.result_bytes(rid))
        srv.release(rid)
    ref = _oracle(oracle_mod, *probe)
    assert alone.tobytes() == ref.tobytes(), first_diff(alone, ref)

    reqs = _mix(seed=40 + n_streams, r=120, max_log2=17)
    # split-word requests too (odd lengths end on a low word)
    reqs += [(4 + (i % 2), 0x3F1E5D7C9B2A4068 + i, 2**64 - 1000 * i - 1, 1000 * i + 7) for i in range(1, 9)]
    reqs.insert(60, probe)
    log(f"server mix of {len(reqs)} requests")
    with sq.Server(256 << 20, max_slots=48, chunk_cap=chunk_cap, n_streams=n_streams,
                   tick_bytes=tick_bytes) as srv:
        ids = [srv.submit(*q) for q in reqs]
        for rid in ids:
            srv.wait(rid)
        for q, rid in zip(reqs, ids):
            got = to_host_bytes(srv.result_bytes(rid))
            exp = _oracle(oracle_mod, *q)
            assert got.tobytes() == exp.tobytes(), (q, first_diff(got, exp))
            if q == probe:
                assert got.tobytes() == alone.tobytes()  # same bits alone and in the mix
            assert srv.latency(rid) > 0
            srv.release(rid)
        st = srv.stats()
        assert st["completed"] == len(reqs) == st["released"]
        assert st["arena_used_bytes"] == 0 and st["active_now"] == 0


K1, K2, K3 = 0x6C8E9CF570932BD5, 0x3F1E5D7C9B2A4069, 0x1234567890ABCDEF


@pytest.mark.parametrize("reqs,n_streams", [
    ([(0, K1, 0, 20000), (0, K2, 100, 20000)], 1),
    ([(0, K1, 0, 20000), (0, K2, 100, 5)], 1),
    ([(0, K1, 0, 5), (0, K2, 100, 20000)], 1),
    ([(0, K1, 0, 20000), (3, K2, 2**64 - 3000, 20000), (4, K3, 7, 9001)], 1),
    ([(0, K1, 0, 20000), (0, K2, 100, 20000), (5, K3, 2**64 - 1, 12345)], 2),
])
def test_server_multi_chunk_requests_share_ticks(sq, oracle_mod, reqs, n_streams):
    """Several multi-chunk requests in the same ticks: each request's state
    lives in its device slot and is advanced once per tick (a request takes
    at most one chunk of a tick), so every output matches the oracle."""
    log(f"server multi-chunk {[(q[0], q[3]) for q in reqs]} n_streams={n_streams}")
    with sq.Server(64 << 20, max_slots=64, chunk_cap=4096, n_streams=n_streams) as srv:
        ids = [srv.submit(*q) for q in reqs]
        for rid in ids:
            srv.wait(rid)
        for q, rid in zip(reqs, ids):
            got = to_host_bytes(srv.result_bytes(rid))
            exp = _oracle(oracle_mod, *q)
            assert got.tobytes() == exp.tobytes(), (q, first_diff(got, exp))
        # one chunk per request per tick: at least as many ticks as the longest request has chunks
        assert srv.stats()["ticks"] >= max(-(-q[3] // 4096) for q in reqs)


@pytest.mark.parametrize("n_streams,max_slots,chunk_cap", [(4, 4, 4096), (3, 16, 8192), (4, 64, 1 << 16)])
def test_server_slot_reuse_stress(sq, oracle_mod, n_streams, max_slots, chunk_cap):
    """Hundreds of requests of every kind through few slots on several lanes:
    each device slot is reused many times, by requests whose chunks run on
    different lanes; every output equals the oracle."""
    rng = np.random.default_rng(1000 + max_slots)
    reqs = []
    for i in range(400):
        kind = int(rng.integers(0, 6))
        n = int(2 ** rng.uniform(0, 16))
        ctr0 = int(rng.integers(0, 2**64, dtype=np.uint64)) if i % 3 else 2**64 - int(rng.integers(1, 70000))
        reqs.append((kind, int(rng.integers(0, 2**64, dtype=np.uint64)), ctr0, n))
    log(f"server stress n_streams={n_streams} max_slots={max_slots} chunk_cap={chunk_cap}")
    with sq.Server(64 << 20, max_slots=max_slots, chunk_cap=chunk_cap, n_streams=n_streams) as srv:
        ids = [srv.submit(*q) for q in reqs]
        for q, rid in zip(reqs, ids):
            srv.wait(rid)
            got = to_host_bytes(srv.result_bytes(rid))
            exp = _oracle(oracle_mod, *q)
            assert got.tobytes() == exp.tobytes(), (q, first_diff(got, exp))
            srv.release(rid)
        st = srv.stats()
        assert st["completed"] == len(reqs) == st["released"]


def test_server_admission_by_budget_queues(sq, oracle_mod):
    """More requests than the arena holds at once: later ones wait in the
    queue until earlier outputs are released, then complete correctly."""
    budget = 1 << 20
    reqs = [(k % 4, 0x1234567 + k, k * 1000003, 60000) for k in range(12)]  # 240-480 KB each
    with sq.Server(budget, max_slots=16, chunk_cap=1 << 14, n_streams=2) as srv:
        ids = [srv.submit(*q) for q in reqs]
        time.sleep(0.05)
        st = srv.stats()
        assert st["queued_now"] > 0, st  # the budget cannot hold all twelve
        for q, rid in zip(reqs, ids):
            srv.wait(rid)
            got = to_host_bytes(srv.result_bytes(rid))
            assert got.tobytes() == _oracle(oracle_mod, *q).tobytes()
            srv.release(rid)
        assert srv.stats()["completed"] == len(reqs)


def test_server_errors_and_cancel(sq):
    with sq.Server(1 << 20, max_slots=4, chunk_cap=4096, n_streams=1) as srv:
        with pytest.raises(sq.SquaresError) as e:
            srv.submit(0, 1, 0, (1 << 20) // 4 + 1)  # larger than the whole budget
        assert e.value.status == -3
        with pytest.raises(sq.SquaresError) as e:
            srv.submit(9, 1, 0, 10)
        assert e.value.status == -1
        with pytest.raises(sq.SquaresError) as e:
            srv.submit(0, 1, 0, 0)
        assert e.value.status == -1
        big = srv.submit(2, 5, 0, (1 << 20) // 8)  # fills the arena
        small = srv.submit(0, 6, 0, 100)           # must wait for `big` to be released
        srv.wait(big)
        time.sleep(0.02)
        assert not srv.poll(small)
        srv.cancel(small)
        with pytest.raises(sq.SquaresError) as e:
            srv.poll(small)
        assert e.value.status == -6
        with pytest.raises(sq.SquaresError) as e:
            srv.cancel(big)  # already admitted
        assert e.value.status == -5
        srv.release(big)
        with pytest.raises(sq.SquaresError):
            srv.release(big)
    with pytest.raises(sq.SquaresError):
        sq.Server(1 << 20, n_streams=0)


def test_server_discard_and_no_stats_flags(sq):
    """SERVE_DISCARD frees a request's output as soon as it completes (poll
    reports it done, result() no longer finds it, the arena is empty again);
    SERVE_NO_STATS leaves a request out of the latency statistics."""
    with sq.Server(64 << 20, max_slots=8, chunk_cap=1 << 16, n_streams=2) as srv:
        flags = sq.SERVE_DISCARD | sq.SERVE_NO_STATS
        ids = [srv.submit(k % 4, 77 + k, k << 30, (1 << 18) + k, flags) for k in range(6)]
        for r in ids:
            srv.wait(r)
            assert srv.poll(r)
            with pytest.raises(sq.SquaresError) as e:
                srv.result(r)
            assert e.value.status == -6
        st = srv.stats()
        assert st["completed"] == st["released"] == 6
        assert st["arena_used_bytes"] == 0 and st["active_now"] == 0
        assert st["p50_s"] == 0 and st["max_s"] == 0          # no latency sample yet
        kept = srv.submit(0, 5, 0, 1000)
        srv.wait(kept)
        st = srv.stats()
        assert st["max_s"] > 0 and st["p50_s"] == st["max_s"] == srv.latency(kept)
        assert st["arena_used_bytes"] == 4096                  # 4000 bytes in 256-byte units
        srv.release(kept)
        assert srv.stats()["arena_used_bytes"] == 0


def test_server_full_size_requests_sampled(sq, oracle_mod):
    """The serving workload at its real sizes, in the benchmark's server
    configuration (32 GiB budget, 4096 slots, chunks of 2^24 outputs, 4
    lanes): 60 requests of the serving trace (log-uniform 2^10..2^28 outputs,
    70% 32-bit) plus two of 2^28 outputs (U32 and U64, the second wrapping its
    counter), submitted at once.  Requests below 2^20 outputs and the 2^28
    U32 request are compared whole (the latter in 2^26-output pieces); the
    other large ones on their first and last 2^14 outputs and 512 random
    positions, each against the oracle."""
    import torch

    from paper_2004_06278_amd import workloads as W

    tr = W.serve_trace(seed=8, r=60, qps=1e9)
    reqs = [(int(tr.kinds[i]), int(tr.keys[i]), int(tr.ctr0s[i]), int(tr.sizes[i])) for i in range(60)]
    reqs += [(0, 0x6C8E9CF570932BD5, 12345, 1 << 28), (2, 0x3F1E5D7C9B2A4069, 2**64 - (1 << 27), 1 << 28)]
    log(f"server full-size requests: {len(reqs)}, largest {max(q[3] for q in reqs)} outputs")
    g = np.random.Generator(np.random.PCG64(81))
    with sq.Server(32 << 30, max_slots=4096, chunk_cap=1 << 24, n_streams=4) as srv:
        ids = [srv.submit(*q) for q in reqs]
        for q, rid in zip(reqs, ids):
            srv.wait(rid)
            kind, key, ctr0, n = q
            W_ = KIND_BYTES[kind]
            out = srv.result_bytes(rid)
            if n < (1 << 20):
                got = to_host_bytes(out)
                exp = _oracle(oracle_mod, kind, key, ctr0, n)
                assert got.tobytes() == exp.tobytes(), (q, first_diff(got, exp))
            elif n == 1 << 28 and kind == 0:
                # the largest request size, compared whole in 2^26-output pieces
                piece = 1 << 26
                for base in range(0, n, piece):
                    got = to_host_bytes(out[base * W_:(base + piece) * W_])
                    exp = oracle_mod.fill(kind, key, (ctr0 + base) % 2**64, piece, threads=HOST_THREADS).view(np.uint8)
                    assert got.tobytes() == exp.tobytes(), (q, base, first_diff(got, exp))
            else:
                k = 1 << 14
                head = to_host_bytes(out[: k * W_])
                tail = to_host_bytes(out[(n - k) * W_:])
                assert head.tobytes() == _oracle(oracle_mod, kind, key, ctr0, k).tobytes(), q
                assert tail.tobytes() == _oracle(oracle_mod, kind, key, (ctr0 + n - k) % 2**64, k).tobytes(), q
                idx = g.integers(0, n, size=512)
                words = out.view(torch.int32 if W_ == 4 else torch.int64)
                got = words[torch.from_numpy(idx.astype(np.int64)).cuda()].cpu().numpy().view(np.uint8).reshape(-1, W_)
                for row, i in zip(got, idx):
                    assert row.tobytes() == oracle_element(oracle_mod, kind, key, ctr0, int(i)), (q, int(i))
            del out
            srv.release(rid)
        st = srv.stats()
        assert st["completed"] == len(reqs) == st["released"] and st["arena_used_bytes"] == 0
    torch.cuda.empty_cache()


def test_server_resume_from_saved_counter(sq, oracle_mod):
    """A stream checkpoint is (key, next counter): serving [c, c+a) then
    [c+a, c+a+b) gives the same outputs as serving [c, c+a+b) at once."""
    key, c, a, b = 0xD1B54A32D192ED03, 2**64 - 5000, 7777, 9999
    with sq.Server(16 << 20, max_slots=8, chunk_cap=4096, n_streams=2) as srv:
        r1 = srv.submit(0, key, c, a)
        r2 = srv.submit(0, key, (c + a) % 2**64, b)
        r3 = srv.submit(0, key, c, a + b)
        for r in (r1, r2, r3):
            srv.wait(r)
        two = np.concatenate([to_host_bytes(srv.result_bytes(r1)), to_host_bytes(srv.result_bytes(r2))])
        one = to_host_bytes(srv.result_bytes(r3))
        assert two.tobytes() == one.tobytes() == _oracle(oracle_mod, 0, key, c, a + b).tobytes()


def test_server_destroy_drains_in_flight_work(sq):
    srv = sq.Server(512 << 20, max_slots=64, chunk_cap=1 << 16, n_streams=2)
    for i in range(200):
        srv.submit(i % 4, 1000 + i, i << 20, 1 << 18, sq.SERVE_DISCARD)
    srv.close()  # returns after admitted work finished; queued requests are dropped


def test_server_open_loop_smoke(sq):
    """A short Poisson run: every request completes and percentiles are ordered."""
    import torch

    from paper_2004_06278_amd import serve_bench
    from paper_2004_06278_amd import workloads as W

    tr = W.serve_trace(seed=8, r=600, qps=5000.0, hi_exp=22)
    res = serve_bench.open_loop(sq, tr, budget=4 << 30, chunk_cap=1 << 22, warmup=100)
    torch.cuda.synchronize()
    assert res["requests"] == 500
    assert 0 < res["p50_ms"] <= res["p90_ms"] <= res["p99_ms"] <= res["max_ms"]
