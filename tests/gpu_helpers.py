"""Shared helpers of the GPU parity tests."""
from __future__ import annotations

import os
import sys
import threading

import numpy as np

KIND_BYTES = {0: 4, 1: 4, 2: 8, 3: 8, 4: 4, 5: 4}
KIND_ALIGN = {0: 4, 1: 4, 2: 8, 3: 8, 4: 8, 5: 8}
NP_DTYPE = {0: np.uint32, 1: np.float32, 2: np.uint64, 3: np.float64, 4: np.uint32, 5: np.float32}


def oracle_element(o, kind: int, key: int, ctr0: int, i: int) -> bytes:
    """Bytes of element i of a fill of `kind` from counter ctr0 (split kinds
    take word i & 1 of squares64 at ctr0 + i // 2)."""
    if kind in (4, 5):
        pair = o.fill(kind, key, (ctr0 + i // 2) % 2**64, 2).view(np.uint8)
        return pair[4 * (i & 1): 4 * (i & 1) + 4].tobytes()
    return o.fill(kind, key, (ctr0 + i) % 2**64, 1).view(np.uint8).tobytes()


HOST_THREADS = max(1, min(16, os.cpu_count() or 1))


def log(msg: str) -> None:
    """Names the case before a GPU step, so a failure can be traced."""
    print(f"[gpu-test] {msg}", flush=True)
    sys.stdout.flush()


def to_host_bytes(t) -> np.ndarray:
    import torch

    return t.contiguous().view(torch.uint8).cpu().numpy()


def oracle_bytes(o, kind: int, key: int, ctr0: int, n: int) -> np.ndarray:
    return o.fill(kind, key, ctr0, n, threads=HOST_THREADS).view(np.uint8)


def first_diff(a: np.ndarray, b: np.ndarray) -> str:
    idx = np.nonzero(a != b)[0]
    if idx.size == 0:
        return "equal"
    return f"{idx.size} differing bytes, first at byte {int(idx[0])}"


def compare_batch_arena(o, gpu_arena, batch, chunk_bytes: int = 1 << 30) -> list[str]:
    """Compares every stream of a batch with the oracle, downloading the arena
    in chunks of whole streams and evaluating the oracle on host threads."""
    import torch

    errors = []
    order = np.argsort(batch.offs)
    s_i = 0
    m = batch.m
    flat = gpu_arena.view(torch.uint8)
    while s_i < m:
        first = int(batch.offs[order[s_i]])
        j = s_i
        end = first
        while j < m:
            s = order[j]
            e = int(batch.offs[s]) + int(batch.lens[s]) * KIND_BYTES[int(batch.kinds[s])]
            if e - first > chunk_bytes and j > s_i:
                break
            end = max(end, e)
            j += 1
        host = flat[first:end].cpu().numpy()
        streams = order[s_i:j]

        def work(part, errs):
            for s in part:
                k = int(batch.kinds[s])
                L = int(batch.lens[s])
                off = int(batch.offs[s]) - first
                ref = o.fill(k, int(batch.keys[s]), int(batch.ctr0s[s]), L).view(np.uint8)
                got = host[off: off + ref.size]
                if got.tobytes() != ref.tobytes():
                    errs.append(f"stream {int(s)} kind {k} len {L}: {first_diff(got, ref)}")

        parts = np.array_split(streams, HOST_THREADS)
        errs_t = [[] for _ in parts]
        ts = [threading.Thread(target=work, args=(p, e)) for p, e in zip(parts, errs_t)]
        for t in ts:
            t.start()
        for t in ts:
            t.join()
        for e in errs_t:
            errors.extend(e)
        if len(errors) > 20:
            break
        s_i = j
    return errors
