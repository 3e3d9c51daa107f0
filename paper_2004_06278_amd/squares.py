"""Python binding of libsquares.so (ctypes).

Argument marshalling only: every call below forwards to the C ABI declared in
include/squares.h, whose entry points launch the HIP kernels.  PyTorch is
used for device memory (tensors passed by data_ptr) and streams (the current
torch stream's HIP handle).  There is no CPU fallback: if the library is not
built, or no GPU is present, calls raise.
"""
from __future__ import annotations

import ctypes
import os
import threading
from dataclasses import dataclass

HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(HERE, "libsquares.so")
TUNE_TABLE = os.path.join(HERE, "tune_gfx950.json")

U32, F32, U64, F64, U32X2, F32X2 = 0, 1, 2, 3, 4, 5
KIND_BYTES = {U32: 4, F32: 4, U64: 8, F64: 8, U32X2: 4, F32X2: 4}
OP_FILL, OP_REDUCE, OP_BATCH = 0, 1, 2
SERVE_DISCARD = 1
SERVE_NO_STATS = 2

STATUS = {0: "SQ_OK", -1: "SQ_EINVAL", -2: "SQ_EALIGN", -3: "SQ_ENOMEM", -4: "SQ_EHIP", -5: "SQ_EBUSY",
          -6: "SQ_ENOTFOUND"}


class SquaresError(RuntimeError):
    def __init__(self, status: int, msg: str):
        super().__init__(f"{STATUS.get(status, status)}: {msg}")
        self.status = status


class LaunchCfg(ctypes.Structure):
    _fields_ = [("block", ctypes.c_uint32), ("unroll", ctypes.c_uint32), ("grid_per_cu", ctypes.c_uint32),
                ("xcd_map", ctypes.c_uint32), ("tile_log2", ctypes.c_uint32)]

    def as_dict(self):
        return {f: getattr(self, f) for f, _ in self._fields_}


class SumResult(ctypes.Structure):
    _fields_ = [("lo", ctypes.c_uint64), ("hi", ctypes.c_uint64), ("value", ctypes.c_double),
                ("n", ctypes.c_uint64)]


class ServerCfg(ctypes.Structure):
    _fields_ = [("hbm_budget_bytes", ctypes.c_uint64), ("max_slots", ctypes.c_uint32),
                ("chunk_cap", ctypes.c_uint64), ("n_streams", ctypes.c_uint32), ("tile_log2", ctypes.c_uint32),
                ("tick_bytes", ctypes.c_uint64)]


class ServerStats(ctypes.Structure):
    _fields_ = [("submitted", ctypes.c_uint64), ("admitted", ctypes.c_uint64), ("completed", ctypes.c_uint64),
                ("released", ctypes.c_uint64), ("outputs", ctypes.c_uint64), ("bytes", ctypes.c_uint64),
                ("ticks", ctypes.c_uint64), ("queued_now", ctypes.c_uint64), ("active_now", ctypes.c_uint64),
                ("arena_used_bytes", ctypes.c_uint64), ("p50_s", ctypes.c_double), ("p90_s", ctypes.c_double),
                ("p99_s", ctypes.c_double), ("max_s", ctypes.c_double), ("mean_s", ctypes.c_double),
                ("first_submit_s", ctypes.c_double), ("last_complete_s", ctypes.c_double)]

    def as_dict(self):
        return {f: getattr(self, f) for f, _ in self._fields_}


# Every exported symbol with its ctypes signature (restype, argtypes).
_u64, _u32, _u8p, _vp, _int = ctypes.c_uint64, ctypes.c_uint32, ctypes.c_void_p, ctypes.c_void_p, ctypes.c_int
SIGNATURES = {
    "sq_last_error": (ctypes.c_char_p, []),
    "sq_version": (_int, []),
    "sq_init": (_int, []),
    "sq32_fill": (_int, [_u64, _u64, _u64, _vp, _vp]),
    "sq64_fill": (_int, [_u64, _u64, _u64, _vp, _vp]),
    "sq_uniform_f32": (_int, [_u64, _u64, _u64, _vp, _vp]),
    "sq_uniform_f64": (_int, [_u64, _u64, _u64, _vp, _vp]),
    "sq64x2_fill": (_int, [_u64, _u64, _u64, _vp, _vp]),
    "sq_uniform_f32x2": (_int, [_u64, _u64, _u64, _vp, _vp]),
    "sq_fill": (_int, [_int, _u64, _u64, _u64, _vp, _vp]),
    "sq_fill_cfg": (_int, [_int, _u64, _u64, _u64, _vp, ctypes.POINTER(LaunchCfg), _vp]),
    "sq_tune_get": (_int, [_int, _int, _u64, ctypes.POINTER(LaunchCfg)]),
    "sq_tune_set": (_int, [_int, _int, _u64, ctypes.POINTER(LaunchCfg)]),
    "sq_tune_load": (_int, [ctypes.c_char_p]),
    "sq_tune_save": (_int, [ctypes.c_char_p]),
    "sq_autotune": (_int, [_u32, _u64, ctypes.c_char_p]),
    "sq_reduce_workspace_bytes": (ctypes.c_size_t, [_u64]),
    "sq_reduce": (_int, [_int, _u64, _u64, _u64, _vp, _vp, ctypes.c_size_t, _vp]),
    "sq_reduce_cfg": (_int, [_int, _u64, _u64, _u64, _vp, _vp, ctypes.c_size_t, ctypes.POINTER(LaunchCfg), _vp]),
    "sq_reduce_noalloc": (_int, [_int, _u64, _u64, _u64, _vp, _vp]),
    "sq_reduce_pair": (_int, [_int, _u64, _u64, _u64, _vp, _vp, _vp, ctypes.c_size_t, _vp]),
    "sq_reduce_pair_cfg": (_int, [_int, _u64, _u64, _u64, _vp, _vp, _vp, ctypes.c_size_t,
                                  ctypes.POINTER(LaunchCfg), _vp]),
    "sq32_at": (_int, [_u64, _u64, ctypes.POINTER(_u32)]),
    "sq64_at": (_int, [_u64, _u64, ctypes.POINTER(_u64)]),
    "sq_u128_to_double_scaled": (ctypes.c_double, [_u64, _u64, _int]),
    "sq_fill_strided": (_int, [_int, _u64, _u64, _u64, _u64, _vp, _vp]),
    "sq_fill_strided_cfg": (_int, [_int, _u64, _u64, _u64, _u64, _vp, ctypes.POINTER(LaunchCfg), _vp]),
    "sq_reduce_strided": (_int, [_int, _u64, _u64, _u64, _u64, _vp, _vp, ctypes.c_size_t, _vp]),
    "sq_reduce_strided_cfg": (_int, [_int, _u64, _u64, _u64, _u64, _vp, _vp, ctypes.c_size_t,
                                     ctypes.POINTER(LaunchCfg), _vp]),
    "sq_fill_keys": (_int, [_int, _u64, _vp, _u64, _vp, _vp]),
    "sq_fill_keys_cfg": (_int, [_int, _u64, _vp, _u64, _vp, ctypes.POINTER(LaunchCfg), _vp]),
    "sq_make_keys": (_int, [_u64, _u64, _u64, _vp, _vp]),
    "sq_batch_workspace_bytes": (ctypes.c_size_t, [_u32, _u64]),
    "sq_fill_batch": (_int, [_vp, _vp, _vp, _vp, _vp, _u32, _vp, _u64, _vp, ctypes.c_size_t, _vp]),
    "sq_fill_batch_cfg": (_int, [_vp, _vp, _vp, _vp, _vp, _u32, _vp, _u64, _vp, ctypes.c_size_t,
                                 ctypes.POINTER(LaunchCfg), _vp]),
    "sq_fill_streams": (_int, [_vp, _vp, _vp, _vp, _vp, _u32, _vp, _u64, _vp]),
    "sq_batch_errors": (_int, [_vp, _vp, ctypes.POINTER(_u32)]),
    "sq_batch_plan_create": (_int, [_vp, _vp, _vp, _vp, _vp, _u32, _vp, _u64, _vp, ctypes.c_size_t,
                                    ctypes.POINTER(LaunchCfg), ctypes.POINTER(_vp)]),
    "sq_batch_plan_launch": (_int, [_vp, _vp]),
    "sq_batch_plan_destroy": (_int, [_vp]),
    "sq_server_create": (_int, [ctypes.POINTER(ServerCfg), ctypes.POINTER(_vp)]),
    "sq_server_submit": (_int, [_vp, _int, _u64, _u64, _u64, _u32, ctypes.POINTER(_u64)]),
    "sq_server_poll": (_int, [_vp, _u64, ctypes.POINTER(_int)]),
    "sq_server_wait": (_int, [_vp, _u64]),
    "sq_server_result": (_int, [_vp, _u64, ctypes.POINTER(_vp), ctypes.POINTER(_u64)]),
    "sq_server_latency": (_int, [_vp, _u64, ctypes.POINTER(ctypes.c_double)]),
    "sq_server_release": (_int, [_vp, _u64]),
    "sq_server_cancel": (_int, [_vp, _u64]),
    "sq_server_stats": (_int, [_vp, ctypes.POINTER(ServerStats)]),
    "sq_server_destroy": (_int, [_vp]),
}

_lib = None
_lock = threading.Lock()


def lib() -> ctypes.CDLL:
    """The loaded library.  Raises if it has not been built."""
    global _lib
    with _lock:
        if _lib is None:
            if not os.path.exists(LIB_PATH):
                raise RuntimeError(f"{LIB_PATH} is missing: build it first (__graft_entry__.build())")
            L = ctypes.CDLL(LIB_PATH)
            missing = [name for name in SIGNATURES if getattr(L, name, None) is None]
            if missing:
                raise RuntimeError(f"{LIB_PATH} does not export {', '.join(missing)}: rebuild it "
                                   "(__graft_entry__.build())")
            for name, (res, args) in SIGNATURES.items():
                fn = getattr(L, name)
                fn.restype = res
                fn.argtypes = args
            if os.path.exists(TUNE_TABLE) and not os.environ.get("SQ_TUNE_CACHE"):
                L.sq_tune_load(TUNE_TABLE.encode())
            _lib = L
    return _lib


def check(rc: int) -> None:
    if rc != 0:
        raise SquaresError(rc, lib().sq_last_error().decode(errors="replace"))


def _torch():
    import torch

    return torch


def _stream(stream=None) -> int:
    torch = _torch()
    s = torch.cuda.current_stream() if stream is None else stream
    return int(s.cuda_stream)


def _ptr(t) -> int:
    """Device address of a CUDA tensor (contiguous), or an int address as-is."""
    if isinstance(t, int):
        return t
    if not t.is_cuda:
        raise ValueError("tensor must live on the GPU")
    if not t.is_contiguous():
        raise ValueError("tensor must be contiguous")
    return int(t.data_ptr())


_DTYPES = None


def _out(out, nbytes: int, dtype):
    """`out` if it is a contiguous CUDA tensor of at least nbytes bytes (the
    library writes through a raw pointer and cannot check), else a new one."""
    torch = _torch()
    if out is None:
        esize = torch.empty(0, dtype=dtype).element_size()
        return torch.empty((nbytes + esize - 1) // esize, dtype=dtype, device="cuda")
    have = out.numel() * out.element_size()
    if have < nbytes:
        raise ValueError(f"output tensor holds {have} bytes, the call writes {nbytes}")
    return out


def kind_dtype(kind: int):
    torch = _torch()
    return {U32: torch.uint32, F32: torch.float32, U64: torch.uint64, F64: torch.float64, U32X2: torch.uint32,
            F32X2: torch.float32}[kind]


def cfg(block=1024, unroll=8, grid_per_cu=16, xcd_map=0, tile_log2=16) -> LaunchCfg:
    return LaunchCfg(block, unroll, grid_per_cu, xcd_map, tile_log2)


# ---------------------------------------------------------------- fills
def fill(kind: int, key: int, ctr0: int, n: int, out=None, stream=None, launch_cfg: LaunchCfg | None = None):
    """out[i] = kind's output at counter ctr0+i under key; returns `out` (a new
    CUDA tensor when not given)."""
    out = _out(out, n * KIND_BYTES.get(kind, 4), kind_dtype(kind) if kind in KIND_BYTES else _torch().uint8)
    key &= (1 << 64) - 1
    ctr0 &= (1 << 64) - 1
    if launch_cfg is None:
        check(lib().sq_fill(kind, key, ctr0, n, _ptr(out), _stream(stream)))
    else:
        check(lib().sq_fill_cfg(kind, key, ctr0, n, _ptr(out), ctypes.byref(launch_cfg), _stream(stream)))
    return out


def fill_ptr(kind: int, key: int, ctr0: int, n: int, addr: int, stream=None) -> None:
    """Fill at a raw device address (tests of alignment handling)."""
    check(lib().sq_fill(kind, key & (2**64 - 1), ctr0 & (2**64 - 1), n, addr, _stream(stream)))


def sq32_fill(key, ctr0, n, out=None, stream=None):
    out = _out(out, 4 * n, _torch().uint32)
    check(lib().sq32_fill(key & (2**64 - 1), ctr0 & (2**64 - 1), n, _ptr(out), _stream(stream)))
    return out


def sq64_fill(key, ctr0, n, out=None, stream=None):
    out = _out(out, 8 * n, _torch().uint64)
    check(lib().sq64_fill(key & (2**64 - 1), ctr0 & (2**64 - 1), n, _ptr(out), _stream(stream)))
    return out


def uniform_f32(key, ctr0, n, out=None, stream=None):
    out = _out(out, 4 * n, _torch().float32)
    check(lib().sq_uniform_f32(key & (2**64 - 1), ctr0 & (2**64 - 1), n, _ptr(out), _stream(stream)))
    return out


def sq64x2_fill(key, ctr0, n, out=None, stream=None):
    out = _out(out, 4 * n, _torch().uint32)
    check(lib().sq64x2_fill(key & (2**64 - 1), ctr0 & (2**64 - 1), n, _ptr(out), _stream(stream)))
    return out


def uniform_f32x2(key, ctr0, n, out=None, stream=None):
    out = _out(out, 4 * n, _torch().float32)
    check(lib().sq_uniform_f32x2(key & (2**64 - 1), ctr0 & (2**64 - 1), n, _ptr(out), _stream(stream)))
    return out


def uniform_f64(key, ctr0, n, out=None, stream=None):
    out = _out(out, 8 * n, _torch().float64)
    check(lib().sq_uniform_f64(key & (2**64 - 1), ctr0 & (2**64 - 1), n, _ptr(out), _stream(stream)))
    return out


M64 = (1 << 64) - 1


def sq32_at(ctr: int, key: int) -> int:
    """squares32(ctr, key) in the paper's argument order, evaluated on the GPU."""
    v = ctypes.c_uint32()
    check(lib().sq32_at(ctr & M64, key & M64, ctypes.byref(v)))
    return int(v.value)


def sq64_at(ctr: int, key: int) -> int:
    """squares64(ctr, key) in the paper's argument order, evaluated on the GPU."""
    v = ctypes.c_uint64()
    check(lib().sq64_at(ctr & M64, key & M64, ctypes.byref(v)))
    return int(v.value)


def u128_to_double_scaled(total: int, pow2_exp: int) -> float:
    """Nearest double (ties to even) of total * 2^pow2_exp, total < 2^128."""
    return float(lib().sq_u128_to_double_scaled(total & M64, (total >> 64) & M64, pow2_exp))


def fill_strided(kind: int, key: int, ctr0: int, step: int, n: int, out=None, stream=None,
                 launch_cfg: LaunchCfg | None = None):
    """out[i] = kind's output at counter ctr0 + i*step (split kinds: word i%2 at
    ctr0 + (i//2)*step)."""
    out = _out(out, n * KIND_BYTES.get(kind, 4), kind_dtype(kind) if kind in KIND_BYTES else _torch().uint8)
    args = (kind, key & M64, ctr0 & M64, step & M64, n, _ptr(out))
    if launch_cfg is None:
        check(lib().sq_fill_strided(*args, _stream(stream)))
    else:
        check(lib().sq_fill_strided_cfg(*args, ctypes.byref(launch_cfg), _stream(stream)))
    return out


def fill_keys(kind: int, ctr: int, keys, out=None, stream=None, launch_cfg: LaunchCfg | None = None, m=None):
    """Key-counter mode: out[j] = kind's output at counter ctr under keys[j]
    (keys: a CUDA uint64/int64 tensor, or a device address with m given)."""
    if m is None:
        m = keys.numel()
    elif not isinstance(keys, int) and keys.numel() * keys.element_size() < 8 * m:
        raise ValueError(f"keys tensor holds fewer than {m} keys")
    out = _out(out, m * KIND_BYTES.get(kind, 4), kind_dtype(kind) if kind in KIND_BYTES else _torch().uint8)
    args = (kind, ctr & M64, _ptr(keys), m, _ptr(out))
    if launch_cfg is None:
        check(lib().sq_fill_keys(*args, _stream(stream)))
    else:
        check(lib().sq_fill_keys_cfg(*args, ctypes.byref(launch_cfg), _stream(stream)))
    return out


def make_keys(gen_key: int, ctr0: int, m: int, out=None, stream=None):
    """m distinct-digit keys generated on the device (key j from squares64 at
    counters ctr0 + 2j and ctr0 + 2j + 1 under gen_key)."""
    out = _out(out, 8 * m, _torch().uint64)
    check(lib().sq_make_keys(gen_key & M64, ctr0 & M64, m, _ptr(out), _stream(stream)))
    return out


# ---------------------------------------------------------------- reduce
def reduce_workspace(n: int = 0):
    torch = _torch()
    return torch.empty(int(lib().sq_reduce_workspace_bytes(n)), dtype=torch.uint8, device="cuda")


def reduce_async(kind: int, key: int, ctr0: int, n: int, result, ws, stream=None,
                 launch_cfg: LaunchCfg | None = None) -> None:
    """Launches the fused exact sum; `result` is a 32-byte CUDA tensor."""
    _out(result, 32, _torch().uint8)
    args = (kind, key & (2**64 - 1), ctr0 & (2**64 - 1), n, _ptr(result), _ptr(ws), ws.numel() * ws.element_size())
    if launch_cfg is None:
        check(lib().sq_reduce(*args, _stream(stream)))
    else:
        check(lib().sq_reduce_cfg(*args, ctypes.byref(launch_cfg), _stream(stream)))


def reduce_noalloc_async(kind: int, key: int, ctr0: int, n: int, result, stream=None) -> None:
    """The fused exact sum on the library's own device scratch (no workspace
    argument, no allocation in the call); `result` is a 32-byte CUDA tensor."""
    _out(result, 32, _torch().uint8)
    check(lib().sq_reduce_noalloc(kind, key & M64, ctr0 & M64, n, _ptr(result), _stream(stream)))


def reduce_strided_async(kind: int, key: int, ctr0: int, step: int, n: int, result, ws, stream=None,
                         launch_cfg: LaunchCfg | None = None) -> None:
    _out(result, 32, _torch().uint8)
    args = (kind, key & M64, ctr0 & M64, step & M64, n, _ptr(result), _ptr(ws), ws.numel() * ws.element_size())
    if launch_cfg is None:
        check(lib().sq_reduce_strided(*args, _stream(stream)))
    else:
        check(lib().sq_reduce_strided_cfg(*args, ctypes.byref(launch_cfg), _stream(stream)))


def reduce_strided(kind: int, key: int, ctr0: int, step: int, n: int, launch_cfg: LaunchCfg | None = None):
    res = result_tensor()
    ws = reduce_workspace(n)
    reduce_strided_async(kind, key, ctr0, step, n, res, ws, launch_cfg=launch_cfg)
    return read_result(res)


def result_tensor():
    torch = _torch()
    return torch.zeros(32, dtype=torch.uint8, device="cuda")


def read_result(result) -> tuple[int, float, int]:
    """(exact integer sum, rounded value, n) from a result tensor (synchronises)."""
    raw = bytes(result.cpu().numpy().tobytes())
    r = SumResult.from_buffer_copy(raw)
    return int(r.lo) | (int(r.hi) << 64), float(r.value), int(r.n)


def reduce(kind: int, key: int, ctr0: int, n: int, launch_cfg: LaunchCfg | None = None):
    res = result_tensor()
    ws = reduce_workspace(n)
    reduce_async(kind, key, ctr0, n, res, ws, launch_cfg=launch_cfg)
    return read_result(res)


def reduce_pair_async(kind32: int, key: int, ctr0: int, n: int, result32, result64, ws, stream=None,
                      launch_cfg: LaunchCfg | None = None) -> None:
    """Launches the paired sum (kind32 U32 with U64, or F32 with F64) into two
    32-byte CUDA result tensors."""
    _out(result32, 32, _torch().uint8)
    _out(result64, 32, _torch().uint8)
    args = (kind32, key & M64, ctr0 & M64, n, _ptr(result32), _ptr(result64), _ptr(ws), ws.numel() * ws.element_size())
    if launch_cfg is None:
        check(lib().sq_reduce_pair(*args, _stream(stream)))
    else:
        check(lib().sq_reduce_pair_cfg(*args, ctypes.byref(launch_cfg), _stream(stream)))


def reduce_pair(kind32: int, key: int, ctr0: int, n: int, launch_cfg: LaunchCfg | None = None):
    """((sum32, value32, n), (sum64, value64, n)) of the paired sum."""
    r32, r64 = result_tensor(), result_tensor()
    ws = reduce_workspace(n)
    reduce_pair_async(kind32, key, ctr0, n, r32, r64, ws, launch_cfg=launch_cfg)
    return read_result(r32), read_result(r64)


# ---------------------------------------------------------------- batch
@dataclass
class DeviceBatch:
    keys: object
    ctr0s: object
    lens: object
    offs: object
    kinds: object
    m: int
    out: object
    out_bytes: int
    ws: object


def batch_to_device(keys, ctr0s, lens, offs, kinds, out_bytes: int, out=None) -> DeviceBatch:
    """Copies host descriptor arrays (numpy) to the GPU and allocates the arena
    and workspace."""
    import numpy as np

    torch = _torch()

    def u64(a):
        return torch.from_numpy(np.ascontiguousarray(a, dtype=np.uint64).view(np.int64)).cuda()

    m = len(keys)
    kd = torch.from_numpy(np.ascontiguousarray(kinds, dtype=np.uint8)).cuda()
    if out is None:
        out = torch.zeros(max(out_bytes, 16), dtype=torch.uint8, device="cuda")
    _out(out, out_bytes, torch.uint8)
    ws = torch.empty(int(lib().sq_batch_workspace_bytes(m, out_bytes)), dtype=torch.uint8, device="cuda")
    return DeviceBatch(u64(keys), u64(ctr0s), u64(lens), u64(offs), kd, m, out, out_bytes, ws)


def fill_batch(b: DeviceBatch, stream=None, launch_cfg: LaunchCfg | None = None) -> None:
    args = (_ptr(b.keys), _ptr(b.ctr0s), _ptr(b.lens), _ptr(b.offs), _ptr(b.kinds), b.m, _ptr(b.out), b.out_bytes,
            _ptr(b.ws), b.ws.numel())
    if launch_cfg is None:
        check(lib().sq_fill_batch(*args, _stream(stream)))
    else:
        check(lib().sq_fill_batch_cfg(*args, ctypes.byref(launch_cfg), _stream(stream)))


def fill_streams(keys, ctr0s, lens, offs, kinds, out, out_bytes: int, stream=None) -> None:
    """One fill launch per stream from HOST descriptor arrays (numpy)."""
    import numpy as np

    _out(out, out_bytes, _torch().uint8)
    arrs = [np.ascontiguousarray(a, dtype=np.uint64) for a in (keys, ctr0s, lens, offs)]
    kd = np.ascontiguousarray(kinds, dtype=np.uint8)
    m = kd.size
    check(lib().sq_fill_streams(*(a.ctypes.data for a in arrs), kd.ctypes.data, m, _ptr(out), out_bytes,
                                _stream(stream)))


def batch_errors(b: DeviceBatch, stream=None) -> int:
    c = ctypes.c_uint32(0)
    check(lib().sq_batch_errors(_ptr(b.ws), _stream(stream), ctypes.byref(c)))
    return int(c.value)


class BatchPlan:
    """A batch captured once into a HIP graph; launch() replays it."""

    def __init__(self, b: DeviceBatch, launch_cfg: LaunchCfg | None = None):
        self.b = b
        h = ctypes.c_void_p()
        check(lib().sq_batch_plan_create(_ptr(b.keys), _ptr(b.ctr0s), _ptr(b.lens), _ptr(b.offs), _ptr(b.kinds),
                                         b.m, _ptr(b.out), b.out_bytes, _ptr(b.ws), b.ws.numel(),
                                         ctypes.byref(launch_cfg) if launch_cfg is not None else None,
                                         ctypes.byref(h)))
        self.h = h

    def launch(self, stream=None) -> None:
        check(lib().sq_batch_plan_launch(self.h, _stream(stream)))

    def close(self) -> None:
        if self.h:
            check(lib().sq_batch_plan_destroy(self.h))
            self.h = ctypes.c_void_p()

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass


# ---------------------------------------------------------------- tuning
def tune_get(op: int, kind: int, n: int) -> LaunchCfg:
    c = LaunchCfg()
    check(lib().sq_tune_get(op, kind, n, ctypes.byref(c)))
    return c


def tune_set(op: int, kind: int, n: int, c: LaunchCfg) -> None:
    check(lib().sq_tune_set(op, kind, n, ctypes.byref(c)))


def tune_load(path: str) -> None:
    check(lib().sq_tune_load(path.encode()))


def tune_save(path: str) -> None:
    check(lib().sq_tune_save(path.encode()))


def autotune(op_mask: int = 7, max_bytes: int = 8 << 30, save_path: str | None = None) -> None:
    check(lib().sq_autotune(op_mask, max_bytes, save_path.encode() if save_path else None))


# ---------------------------------------------------------------- serving
class Server:
    """Continuous-batching request loop (see sq_server_* in squares.h)."""

    def __init__(self, hbm_budget_bytes: int, max_slots: int = 4096, chunk_cap: int = 1 << 22, n_streams: int = 4,
                 tile_log2: int = 0, tick_bytes: int = 0):
        c = ServerCfg(hbm_budget_bytes, max_slots, chunk_cap, n_streams, tile_log2, tick_bytes)
        h = ctypes.c_void_p()
        check(lib().sq_server_create(ctypes.byref(c), ctypes.byref(h)))
        self.h = h

    def submit(self, kind: int, key: int, ctr0: int, n: int, flags: int = 0) -> int:
        rid = ctypes.c_uint64(0)
        check(lib().sq_server_submit(self.h, kind, key & (2**64 - 1), ctr0 & (2**64 - 1), n, flags,
                                     ctypes.byref(rid)))
        return int(rid.value)

    def poll(self, rid: int) -> bool:
        d = ctypes.c_int(0)
        check(lib().sq_server_poll(self.h, rid, ctypes.byref(d)))
        return bool(d.value)

    def wait(self, rid: int) -> None:
        check(lib().sq_server_wait(self.h, rid))

    def result(self, rid: int) -> tuple[int, int]:
        p = ctypes.c_void_p()
        nb = ctypes.c_uint64()
        check(lib().sq_server_result(self.h, rid, ctypes.byref(p), ctypes.byref(nb)))
        return int(p.value or 0), int(nb.value)

    def result_bytes(self, rid: int):
        """Copies a completed request's output to a new uint8 CUDA tensor."""
        torch = _torch()
        p, nb = self.result(rid)
        out = torch.empty(nb, dtype=torch.uint8, device="cuda")
        import ctypes as C

        hip = _hip()
        check_hip(hip.hipMemcpy(C.c_void_p(out.data_ptr()), C.c_void_p(p), C.c_size_t(nb), 3))
        return out

    def latency(self, rid: int) -> float:
        s = ctypes.c_double()
        check(lib().sq_server_latency(self.h, rid, ctypes.byref(s)))
        return float(s.value)

    def release(self, rid: int) -> None:
        check(lib().sq_server_release(self.h, rid))

    def cancel(self, rid: int) -> None:
        check(lib().sq_server_cancel(self.h, rid))

    def stats(self) -> dict:
        s = ServerStats()
        check(lib().sq_server_stats(self.h, ctypes.byref(s)))
        return s.as_dict()

    def close(self) -> None:
        if self.h:
            check(lib().sq_server_destroy(self.h))
            self.h = ctypes.c_void_p()

    def __enter__(self):
        return self

    def __exit__(self, *a):
        self.close()


_hip_lib = None


def _hip():
    """The HIP runtime (for plain device-to-device copies of server results)."""
    global _hip_lib
    if _hip_lib is None:
        _hip_lib = ctypes.CDLL("libamdhip64.so")
        _hip_lib.hipMemcpy.restype = ctypes.c_int
        _hip_lib.hipMemcpy.argtypes = [ctypes.c_void_p, ctypes.c_void_p, ctypes.c_size_t, ctypes.c_int]
    return _hip_lib


def check_hip(rc: int) -> None:
    if rc != 0:
        raise RuntimeError(f"HIP error {rc}")
