"""CPU checks of the C ABI: the library loads (no GPU needed to load it) and
exports every function that include/squares.h declares, and the binding
knows each of them.  No compute call is made."""
from __future__ import annotations

import ctypes
import os
import re

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
HEADER = os.path.join(ROOT, "include", "squares.h")


def declared_functions() -> list[str]:
    text = open(HEADER).read()
    text = re.sub(r"/\*.*?\*/", " ", text, flags=re.S)
    names = re.findall(r"\b(sq[0-9a-z_]+)\s*\(", text)
    return sorted(set(names))


def test_header_declares_the_boundary():
    names = declared_functions()
    for must in ("sq32_fill", "sq64_fill", "sq_uniform_f32", "sq_uniform_f64", "sq_reduce", "sq_fill_batch",
                 "sq_batch_plan_create", "sq_autotune", "sq_server_create", "sq_server_submit"):
        assert must in names


def test_library_exports_every_declared_symbol():
    from paper_2004_06278_amd import squares

    if not os.path.exists(squares.LIB_PATH):
        pytest.fail("libsquares.so is not built (run __graft_entry__.build())")
    lib = ctypes.CDLL(squares.LIB_PATH)
    missing = [n for n in declared_functions() if not hasattr(lib, n)]
    assert not missing, missing
    unbound = [n for n in declared_functions() if n not in squares.SIGNATURES]
    assert not unbound, unbound


def test_version_and_error_string_without_gpu():
    from paper_2004_06278_amd import squares

    L = squares.lib()
    assert L.sq_version() >= 10000
    assert isinstance(L.sq_last_error(), bytes)
    assert L.sq_reduce_workspace_bytes(1 << 32) >= 16
    assert L.sq_batch_workspace_bytes(4096, 1 << 30) >= 64 + 8 * 4097 + 4 * (1 << 16)
