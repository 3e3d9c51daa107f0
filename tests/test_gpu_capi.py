"""The library used from plain C: tests/capi_consumer.c calls the C ABI of
libsquares.so through include/squares.h (device memory from the HIP C API)
and compares fills, uniforms, an exact sum and a ragged batch with the C
oracle compiled into the same program."""
from __future__ import annotations

import os
import subprocess

import pytest

from gpu_helpers import log

pytestmark = pytest.mark.gpu

BIN = os.path.join(os.path.dirname(os.path.abspath(__file__)), "capi_consumer")


def test_c_program_through_the_c_abi():
    assert os.path.exists(BIN), f"{BIN} is missing: run __graft_entry__.build() first"
    log("capi consumer")
    r = subprocess.run([BIN], capture_output=True, text=True, timeout=120)
    assert r.returncode == 0, r.stdout + r.stderr
    assert "match the oracle" in r.stdout
