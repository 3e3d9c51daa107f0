"""CPU checks of the gfx950 assembly of the fill kernels (hipcc -S with the
library's flags; no GPU involved).

k_fill_lanes writes each lane's vector with a structured-buffer store and
relies on that store ending the lane's work: on every control-flow path the
next VALU instruction, if any, comes at least two instructions later, so no
VALU write can reach the store's data registers before the store has read
them.  The test also checks that the kernel reads its lane table with an
indexed buffer load and stores with an indexed buffer store (no address
arithmetic on the VALU), and that the rounds stay one v_mad_u64_u32, one
v_mul_lo_u32 and one v_lshl_add_u32 each."""
from __future__ import annotations

import os
import re
import subprocess
import sys

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
sys.path.insert(0, ROOT)


@pytest.fixture(scope="module")
def asm(tmp_path_factory):
    from paper_2004_06278_amd import build as b

    hipcc = os.environ.get("HIPCC", "/opt/rocm/bin/hipcc")
    if not os.path.exists(hipcc):
        pytest.skip("hipcc not available")
    out = str(tmp_path_factory.mktemp("isa") / "sq_kernels.s")
    flags = [f for f in b.FLAGS if f not in ("-fPIC",)]
    cmd = [hipcc, *flags, "--cuda-device-only", "-S", os.path.join(b.CSRC, "sq_kernels.hip"), "-o", out]
    r = subprocess.run(cmd, capture_output=True, text=True)
    assert r.returncode == 0, r.stderr[-3000:]
    return open(out).read()


def kernel_bodies(text: str, pattern: str) -> dict[str, list[str]]:
    """Instruction and label lines (comments and directives dropped) of every
    kernel whose symbol matches `pattern`, from its label to its s_endpgm."""
    bodies = {}
    lines = text.splitlines()
    for i, line in enumerate(lines):
        m = re.match(r"^(_Z\S+):", line)
        if not m or not re.search(pattern, m.group(1)):
            continue
        body = []
        for l2 in lines[i + 1:]:
            s = l2.split(";")[0].strip()
            if not s or (s.startswith(".") and not s.endswith(":")):
                continue
            body.append(s)
            if s.startswith("s_endpgm"):
                break
        bodies[m.group(1)] = body
    return bodies


def first_vector_op_distance(body: list[str], start: int) -> int | None:
    """Fewest instructions (labels not counted, s_nop N counted N + 1 times)
    issued after body[start] before a VALU instruction, over every
    control-flow path (branches followed; a conditional branch also falls
    through); None when no path reaches one before s_endpgm."""
    labels = {s[:-1]: i for i, s in enumerate(body) if s.endswith(":")}
    best = None
    todo = [(start + 1, 0)]
    seen = {}
    while todo:
        i, d = todo.pop()
        while i < len(body):
            if seen.get(i, 1 << 30) <= d:
                break
            seen[i] = d
            s = body[i]
            if s.endswith(":"):
                i += 1
                continue
            if s.startswith("v_"):
                best = d if best is None else min(best, d)
                break
            if s.startswith("s_endpgm"):
                break
            if s.startswith("s_nop"):
                d += int(s.split()[-1], 0) + 1
            else:
                d += 1
            if s.startswith(("s_branch", "s_cbranch")):
                todo.append((labels[s.split()[-1]], d))
                if s.startswith("s_branch"):
                    break
            i += 1
    return best


def test_first_vector_op_distance_on_listings():
    """The path walk on small hand-written listings: a VALU right after the
    store, one reached only through a taken branch, and one behind s_nop."""
    store = "buffer_store_dwordx4 v[4:7], v0, s[8:11], 0 idxen"
    assert first_vector_op_distance([store, "v_mov_b32 v4, 0", "s_endpgm"], 0) == 0
    assert first_vector_op_distance([store, ".L1:", "s_endpgm"], 0) is None
    branchy = [store, "s_cbranch_vccnz .L2", "s_endpgm", ".L2:", "s_mov_b32 s0, 0", "v_mov_b32 v4, 0", "s_endpgm"]
    assert first_vector_op_distance(branchy, 0) == 2
    assert first_vector_op_distance([store, "s_nop 3", "v_add_u32 v5, v5, v5", "s_endpgm"], 0) == 4
    loop = [".L0:", store, "s_cbranch_scc1 .L0", "s_endpgm"]
    assert first_vector_op_distance(loop, 1) is None


def test_lane_table_fill_stores_last(asm):
    bodies = kernel_bodies(asm, r"k_fill_lanes")
    assert len(bodies) == 12, sorted(bodies)  # six kinds, unit and other increments
    for name, body in bodies.items():
        stores = [i for i, s in enumerate(body) if s.startswith("buffer_store_dwordx4")]
        assert stores, name
        assert all(" idxen" in body[i] for i in stores), name
        assert not any(s.startswith(("global_store_dwordx4", "flat_store_dwordx4")) for s in body), name
        loads = [s for s in body if s.startswith("buffer_load_dwordx2")]
        assert loads and all(" idxen" in s for s in loads), name
        for i in stores:
            d = first_vector_op_distance(body, i)
            assert d is None or d >= 2, f"{name}: VALU {d} instruction(s) after the store at {i}"


def test_rounds_are_three_instructions(asm):
    """Every squares32 round is one v_mad_u64_u32, one v_mul_lo_u32 and one
    v_lshl_add_u32: the kernel evaluates squares32 nine times (the vector's
    four outputs on the full-chunk and on the partial-chunk path, one head or
    tail element), 36 rounds, plus a few multiplies for that element's Weyl
    product ctr * key."""
    bodies = kernel_bodies(asm, r"k_fill_lanesILi0ELb0E")
    assert len(bodies) == 1
    (ins,) = bodies.values()
    mad = sum(s.startswith("v_mad_u64_u32") for s in ins)
    mul = sum(s.startswith("v_mul_lo_u32") for s in ins)
    lsh = sum(s.startswith("v_lshl_add_u32") for s in ins)
    assert lsh == 36 and 36 <= mad <= 40 and 36 <= mul <= 40, (mad, mul, lsh)
