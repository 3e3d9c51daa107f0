"""Builds libsquares.so (the HIP kernels and the C ABI) for gfx950 with hipcc."""
from __future__ import annotations

import os
import subprocess
import sys

HERE = os.path.dirname(os.path.abspath(__file__))
CSRC = os.path.join(HERE, "csrc")
LIB = os.path.join(HERE, "libsquares.so")
SOURCES = ["sq_kernels.hip", "sq_capi.hip", "sq_tune.hip", "sq_server.hip"]
ARCH = os.environ.get("SQ_OFFLOAD_ARCH", "gfx950")

# Packed FP32 instructions are disabled for all device code (-packed-fp32-ops);
# hipcc's host pass warns that it does not know the feature.
FLAGS = [
    "-O3", "-std=c++17", "-fPIC", f"--offload-arch={ARCH}",
    "-Xclang", "-target-feature", "-Xclang", "-packed-fp32-ops",
    "-Wall", "-Wextra", "-Wno-unused-result",
]


def build(verbose: bool = False) -> str:
    hipcc = os.environ.get("HIPCC", "/opt/rocm/bin/hipcc")
    objs = []
    for src in SOURCES:
        path = os.path.join(CSRC, src)
        if not os.path.exists(path):
            continue
        obj = os.path.join(CSRC, "_build", src + ".o")
        os.makedirs(os.path.dirname(obj), exist_ok=True)
        cmd = [hipcc, *FLAGS, "-c", path, "-o", obj]
        if verbose:
            print(" ".join(cmd), flush=True)
        r = subprocess.run(cmd, capture_output=True, text=True)
        if r.returncode != 0:
            sys.stderr.write(r.stdout + r.stderr)
            raise RuntimeError(f"hipcc failed on {src}")
        objs.append(obj)
    tmp = LIB + ".tmp"
    cmd = [hipcc, f"--offload-arch={ARCH}", "-shared", "-fPIC", *objs, "-o", tmp, "-lpthread"]
    if verbose:
        print(" ".join(cmd), flush=True)
    r = subprocess.run(cmd, capture_output=True, text=True)
    if r.returncode != 0:
        sys.stderr.write(r.stdout + r.stderr)
        raise RuntimeError("hipcc link failed")
    os.replace(tmp, LIB)
    write_build_info()
    return LIB


BUILD_INFO = os.path.join(HERE, "build_info.json")


def write_build_info() -> None:
    """Records next to the library the git revision it was built from (and
    whether the tree had changes), for run records made where no git
    checkout is present."""
    import json

    rev, dirty = None, None
    try:
        rev = subprocess.run(["git", "-C", HERE, "rev-parse", "--short=12", "HEAD"], capture_output=True, text=True,
                             timeout=10).stdout.strip() or None
        if rev:
            dirty = bool(subprocess.run(["git", "-C", HERE, "status", "--porcelain", "--untracked-files=no"],
                                        capture_output=True, text=True, timeout=10).stdout.strip())
    except (OSError, subprocess.SubprocessError):
        pass
    with open(BUILD_INFO, "w") as f:
        json.dump({"git_rev": rev, "tree_had_changes": dirty}, f)


def build_calib(verbose: bool = False) -> str:
    """Builds the calibration program (VALU issue rates, HBM store ceiling)."""
    hipcc = os.environ.get("HIPCC", "/opt/rocm/bin/hipcc")
    src = os.path.join(HERE, "calib", "sq_calib.hip")
    exe = os.path.join(HERE, "calib", "sq_calib")
    cmd = [hipcc, *FLAGS, src, "-o", exe]
    if verbose:
        print(" ".join(cmd), flush=True)
    r = subprocess.run(cmd, capture_output=True, text=True)
    if r.returncode != 0:
        sys.stderr.write(r.stdout + r.stderr)
        raise RuntimeError("hipcc failed on sq_calib.hip")
    return exe


MEASURE_LIB = os.path.join(HERE, "calib", "libsqmeasure.so")


def build_measure(verbose: bool = False) -> str:
    """Builds libsqmeasure.so: the benchmark's store-only ceiling kernel and
    clock sampler (measurement code, not part of libsquares.so)."""
    hipcc = os.environ.get("HIPCC", "/opt/rocm/bin/hipcc")
    src = os.path.join(HERE, "calib", "sq_measure.hip")
    tmp = MEASURE_LIB + ".tmp"
    cmd = [hipcc, *FLAGS, "-shared", src, "-o", tmp]
    if verbose:
        print(" ".join(cmd), flush=True)
    r = subprocess.run(cmd, capture_output=True, text=True)
    if r.returncode != 0:
        sys.stderr.write(r.stdout + r.stderr)
        raise RuntimeError("hipcc failed on sq_measure.hip")
    os.replace(tmp, MEASURE_LIB)
    return MEASURE_LIB


if __name__ == "__main__":
    print(build(verbose=True))
    print(build_calib(verbose=True))
    print(build_measure(verbose=True))
