"""Driver of the library's autotuner (sq_autotune).

Runs the tuner for fill, reduce and batch on the current GPU and writes the
table as JSON.  The Python binding loads `tune_gfx950.json` (next to the
library) when it first loads the library, unless $SQ_TUNE_CACHE names another
table, which the library then loads itself; a C program calls sq_tune_load.

    python -m paper_2004_06278_amd.autotune [--out PATH] [--max-gib 64]
"""
from __future__ import annotations

import argparse
import json
import os
import sys
import time


def main() -> int:
    from . import squares as sq

    p = argparse.ArgumentParser()
    p.add_argument("--out", default=sq.TUNE_TABLE)
    p.add_argument("--max-gib", type=int, default=64)
    p.add_argument("--ops", type=int, default=7, help="bit mask: 1 fill, 2 reduce, 4 batch")
    a = p.parse_args()
    import torch

    assert torch.cuda.is_available(), "the autotuner needs a GPU"
    t0 = time.time()
    sq.autotune(a.ops, a.max_gib << 30, a.out)
    with open(a.out) as f:
        rows = json.load(f)
    print(f"autotune: {len(rows)} entries in {time.time() - t0:.1f} s -> {a.out}", flush=True)
    for r in rows:
        print(json.dumps(r), flush=True)
    return 0


if __name__ == "__main__":
    sys.exit(main())
