"""Build the oracle libraries (test infrastructure only).

liboracle.so        FP64 oracle, OpenMP
liboracle_count.so  the same source with the FLOP-counting scalar type
"""
from __future__ import annotations

import os
import subprocess
import sys

HERE = os.path.dirname(os.path.abspath(__file__))
SRC = os.path.join(HERE, "gvof_oracle.cpp")


def build(verbose: bool = False) -> None:
    common = ["g++", "-O2", "-std=c++17", "-ffp-contract=off", "-fno-fast-math", "-fPIC", "-shared", "-Wall",
              "-Wno-unknown-pragmas"]
    jobs = [
        common + ["-fopenmp", "-o", os.path.join(HERE, "liboracle.so"), SRC],
        common + ["-DORC_COUNT_FLOPS", "-o", os.path.join(HERE, "liboracle_count.so"), SRC],
    ]
    for cmd in jobs:
        if verbose:
            print(" ".join(cmd), flush=True)
        r = subprocess.run(cmd, capture_output=True, text=True)
        if r.returncode != 0:
            sys.stderr.write(r.stdout + r.stderr)
            raise RuntimeError("oracle build failed")


if __name__ == "__main__":
    build(verbose=True)
