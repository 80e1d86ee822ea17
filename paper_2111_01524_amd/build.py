"""Build libgvof.so (HIP, gfx950) and the probe library libgvof_probe.so in-tree.

    python -m paper_2111_01524_amd.build

Flags: FP64 with no contraction unless written as fma() (-ffp-contract=off),
no fast-math, packed-FP32 instructions disabled, position independent.
"""
from __future__ import annotations

import os
import shutil
import subprocess
import sys
import tempfile

HERE = os.path.dirname(os.path.abspath(__file__))
CSRC = os.path.join(HERE, "csrc")
ROOT = os.path.dirname(HERE)
LIB = os.path.join(HERE, "libgvof.so")
SOURCES = ["gvof_kernels.hip", "gvof_api.cpp"]
PROBE_LIB = os.path.join(HERE, "libgvof_probe.so")
PROBE_SOURCES = ["gvof_probe.hip"]
ARCH = os.environ.get("GVOF_ARCH", "gfx950")


def hipcc() -> str:
    for c in (os.environ.get("HIPCC"), "/opt/rocm/bin/hipcc", shutil.which("hipcc")):
        if c and os.path.exists(c):
            return c
    raise RuntimeError("hipcc not found")


def common_flags():
    return ["-O3", "-std=c++17", f"--offload-arch={ARCH}", "-fPIC", "-ffp-contract=off", "-fno-fast-math",
            "-Xclang", "-target-feature", "-Xclang", "-packed-fp32-ops", "-I", CSRC,
            "-I", os.path.join(ROOT, "include"), "-Wall", "-Wno-unused-function"]


def build(verbose: bool = False, jobs: int = 4) -> str:
    """Builds both libraries; returns the path of libgvof.so."""
    _build_lib(LIB, SOURCES, verbose)
    _build_lib(PROBE_LIB, PROBE_SOURCES, verbose)
    return LIB


def _build_lib(lib_path: str, sources, verbose: bool) -> None:
    cc = hipcc()
    tmp = tempfile.mkdtemp(prefix="gvof_build_")
    try:
        procs = []
        objs = []
        for src in sources:
            obj = os.path.join(tmp, src + ".o")
            cmd = [cc] + common_flags() + ["-c", os.path.join(CSRC, src), "-o", obj]
            if verbose:
                print(" ".join(cmd), flush=True)
            procs.append((cmd, subprocess.Popen(cmd, stdout=subprocess.PIPE, stderr=subprocess.STDOUT, text=True)))
            objs.append(obj)
        failed = False
        for cmd, p in procs:
            out, _ = p.communicate()
            if p.returncode != 0:
                failed = True
                sys.stderr.write(out)
            elif verbose and out.strip():
                sys.stderr.write(out)
        if failed:
            raise RuntimeError("HIP build failed")
        tmp_lib = lib_path + ".tmp"
        cmd = [cc, f"--offload-arch={ARCH}", "-shared", "-fPIC", "-o", tmp_lib] + objs
        if verbose:
            print(" ".join(cmd), flush=True)
        r = subprocess.run(cmd, capture_output=True, text=True)
        if r.returncode != 0:
            sys.stderr.write(r.stdout + r.stderr)
            raise RuntimeError("HIP link failed")
        os.replace(tmp_lib, lib_path)
    finally:
        shutil.rmtree(tmp, ignore_errors=True)


if __name__ == "__main__":
    print(build(verbose=True))
