"""Binding of libgvof_probe.so (include/gvof_probe.h): chip probes that give
the benchmark a measured FP64 vector ceiling beside the published one."""
from __future__ import annotations

import ctypes as C
import os

HERE = os.path.dirname(os.path.abspath(__file__))
PROBE_LIB_PATH = os.path.join(HERE, "libgvof_probe.so")

_lib = None


def lib() -> C.CDLL:
    global _lib
    if _lib is None:
        import torch  # noqa: F401  (one HIP runtime per process: torch's)
        if not os.path.exists(PROBE_LIB_PATH):
            raise RuntimeError(f"{PROBE_LIB_PATH} is not built: run `python -m paper_2111_01524_amd.build`")
        L = C.CDLL(PROBE_LIB_PATH)
        L.gvof_probe_fp64_fma.argtypes = [C.c_void_p, C.c_int32, C.c_int32, C.c_double, C.c_double, C.c_void_p]
        L.gvof_probe_fp64_fma.restype = C.c_int
        _lib = L
    return _lib


def exported_symbols():
    """Names of every function include/gvof_probe.h declares."""
    return ["gvof_probe_fp64_fma"]


def fp64_fma(out, blocks: int, iters: int, a: float = 1.0, b: float = 1.0, stream=None) -> None:
    """Launches the FMA loop into the device tensor out (blocks * 256 doubles)
    on stream (a torch stream; its current one when None)."""
    import torch
    if out.dtype != torch.float64 or not out.is_cuda or out.numel() < blocks * 256:
        raise ValueError("out: a device float64 tensor of blocks * 256 elements")
    s = stream if stream is not None else torch.cuda.current_stream(out.device)
    rc = lib().gvof_probe_fp64_fma(C.c_void_p(out.data_ptr()), blocks, iters, a, b, C.c_void_p(s.cuda_stream))
    if rc != 0:
        raise RuntimeError(f"gvof_probe_fp64_fma failed: {rc}")


def fp64_fma_flops(blocks: int, iters: int) -> int:
    return blocks * 256 * iters * 16


def measure_fp64_fma(device, blocks: int = 16384, iters: int = 2048, repeats: int = 5) -> float:
    """Best of `repeats` timed launches, in FP64 TFLOP/s."""
    import torch
    out = torch.empty(blocks * 256, dtype=torch.float64, device=device)
    fp64_fma(out, blocks, 16)  # warm-up (first launch loads the code object)
    torch.cuda.synchronize(device)
    best = float("inf")
    for _ in range(repeats):
        e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
        e0.record()
        fp64_fma(out, blocks, iters)
        e1.record()
        torch.cuda.synchronize(device)
        best = min(best, e0.elapsed_time(e1) * 1e-3)
    return fp64_fma_flops(blocks, iters) / best / 1e12


def measure_copy(device, mib: int = 1024, repeats: int = 5) -> float:
    """Best of `repeats` timed FP64 copies of mib MiB, in GB/s of HBM traffic
    (bytes read + bytes written)."""
    import torch
    n = mib * (1 << 20) // 8
    src = torch.ones(n, dtype=torch.float64, device=device)
    dst = torch.empty_like(src)
    dst.copy_(src)
    torch.cuda.synchronize(device)
    best = float("inf")
    for _ in range(repeats):
        e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
        e0.record()
        dst.copy_(src)
        e1.record()
        torch.cuda.synchronize(device)
        best = min(best, e0.elapsed_time(e1) * 1e-3)
    return 2 * n * 8 / best / 1e9
