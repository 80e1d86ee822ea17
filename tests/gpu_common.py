"""Shared helpers for the GPU parity tests (HIP library vs CPU oracle)."""
from __future__ import annotations

import sys

import numpy as np


def log(msg):
    print(msg, flush=True)
    sys.stdout.flush()


def torch_dev():
    import torch
    if not torch.cuda.is_available():
        raise RuntimeError("GPU tests need a HIP device")
    return torch, torch.device("cuda:0")


def to_dev(torch, dev, a, dtype=None):
    a = np.ascontiguousarray(a)
    t = torch.from_numpy(a.copy())
    if dtype is not None:
        t = t.to(dtype)
    return t.to(dev)


def host(t):
    return t.detach().cpu().numpy()


def max_abs(a, b):
    a = np.asarray(a, float); b = np.asarray(b, float)
    return float(np.abs(a - b).max()) if a.size else 0.0
