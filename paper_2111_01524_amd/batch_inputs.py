"""Host-side generation of many problems' inputs (grids, Enright field, time
steps, bodies) on a pool of threads: the generators spend their time in numpy,
which releases the interpreter lock, and a thread pool starts no process (so
it also runs under a profiler that has already initialised the GPU)."""
from __future__ import annotations

import os
from concurrent.futures import ThreadPoolExecutor

from . import inputs


def _workers(n_items: int, workers: int | None) -> int:
    return workers or min(16, os.cpu_count() or 1, max(1, n_items))


def generate(specs, workers: int | None = None, steps=None):
    """problem_inputs(spec) for every spec, in order (steps: None, or one count per spec)."""
    steps = steps if steps is not None else [None] * len(specs)
    with ThreadPoolExecutor(_workers(len(specs), workers)) as pool:
        return list(pool.map(lambda w: inputs.problem_inputs(w[0], steps=w[1]), zip(specs, steps)))


def grids(specs, workers: int | None = None) -> dict:
    """inputs.grid_inputs of every distinct grid among the specs (grid_key -> inputs), built in parallel."""
    uniq = {}
    for s in specs:
        uniq.setdefault(inputs.grid_key(s), s)
    with ThreadPoolExecutor(_workers(len(uniq), workers)) as pool:
        return dict(zip(uniq, pool.map(inputs.grid_inputs, uniq.values())))
