"""Parallel host-side generation of many problems' inputs (grids, Enright
field, time steps, bodies) with a spawned process pool: the generators are
numpy-bound and independent per problem.  Spawned workers import only numpy
and the input generators, never the GPU runtime."""
from __future__ import annotations

import multiprocessing as mp
import os

from . import inputs


def _one(args):
    spec, steps = args
    return inputs.problem_inputs(spec, steps=steps)


def generate(specs, workers: int | None = None, steps=None):
    """problem_inputs(spec) for every spec, in order (steps: None, or one count per spec)."""
    steps = steps if steps is not None else [None] * len(specs)
    work = list(zip(specs, steps))
    n = workers or min(16, os.cpu_count() or 1, max(1, len(work)))
    if n <= 1 or len(work) <= 1:
        return [_one(w) for w in work]
    ctx = mp.get_context("spawn")
    with ctx.Pool(n) as pool:
        return pool.map(_one, work, chunksize=1)
