"""The serving loop on the GPU: jobs arriving over time are admitted under an
HBM budget into cohorts that run concurrently on their own streams; every
job's result must be bit-identical to the same job advanced alone through the
single-problem calls."""
from __future__ import annotations

import numpy as np
import pytest

from paper_2111_01524_amd import inputs
from tests.gpu_common import host, log, to_dev, torch_dev

pytestmark = pytest.mark.gpu


def test_served_results_equal_alone():
    torch, dev = torch_dev()
    from paper_2111_01524_amd import gvof, serve
    specs = []
    for i, (side, kind, steps, arr) in enumerate([(8, "cartesian", 6, 0.0), (6, "jittered", 4, 0.0),
                                                  (10, "cartesian", 9, 0.05), (7, "jittered", 5, 0.06),
                                                  (9, "cartesian", 3, 0.4), (6, "jittered", 7, 0.41),
                                                  (12, "cartesian", 5, 0.8)]):
        specs.append(dict(arrival=arr, side=side, kind=kind, radius=0.15 + 0.01 * i,
                          center=(0.45 + 0.02 * i, 0.5, 0.5 - 0.01 * i), period=1.5 + 0.2 * i, steps=steps,
                          jitter_seed=100 + i))
    problems = [inputs.problem_inputs(s) for s in specs]
    jobs = serve.jobs_from_specs(specs, problems)
    ex = serve.GpuExecutor(dev, n_div=6)
    probe = serve.Job(id=-1, arrival=0, nsteps=1, faces=0, cells=0, payload=problems[2])
    ex.estimate(probe)
    ex.reject(probe)
    budget = int(2.5 * probe.bytes)  # about two jobs at a time
    rep = serve.Server(ex, budget_bytes=budget, max_cohorts=2, depth=2, max_jobs_per_cohort=2).run(jobs)
    S = rep.summary()
    log(f"served: {S}")
    assert S["completed"] == len(jobs) and S["rejected"] == 0
    assert rep.cohorts >= 3 and rep.peak_bytes <= budget
    for j, p in zip(jobs, problems):
        g = gvof.GvofMesh(p["mesh"], dev)
        F = g.init_fraction(p["shape"][0], p["shape"][1], 6)
        ufa, uva = to_dev(torch, dev, p["uf"]), to_dev(torch, dev, p["uv"])
        for s in range(p["nsteps"]):
            g.reconstruct(F)
            g.advect_step(ufa, uva, p["dt_eff"][s], F, F)
        Fa = host(F)
        g.status()
        assert np.array_equal(j.result.numpy(), Fa), j.id
        assert j.t_done - j.arrival > 0
