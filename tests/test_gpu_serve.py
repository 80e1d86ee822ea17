"""The serving loop on the GPU: jobs arriving over time are admitted under an
HBM budget and join the running jobs at step boundaries, each on its own
stream, and release their memory when done; every job's result must be
bit-identical to the same job advanced alone through the single-problem
calls."""
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
    for i, (side, kind, steps, arr) in enumerate([(8, "cartesian", 60, 0.0), (6, "jittered", 4, 0.0),
                                                  (10, "cartesian", 9, 0.05), (7, "jittered", 5, 0.06),
                                                  (9, "cartesian", 3, 0.4), (6, "jittered", 7, 0.41),
                                                  (12, "cartesian", 5, 0.8)]):
        specs.append(dict(arrival=arr, side=side, kind=kind, radius=0.15 + 0.01 * i,
                          center=(0.45 + 0.02 * i, 0.5, 0.5 - 0.01 * i), period=1.5 + 0.2 * i, steps=steps,
                          jitter_seed=100 + i))
    problems = [inputs.problem_inputs(s) for s in specs]
    jobs = serve.jobs_from_specs(specs, problems)
    ex = serve.GpuExecutor(dev, n_div=6)
    sizes = []
    for p in problems:
        probe = serve.Job(id=-1, arrival=0, nsteps=p["nsteps"], faces=0, cells=0, payload=p)
        ex.estimate(probe)
        ex.reject(probe)
        sizes.append(probe.bytes)
    budget = int(2.2 * max(sizes))  # any two jobs at a time, some threes
    rep = serve.Server(ex, budget_bytes=budget, slots=3, depth=2).run(jobs)
    S = rep.summary()
    log(f"served: {S}")
    assert S["completed"] == len(jobs) and S["rejected"] == 0 and S["admitted"] == len(jobs)
    assert rep.peak_bytes <= budget and rep.max_running >= 2
    # some job started while another was still running (the two overlapped on the device)
    assert any(a.t_start < b.t_done and b.t_start < a.t_done for a in jobs for b in jobs if a is not b)
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
