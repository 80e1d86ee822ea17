"""Device runtime of a batch of independent problems.

`BatchRun` holds everything one batch keeps resident in HBM: the batch
handle and its workspace, the face and vertex velocities, the fractions, and
a per-step table of every problem's time step and activity (a problem drops
out after its own last step).  One `step()` copies that step's row of the
table into the arrays the captured step reads and replays the HIP graph: one
graph launch per step for all problems.  All work is enqueued on the batch's
own stream.
"""
from __future__ import annotations

import numpy as np

from . import gvof, inputs


class BatchRun:
    def __init__(self, problems, device, stream, n_div: int = 10, autotune: bool = True, graph: bool = True,
                 tune_reps: int = 2, launch_config: dict | None = None, parts=None):
        import torch
        self.torch = torch
        self.stream = stream
        self.problems = problems
        self.nprob = len(problems)
        self.nsteps = np.array([p["nsteps"] for p in problems], np.int64)
        self.max_steps = int(self.nsteps.max())
        with torch.cuda.stream(stream):
            self.B = gvof.GvofBatch([p["mesh"] for p in problems], device, stream=stream, parts=parts)
            self.nf_q = np.diff(self.B.face_off).astype(np.int64)
            self.nc_q = np.diff(self.B.cell_off).astype(np.int64)
            self.uf = torch.from_numpy(inputs.concat_soa([p["uf"] for p in problems])).to(device)
            self.uv = torch.from_numpy(inputs.concat_soa([p["uv"] for p in problems])).to(device)
            dt = np.zeros((self.max_steps, self.nprob))
            act = np.zeros((self.max_steps, self.nprob), np.uint8)
            for q, p in enumerate(problems):
                dt[: p["nsteps"], q] = p["dt_eff"]
                act[: p["nsteps"], q] = 1
            self.act_host = act
            self.dt_tab = torch.from_numpy(dt).to(device)
            self.act_tab = torch.from_numpy(act).to(device)
            self.dt = self.dt_tab[0].clone()
            self.act = self.act_tab[0].clone()
            self.F = self.B.init_fraction_each([p["shape"] for p in problems], n_div)
            self.tuned = None
            if launch_config is not None:
                gvof.gvof_set_launch_config(self.B.h, gvof.gvof_launch_config(**launch_config))
            elif autotune:
                cfg, ms = self.B.autotune(self.uf, self.uv, self.dt, self.act, self.F, reps=tune_reps)
                self.tuned = (cfg.as_dict(), ms)
            self.graph = graph
            if graph:
                self.B.capture(self.uf, self.uv, self.dt, self.act, self.F)
        self.s = 0

    @property
    def done(self) -> bool:
        return self.s >= self.max_steps

    def step(self):
        """Enqueue step s of every problem that still has steps left."""
        s = self.s
        with self.torch.cuda.stream(self.stream):
            self.dt.copy_(self.dt_tab[s])
            self.act.copy_(self.act_tab[s])
            if self.graph:
                self.B.replay()
            else:
                self.B.step(self.uf, self.uv, self.dt, self.act, self.F)
        self.s = s + 1

    def finishing_at(self, s: int):
        """Problems whose last step is step s."""
        return np.nonzero(self.nsteps == s + 1)[0]

    def face_steps(self, s0: int, s1: int) -> int:
        """Faces x steps advanced by steps s0 .. s1-1 (active problems only)."""
        return int((self.act_host[s0:s1].astype(np.int64) @ self.nf_q).sum())

    def fractions(self, q: int):
        """Device view of problem q's fractions."""
        return self.F[self.B.cells(q)]

    def status(self):
        return self.B.status()

    def close(self):
        self.B.close()
