"""Serving loop: advection jobs arriving over time, admitted under an HBM
budget, advanced with continuous batching.

The scheduler is written against a small executor interface so that its
logic (arrival order, admission by budget, concurrent cohorts, completion and
latency accounting) runs unchanged on the GPU executor and on a fake one with
a virtual clock (the CPU tests).

Policy.  Every arriving job is sized first (its mesh topology and workspace
size, on a host worker, while the device keeps running).  Sized jobs queue in
arrival order; a job never overtakes an earlier arrival.  Whenever fewer than
`max_cohorts` cohorts are starting or running, the jobs at the head of the
queue that fit the remaining budget (at most `max_jobs_per_cohort` of them)
are admitted together as one cohort: one batch handle, set up on a host worker
and then resident until every job in it is done.  A job whose own footprint
exceeds the whole budget is rejected.  Every running cohort keeps up to
`depth` steps in flight on its own stream, so cohorts overlap on the device
and new cohorts join while others run.  A job's result is ready when the copy
of its fractions after its own last step has completed; latency = ready time
- arrival time.
"""
from __future__ import annotations

import time
from collections import deque
from concurrent.futures import ThreadPoolExecutor
from dataclasses import dataclass, field

import numpy as np


@dataclass
class Job:
    id: int
    arrival: float
    nsteps: int
    faces: int
    cells: int
    payload: object = None        # executor-specific inputs
    bytes: int = 0                # device footprint estimate, set by the executor
    t_admit: float | None = None
    t_done: float | None = None
    rejected: bool = False
    result: object = None
    part: object = None           # executor state held between estimate and start


@dataclass
class Report:
    jobs: list = field(default_factory=list)
    makespan: float = 0.0
    peak_bytes: int = 0
    cohorts: int = 0

    def summary(self, arrival_window: float | None = None) -> dict:
        done = [j for j in self.jobs if j.t_done is not None]
        lat = np.array([j.t_done - j.arrival for j in done]) if done else np.zeros(0)
        wait = np.array([j.t_admit - j.arrival for j in done]) if done else np.zeros(0)
        fs = sum(j.faces * j.nsteps for j in done)
        win = arrival_window if arrival_window is not None else (max(j.arrival for j in self.jobs) if self.jobs else 0)
        out = {
            "jobs": len(self.jobs), "completed": len(done), "rejected": sum(j.rejected for j in self.jobs),
            "cohorts": self.cohorts, "makespan_s": self.makespan, "peak_hbm_bytes": self.peak_bytes,
            "face_steps": fs, "value": fs / self.makespan if self.makespan > 0 else 0.0,
            "p50_latency_s": float(np.percentile(lat, 50)) if lat.size else None,
            "p99_latency_s": float(np.percentile(lat, 99)) if lat.size else None,
            "mean_queue_wait_s": float(wait.mean()) if wait.size else None,
        }
        if win and win > 0:
            out["offered_face_steps_per_s"] = sum(j.faces * j.nsteps for j in self.jobs) / win
        return out


class Server:
    def __init__(self, executor, budget_bytes: int, max_cohorts: int = 4, depth: int = 4,
                 max_jobs_per_cohort: int | None = None, idle_sleep: float = 2e-4):
        self.ex = executor
        self.budget = int(budget_bytes)
        self.max_cohorts = max_cohorts
        self.depth = depth
        self.max_jobs = max_jobs_per_cohort
        self.idle_sleep = idle_sleep

    def run(self, jobs) -> Report:
        ex = self.ex
        pending = deque(sorted(jobs, key=lambda j: (j.arrival, j.id)))
        sizing: list = []             # arrived, being sized
        queue: list = []              # sized, in arrival order
        starting: list = []           # (cohort, charged bytes)
        running: list = []            # (cohort, charged bytes)
        rep = Report(jobs=list(jobs))
        t0 = ex.now()
        used = 0
        while pending or sizing or queue or starting or running:
            now = ex.now() - t0
            progressed = False
            while pending and pending[0].arrival <= now:
                j = pending.popleft()
                ex.submit_estimate(j)
                sizing.append(j)
                progressed = True
            still = []
            for j in sizing:
                if not ex.estimate_ready(j):
                    still.append(j)
                elif j.bytes > self.budget:
                    j.rejected = True
                    ex.reject(j)
                else:
                    queue.append(j)
                    progressed = True
            sizing = still
            queue.sort(key=lambda j: (j.arrival, j.id))
            # admission: the queue head in arrival order (nothing overtakes a job still being sized)
            first_unsized = min((j.arrival, j.id) for j in sizing) if sizing else None
            if queue and len(starting) + len(running) < self.max_cohorts:
                take, extra = [], 0
                while (queue and used + extra + queue[0].bytes <= self.budget
                       and (first_unsized is None or (queue[0].arrival, queue[0].id) < first_unsized)
                       and (self.max_jobs is None or len(take) < self.max_jobs)):
                    take.append(queue.pop(0))
                    extra += take[-1].bytes
                if take:
                    t_adm = ex.now() - t0
                    for j in take:
                        j.t_admit = t_adm
                    starting.append((ex.submit_start(take), extra))
                    used += extra
                    rep.cohorts += 1
                    rep.peak_bytes = max(rep.peak_bytes, used)
                    progressed = True
            still = []
            for c, charged in starting:
                if ex.start_ready(c):
                    exact = ex.cohort_bytes(c)
                    used += exact - charged
                    rep.peak_bytes = max(rep.peak_bytes, used)
                    running.append((c, exact))
                    progressed = True
                else:
                    still.append((c, charged))
            starting = still
            for c, _ in running:
                while not ex.finished_enqueue(c) and ex.in_flight(c) < self.depth:
                    ex.step(c)
                    progressed = True
            keep = []
            for c, nbytes in running:
                for j, t in ex.poll(c):
                    j.t_done = t - t0
                    progressed = True
                if ex.all_done(c):
                    ex.release(c)
                    used -= nbytes
                else:
                    keep.append((c, nbytes))
            running = keep
            if not progressed:
                idle_all = not (sizing or queue or starting or running)
                nxt = pending[0].arrival - (ex.now() - t0) if pending and idle_all else None
                ex.idle(self.idle_sleep if nxt is None else max(min(nxt, 0.05), 0.0))
        rep.makespan = ex.now() - t0
        ex.shutdown()
        return rep


# ----------------------------------------------------------------------------- GPU executor
class GpuExecutor:
    """Cohorts as batch handles (BatchRun) on their own streams.  Job payloads
    are problem inputs (inputs.problem_inputs); the device footprint of a job
    is the workspace its mesh needs plus its resident arrays.  Sizing and
    cohort set-up run on host worker threads (the library's calls release the
    interpreter lock), so the loop keeps the device fed meanwhile."""

    def __init__(self, device, launch_config: dict | None = None, n_div: int = 10, workers: int = 2):
        import torch

        from . import gvof
        self.torch = torch
        self.gvof = gvof
        self.device = device
        self.launch_config = launch_config
        self.n_div = n_div
        self.pool = ThreadPoolExecutor(max_workers=workers)

    def now(self):
        return time.perf_counter()

    def idle(self, dt):
        time.sleep(dt)

    def shutdown(self):
        self.pool.shutdown(wait=True)

    # -- sizing: the job's mesh handle (kept for its cohort) and its footprint
    def estimate(self, job):
        g, m = self.gvof, job.payload["mesh"]
        h = g.gvof_mesh_create(m.vx, m.vy, m.vz, m.fv_ptr, m.fv_idx, m.owner, m.neigh, m.nc)
        job.part = h
        arrays = 8 * (3 * m.nf + 3 * m.nv + 2 * m.nc) + 9 * job.nsteps
        job.bytes = g.gvof_mesh_workspace_bytes(h) + arrays

    def submit_estimate(self, job):
        job._fut = self.pool.submit(self.estimate, job)

    def estimate_ready(self, job):
        if not job._fut.done():
            return False
        job._fut.result()  # re-raises a failure
        return True

    def reject(self, job):
        if getattr(job, "part", None) is not None:
            self.gvof.gvof_mesh_destroy(job.part)
            job.part = None

    # -- cohorts
    def _start(self, jobs):
        from .runtime import BatchRun
        torch = self.torch
        st = torch.cuda.Stream()
        parts = [j.part for j in jobs]
        for j in jobs:
            j.part = None
        R = BatchRun([j.payload for j in jobs], self.device, st, n_div=self.n_div, autotune=False,
                     launch_config=self.launch_config, parts=parts)
        for j in jobs:
            j.result = torch.empty(j.cells, dtype=torch.float64, pin_memory=True)
        st.synchronize()
        nbytes = int(R.B.ws_bytes) + sum(8 * (3 * j.payload["mesh"].nf + 3 * j.payload["mesh"].nv + 2 * j.cells)
                                         + 9 * j.nsteps for j in jobs)
        return dict(R=R, stream=st, events=deque(), pending=[], done=0, nbytes=nbytes)

    def submit_start(self, jobs):
        return dict(jobs=jobs, fut=self.pool.submit(self._start, jobs))

    def start_ready(self, c):
        if "R" in c:
            return True
        if not c["fut"].done():
            return False
        c.update(c["fut"].result())
        return True

    def cohort_bytes(self, c):
        return c["nbytes"]

    def finished_enqueue(self, c):
        return c["R"].done

    def in_flight(self, c):
        ev = c["events"]
        while ev and ev[0].query():
            ev.popleft()
        return len(ev)

    def step(self, c):
        R, st = c["R"], c["stream"]
        s = R.s
        R.step()
        with self.torch.cuda.stream(st):
            for q in R.finishing_at(s):
                j = c["jobs"][q]
                j.result.copy_(R.fractions(q), non_blocking=True)
                e = self.torch.cuda.Event()
                e.record(st)
                c["pending"].append((j, e))
            e = self.torch.cuda.Event()
            e.record(st)
        c["events"].append(e)

    def poll(self, c):
        out, keep = [], []
        for j, e in c["pending"]:
            if e.query():
                out.append((j, self.now()))
                c["done"] += 1
            else:
                keep.append((j, e))
        c["pending"] = keep
        return out

    def all_done(self, c):
        return c["done"] == len(c["jobs"])

    def release(self, c):
        c["stream"].synchronize()
        c["R"].status()
        c["R"].close()
        c["R"] = None


def jobs_from_specs(specs, problems):
    """Jobs from served-job specs and their generated inputs (same order)."""
    out = []
    for i, (s, p) in enumerate(zip(specs, problems)):
        out.append(Job(id=i, arrival=float(s["arrival"]), nsteps=int(p["nsteps"]), faces=int(p["mesh"].nf),
                       cells=int(p["mesh"].nc), payload=p))
    return out
