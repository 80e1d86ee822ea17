"""Serving loop: advection jobs arriving over time, admitted under an HBM
budget, advanced with continuous (step-level) batching.

The scheduler is written against a small executor interface so that its
logic (arrival order, admission by budget and slots, joins at step
boundaries, release on completion, latency accounting) runs unchanged on the
GPU executor and on a fake one with a virtual clock (the CPU tests).

Policy.
  - Every arriving job is sized first (its mesh topology and device
    footprint, on a host worker, while the device keeps running).
  - Sized jobs queue in arrival order; a job never overtakes an earlier
    arrival, nor one still being sized.
  - The job at the head of the queue is admitted as soon as a slot is free
    (at most `slots` jobs starting or running) and its footprint fits what is
    left of the budget.  Its device state (mesh and workspace, velocities,
    fractions; the PLIC planes live in the workspace) is set up on a host
    worker and stays resident until the job is done.  A job larger than the
    whole budget is rejected.
  - At every step boundary of the loop each running job gets its next steps
    enqueued (up to `depth` in flight per job, each job on its own stream), so
    a job admitted while others run joins them at the next boundary and the
    steps of all running jobs overlap on the device.
  - A job's result is ready when the copy of its fractions after its own last
    step has completed; latency = ready time - arrival time.  The job's slot
    and its memory are released at that moment, and the queue head may start.
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
    t_start: float | None = None  # set-up done: the job joins the running set
    t_done: float | None = None
    rejected: bool = False
    result: object = None
    part: object = None           # executor state held between sizing and set-up


@dataclass
class Report:
    jobs: list = field(default_factory=list)
    makespan: float = 0.0
    peak_bytes: int = 0
    admitted: int = 0
    max_running: int = 0          # most jobs starting or running at once

    def summary(self, arrival_window: float | None = None) -> dict:
        done = [j for j in self.jobs if j.t_done is not None]
        lat = np.array([j.t_done - j.arrival for j in done]) if done else np.zeros(0)
        wait = np.array([j.t_admit - j.arrival for j in done]) if done else np.zeros(0)
        fs = sum(j.faces * j.nsteps for j in done)
        win = arrival_window if arrival_window is not None else (max(j.arrival for j in self.jobs) if self.jobs else 0)
        out = {
            "jobs": len(self.jobs), "completed": len(done), "rejected": sum(j.rejected for j in self.jobs),
            "admitted": self.admitted, "max_concurrent_jobs": self.max_running, "makespan_s": self.makespan,
            "peak_hbm_bytes": self.peak_bytes, "face_steps": fs,
            "value": fs / self.makespan if self.makespan > 0 else 0.0,
            "p50_latency_s": float(np.percentile(lat, 50)) if lat.size else None,
            "p99_latency_s": float(np.percentile(lat, 99)) if lat.size else None,
            "mean_queue_wait_s": float(wait.mean()) if wait.size else None,
        }
        if win and win > 0:
            out["arrival_window_s"] = win
            out["offered_face_steps_per_s"] = sum(j.faces * j.nsteps for j in self.jobs) / win
        return out


class Server:
    def __init__(self, executor, budget_bytes: int, slots: int = 16, depth: int = 2, idle_sleep: float = 2e-4):
        self.ex = executor
        self.budget = int(budget_bytes)
        self.slots = slots
        self.depth = depth
        self.idle_sleep = idle_sleep

    def run(self, jobs, on_done=None) -> Report:
        """Serve the jobs; on_done(job) is called when a job's result is ready."""
        ex = self.ex
        key = lambda j: (j.arrival, j.id)  # noqa: E731
        pending = deque(sorted(jobs, key=key))
        sizing: list = []             # arrived, being sized
        queue: list = []              # sized, in arrival order
        starting: list = []           # (job, handle, charged bytes)
        running: list = []            # (job, handle, bytes)
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
            queue.sort(key=key)
            # admission: the queue head, while a slot is free and it fits (nothing overtakes a job still being sized)
            first_unsized = min(key(j) for j in sizing) if sizing else None
            while (queue and len(starting) + len(running) < self.slots and used + queue[0].bytes <= self.budget
                   and (first_unsized is None or key(queue[0]) < first_unsized)):
                j = queue.pop(0)
                j.t_admit = ex.now() - t0
                starting.append((j, ex.submit_start(j), j.bytes))
                used += j.bytes
                rep.admitted += 1
                rep.peak_bytes = max(rep.peak_bytes, used)
                rep.max_running = max(rep.max_running, len(starting) + len(running))
                progressed = True
            # set-ups that are done join the running jobs at this step boundary
            still = []
            for j, h, charged in starting:
                if ex.start_ready(h):
                    exact = ex.job_bytes(h)
                    used += exact - charged
                    rep.peak_bytes = max(rep.peak_bytes, used)
                    j.t_start = ex.now() - t0
                    running.append((j, h, exact))
                    progressed = True
                else:
                    still.append((j, h, charged))
            starting = still
            # the step boundary: the next steps of every running job
            for j, h, _ in running:
                while ex.steps_left(h) and ex.in_flight(h) < self.depth:
                    ex.step(h)
                    progressed = True
            # completions: the slot and the memory come back at once
            keep = []
            for j, h, nbytes in running:
                t = ex.poll(h)
                if t is None:
                    keep.append((j, h, nbytes))
                    continue
                j.t_done = t - t0
                ex.release(h)
                if on_done is not None:
                    on_done(j)
                used -= nbytes
                progressed = True
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
    """Each running job is a resident single-problem handle with its own
    stream.  Job payloads are problem inputs (inputs.problem_inputs); the
    device footprint of a job is the workspace its mesh needs plus its
    resident arrays.  Sizing and set-up run on host worker threads (the
    library's calls release the interpreter lock), so the loop keeps the
    device fed meanwhile."""

    def __init__(self, device, launch_config: dict | None = None, n_div: int = 10, workers: int = 2,
                 reserve_cap_bytes: int | None = None):
        import torch

        from . import gvof
        self.torch = torch
        self.gvof = gvof
        self.device = device
        self.launch_config = launch_config
        self.n_div = n_div
        self.pool = ThreadPoolExecutor(max_workers=workers)
        # torch's caching allocator keeps a released job's blocks for its stream; jobs of other sizes on other
        # streams then allocate afresh, so the cache can outgrow the budget.  Past this cap (by default 85% of
        # the device), a set-up about to allocate and a release hand the unused blocks back to the device.
        total = torch.cuda.get_device_properties(device).total_memory
        self.reserve_cap = int(reserve_cap_bytes if reserve_cap_bytes is not None else 0.85 * total)

    def now(self):
        return time.perf_counter()

    def idle(self, dt):
        time.sleep(dt)

    def shutdown(self):
        self.pool.shutdown(wait=True)

    @staticmethod
    def array_bytes(mesh, nsteps: int) -> int:
        """Resident arrays of a job besides its workspace: u at faces and vertices, two fraction buffers."""
        return 8 * (3 * mesh.nf + 3 * mesh.nv + 2 * mesh.nc) + 9 * nsteps

    # -- sizing: the job's mesh handle (kept for its set-up) and its footprint
    def estimate(self, job):
        g, m = self.gvof, job.payload["mesh"]
        h = g.gvof_mesh_create(m.vx, m.vy, m.vz, m.fv_ptr, m.fv_idx, m.owner, m.neigh, m.nc)
        job.part = h
        job.bytes = g.gvof_mesh_workspace_bytes(h) + self.array_bytes(m, job.nsteps)

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

    # -- set-up: bind the handle to a workspace, upload the velocities, initialise the fractions
    def _start(self, job):
        torch, p = self.torch, job.payload
        if torch.cuda.memory_reserved(self.device) + job.bytes > self.reserve_cap:
            torch.cuda.empty_cache()
        st = torch.cuda.Stream(self.device)
        h, job.part = job.part, None
        with torch.cuda.stream(st):
            g = self.gvof.GvofMesh(p["mesh"], self.device, stream=st, handle=h)
            if self.launch_config is not None:
                d = self.gvof.gvof_get_launch_config(g.h).as_dict()
                d.update(self.launch_config)
                self.gvof.gvof_set_launch_config(g.h, self.gvof.gvof_launch_config(**d))
            uf = torch.from_numpy(p["uf"]).to(self.device)
            uv = torch.from_numpy(p["uv"]).to(self.device)
            F = g.init_fraction(p["shape"][0], p["shape"][1], self.n_div)
            Fn = torch.empty_like(F)
        job.result = torch.empty(p["mesh"].nc, dtype=torch.float64, pin_memory=True)
        st.synchronize()
        nbytes = int(g.ws_bytes) + self.array_bytes(p["mesh"], job.nsteps)
        return dict(job=job, g=g, stream=st, uf=uf, uv=uv, F=F, Fn=Fn, s=0, events=deque(), done_ev=None,
                    nbytes=nbytes)

    def submit_start(self, job):
        return dict(fut=self.pool.submit(self._start, job))

    def start_ready(self, h):
        if "g" in h:
            return True
        if not h["fut"].done():
            return False
        h.update(h["fut"].result())
        return True

    def job_bytes(self, h):
        return h["nbytes"]

    def steps_left(self, h):
        return h["s"] < h["job"].nsteps

    def in_flight(self, h):
        ev = h["events"]
        while ev and ev[0].query():
            ev.popleft()
        return len(ev)

    def step(self, h):
        torch, j, s = self.torch, h["job"], h["s"]
        with torch.cuda.stream(h["stream"]):
            h["g"].reconstruct(h["F"])
            h["g"].advect_step(h["uf"], h["uv"], float(j.payload["dt_eff"][s]), h["F"], h["Fn"])
            h["F"], h["Fn"] = h["Fn"], h["F"]
            e = torch.cuda.Event()
            e.record(h["stream"])
            if s + 1 == j.nsteps:
                j.result.copy_(h["F"], non_blocking=True)
                h["done_ev"] = torch.cuda.Event()
                h["done_ev"].record(h["stream"])
        h["events"].append(e)
        h["s"] = s + 1

    def poll(self, h):
        e = h["done_ev"]
        if e is not None and e.query():
            return self.now()
        return None

    def release(self, h):
        h["stream"].synchronize()
        g = h["g"]
        g.status()
        g.close()
        for k in ("g", "uf", "uv", "F", "Fn", "events", "done_ev"):
            h[k] = None
        if self.torch.cuda.memory_reserved(self.device) > self.reserve_cap:
            self.torch.cuda.empty_cache()


def jobs_from_specs(specs, problems):
    """Jobs from served-job specs and their generated inputs (same order)."""
    out = []
    for i, (s, p) in enumerate(zip(specs, problems)):
        out.append(Job(id=i, arrival=float(s["arrival"]), nsteps=int(p["nsteps"]), faces=int(p["mesh"].nf),
                       cells=int(p["mesh"].nc), payload=p))
    return out
