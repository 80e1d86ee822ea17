"""Serving loop logic on the CPU: a fake executor with a virtual clock and a
single virtual device that runs enqueued steps in order.  Checks admission by
budget and slots in arrival order, joins at step boundaries while other jobs
run, release of each job's memory when it finishes, rejection of jobs larger
than the budget, completion and latency accounting."""
from __future__ import annotations

import math

import pytest

from paper_2111_01524_amd import inputs
from paper_2111_01524_amd.serve import Job, Server


class FakeExecutor:
    """Sizing takes size_delay(job); a job's set-up is done setup_s after its
    admission (the loop does not wait for it); the device runs enqueued steps
    in order, a step of job j taking sec_per_face_step x its faces."""

    def __init__(self, sec_per_face_step=1e-8, setup_s=0.01, arrivals=(), size_delay=None):
        self.t = 0.0
        self.arrivals = sorted(arrivals)
        self.ends_all = []
        self.device_free = 0.0
        self.k = sec_per_face_step
        self.setup_s = setup_s
        self.size_delay = size_delay or (lambda job: 0.0)
        self.log = []          # (time, event, job id)
        self.live = 0          # bytes of jobs admitted and not released
        self.max_live = 0

    def now(self):
        return self.t

    def idle(self, dt):
        # jump to the next event (a step ending, a set-up or a size becoming ready, a job arriving)
        nxt = [e for e in self.ends_all if e > self.t] + [a for a in self.arrivals if a > self.t]
        self.t = max(self.t + max(dt, 1e-9), min(nxt)) if nxt else self.t + max(dt, 1e-6)

    def shutdown(self):
        pass

    def submit_estimate(self, job):
        job.bytes = job.faces * 100
        job._ready = self.t + self.size_delay(job)
        self.ends_all.append(job._ready)

    def estimate_ready(self, job):
        return self.t >= job._ready

    def reject(self, job):
        self.log.append((self.t, "reject", job.id))

    def submit_start(self, job):
        self.live += job.bytes
        self.max_live = max(self.max_live, self.live)
        self.log.append((self.t, "start", job.id))
        ready = self.t + self.setup_s
        self.ends_all.append(ready)
        return dict(job=job, s=0, ends=[], fin=None, ready=ready)

    def start_ready(self, h):
        return self.t >= h["ready"]

    def job_bytes(self, h):
        return h["job"].bytes

    def steps_left(self, h):
        return h["s"] < h["job"].nsteps

    def in_flight(self, h):
        return sum(1 for e in h["ends"] if e > self.t)

    def step(self, h):
        j = h["job"]
        if h["s"] == 0:
            self.log.append((self.t, "first_step", j.id))
        start = max(self.device_free, self.t)
        self.device_free = start + self.k * j.faces
        h["ends"].append(self.device_free)
        self.ends_all.append(self.device_free)
        h["s"] += 1
        if h["s"] == j.nsteps:
            h["fin"] = self.device_free

    def poll(self, h):
        return h["fin"] if h["fin"] is not None and h["fin"] <= self.t else None

    def release(self, h):
        self.live -= h["job"].bytes
        self.log.append((self.t, "release", h["job"].id))


def make_jobs(n=40, seed=3):
    specs = inputs.served_job_specs(duration_s=2.0, rate=20.0, seed=seed)[:n]
    jobs = []
    for i, s in enumerate(specs):
        faces = 3 * s["side"] ** 2 * (s["side"] + 1) * (4 if s["kind"] == "jittered" else 1)
        jobs.append(Job(id=i, arrival=s["arrival"], nsteps=s["steps"], faces=faces, cells=s["side"] ** 3))
    return jobs


def events(ex, kind):
    return {i: t for t, ev, i in ex.log if ev == kind}


def test_all_jobs_complete_with_correct_latency():
    jobs = make_jobs()
    ex = FakeExecutor(arrivals=[j.arrival for j in jobs])
    rep = Server(ex, budget_bytes=10 ** 12, slots=8, depth=4).run(jobs)
    S = rep.summary()
    assert S["completed"] == len(jobs) and S["rejected"] == 0 and S["admitted"] == len(jobs)
    for j in jobs:
        assert j.arrival - 1e-12 <= j.t_admit <= j.t_start < j.t_done
    # the virtual device is never idle while work is queued, so the makespan is
    # at least the total device time, and latency percentiles are ordered
    total = sum(ex.k * j.faces * j.nsteps for j in jobs)
    assert rep.makespan >= total - 1e-9
    assert S["p50_latency_s"] <= S["p99_latency_s"]
    assert S["value"] == pytest.approx(sum(j.faces * j.nsteps for j in jobs) / rep.makespan)


def test_budget_is_never_exceeded_and_oversized_jobs_are_rejected():
    jobs = make_jobs()
    big = max(j.faces for j in jobs)
    budget = big * 100 * 2 - 1  # at most one of the largest jobs at a time, plus smaller ones
    jobs.append(Job(id=999, arrival=0.5, nsteps=10, faces=budget, cells=10))  # 100x over the budget
    ex = FakeExecutor(arrivals=[j.arrival for j in jobs])
    rep = Server(ex, budget_bytes=budget, slots=8, depth=2).run(jobs)
    assert ex.max_live <= budget
    assert rep.peak_bytes <= budget
    rej = [j for j in jobs if j.rejected]
    assert [j.id for j in rej] == [999]
    assert rep.summary()["completed"] == len(jobs) - 1


def test_admission_is_in_arrival_order_and_respects_slots():
    jobs = make_jobs(30)
    ex = FakeExecutor(arrivals=[j.arrival for j in jobs])
    rep = Server(ex, budget_bytes=10 ** 12, slots=3, depth=1).run(jobs)
    started = [i for t, ev, i in ex.log if ev == "start"]
    assert started == sorted(range(len(jobs)), key=lambda i: (jobs[i].arrival, i))
    live = 0
    for t, ev, i in ex.log:
        live += 1 if ev == "start" else (-1 if ev == "release" else 0)
        assert live <= 3
    assert rep.max_running == 3


def test_arrivals_join_running_jobs_at_the_next_step_boundary():
    # a long job runs; later arrivals start and take steps while it still runs
    long = Job(id=0, arrival=0.0, nsteps=1000, faces=10 ** 6, cells=10)
    short = [Job(id=i, arrival=0.1 * i, nsteps=20, faces=10 ** 5, cells=10) for i in range(1, 6)]
    ex = FakeExecutor(sec_per_face_step=1e-9, setup_s=0.005, arrivals=[j.arrival for j in [long] + short])
    Server(ex, budget_bytes=10 ** 12, slots=8, depth=2).run([long] + short)
    first, rel = events(ex, "first_step"), events(ex, "release")
    for j in short:
        # its first step is enqueued once its set-up is done, at the first boundary after that
        assert j.t_start == pytest.approx(j.arrival + 0.005, abs=1e-3)
        assert first[j.id] == pytest.approx(j.t_start, abs=1e-3)
        assert j.t_done < rel[0]  # and it finishes while the long job still runs


def test_each_job_releases_its_memory_when_it_finishes():
    # room for two jobs: A (short) and B (long) run, C waits for memory and starts as soon as A is done
    A = Job(id=0, arrival=0.0, nsteps=10, faces=10 ** 5, cells=10)
    B = Job(id=1, arrival=0.0, nsteps=500, faces=10 ** 5, cells=10)
    C = Job(id=2, arrival=0.001, nsteps=10, faces=10 ** 5, cells=10)
    ex = FakeExecutor(sec_per_face_step=1e-8, setup_s=0.0, arrivals=[0.0, 0.001])
    rep = Server(ex, budget_bytes=2 * 10 ** 7, slots=8, depth=2).run([A, B, C])
    start, rel = events(ex, "start"), events(ex, "release")
    assert rel[0] <= start[2] < rel[1]
    assert start[2] == pytest.approx(A.t_done, abs=1e-3)
    assert rep.peak_bytes <= 2 * 10 ** 7


def test_latency_matches_single_job_service_time_when_idle():
    j = Job(id=0, arrival=0.0, nsteps=100, faces=10 ** 6, cells=10)
    ex = FakeExecutor(sec_per_face_step=1e-9, setup_s=0.02)
    rep = Server(ex, budget_bytes=10 ** 12).run([j])
    service = 0.02 + 100 * 1e-9 * 10 ** 6
    assert math.isclose(j.t_done - j.arrival, service, rel_tol=1e-6, abs_tol=5e-4)
    assert rep.summary()["p50_latency_s"] == pytest.approx(j.t_done - j.arrival)


def test_arrival_order_with_slow_sizing():
    # sizing takes longer for larger jobs, so sizes complete out of arrival order;
    # admission must still follow arrival order
    jobs = make_jobs(20)
    ex = FakeExecutor(arrivals=[j.arrival for j in jobs], size_delay=lambda j: j.faces * 2e-8)
    rep = Server(ex, budget_bytes=10 ** 12, slots=3, depth=2).run(jobs)
    started = [i for t, ev, i in ex.log if ev == "start"]
    assert started == sorted(range(len(jobs)), key=lambda i: (jobs[i].arrival, i))
    assert rep.summary()["completed"] == len(jobs)
