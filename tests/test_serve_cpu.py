"""Serving loop logic on the CPU: a fake executor with a virtual clock and a
single virtual device that runs enqueued steps in order.  Checks admission by
budget, arrival order, concurrency limits, rejection of jobs larger than the
budget, completion and latency accounting."""
from __future__ import annotations

import math

import numpy as np
import pytest

from paper_2111_01524_amd import inputs
from paper_2111_01524_amd.serve import Job, Server


class FakeExecutor:
    """Sizing is immediate; a cohort becomes ready setup_s after its admission
    (the loop does not wait for it); the device runs enqueued steps in order."""

    def __init__(self, sec_per_face_step=1e-8, setup_s=0.01, arrivals=(), size_delay=None):
        self.t = 0.0
        self.arrivals = sorted(arrivals)
        self.ends_all = []
        self.device_free = 0.0
        self.k = sec_per_face_step
        self.setup_s = setup_s
        self.size_delay = size_delay or (lambda job: 0.0)
        self.log = []          # (time, event, job ids)
        self.live = 0          # bytes of cohorts admitted and not released
        self.max_live = 0

    def now(self):
        return self.t

    def idle(self, dt):
        # jump to the next event (a step ending, a cohort or a size becoming ready, a job arriving)
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
        self.log.append((self.t, "reject", [job.id]))

    def submit_start(self, jobs):
        nbytes = sum(j.bytes for j in jobs)
        self.live += nbytes
        self.max_live = max(self.max_live, self.live)
        self.log.append((self.t, "start", [j.id for j in jobs]))
        ready = self.t + self.setup_s
        self.ends_all.append(ready)
        return dict(jobs=jobs, s=0, max=max(j.nsteps for j in jobs), ends=[], fin={}, done=set(), bytes=nbytes,
                    ready=ready)

    def start_ready(self, c):
        return self.t >= c["ready"]

    def cohort_bytes(self, c):
        return c["bytes"]

    def finished_enqueue(self, c):
        return c["s"] >= c["max"]

    def in_flight(self, c):
        return sum(1 for e in c["ends"] if e > self.t)

    def step(self, c):
        s = c["s"]
        faces = sum(j.faces for j in c["jobs"] if s < j.nsteps)
        start = max(self.device_free, self.t)
        self.device_free = start + self.k * faces
        c["ends"].append(self.device_free)
        self.ends_all.append(self.device_free)
        for j in c["jobs"]:
            if j.nsteps == s + 1:
                c["fin"][j.id] = self.device_free
        c["s"] = s + 1

    def poll(self, c):
        out = []
        for j in c["jobs"]:
            if j.id not in c["done"] and j.id in c["fin"] and c["fin"][j.id] <= self.t:
                c["done"].add(j.id)
                out.append((j, c["fin"][j.id]))
        return out

    def all_done(self, c):
        return len(c["done"]) == len(c["jobs"])

    def release(self, c):
        self.live -= c["bytes"]
        self.log.append((self.t, "release", [j.id for j in c["jobs"]]))


def make_jobs(n=40, seed=3):
    specs = inputs.served_job_specs(duration_s=2.0, rate=20.0, seed=seed)[:n]
    jobs = []
    for i, s in enumerate(specs):
        faces = 3 * s["side"] ** 2 * (s["side"] + 1) * (4 if s["kind"] == "jittered" else 1)
        jobs.append(Job(id=i, arrival=s["arrival"], nsteps=s["steps"], faces=faces, cells=s["side"] ** 3))
    return jobs


def test_all_jobs_complete_with_correct_latency():
    jobs = make_jobs()
    ex = FakeExecutor(arrivals=[j.arrival for j in jobs])
    rep = Server(ex, budget_bytes=10 ** 12, max_cohorts=4, depth=4).run(jobs)
    S = rep.summary()
    assert S["completed"] == len(jobs) and S["rejected"] == 0
    for j in jobs:
        assert j.t_admit >= j.arrival - 1e-12
        assert j.t_done > j.t_admit
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
    rep = Server(ex, budget_bytes=budget, max_cohorts=8, depth=2).run(jobs)
    assert ex.max_live <= budget
    assert rep.peak_bytes <= budget
    rej = [j for j in jobs if j.rejected]
    assert [j.id for j in rej] == [999]
    assert rep.summary()["completed"] == len(jobs) - 1


def test_admission_is_in_arrival_order_and_respects_cohort_limit():
    jobs = make_jobs(30)
    ex = FakeExecutor(arrivals=[j.arrival for j in jobs])
    Server(ex, budget_bytes=10 ** 12, max_cohorts=2, depth=1).run(jobs)
    started = [i for t, ev, ids in ex.log if ev == "start" for i in ids]
    order = sorted(range(len(jobs)), key=lambda i: (jobs[i].arrival, i))
    assert started == order
    # never more than two cohorts at a time
    live = 0
    for t, ev, ids in ex.log:
        live += 1 if ev == "start" else (-1 if ev == "release" else 0)
        assert live <= 2


def test_jobs_arriving_while_others_run_join_new_cohorts():
    # slow device: later arrivals are admitted while earlier cohorts are still running
    jobs = make_jobs(12)
    ex = FakeExecutor(sec_per_face_step=1e-9, arrivals=[j.arrival for j in jobs])
    rep = Server(ex, budget_bytes=10 ** 12, max_cohorts=4, depth=4).run(jobs)
    assert rep.cohorts >= 2
    starts = [(t, ids) for t, ev, ids in ex.log if ev == "start"]
    releases = [t for t, ev, ids in ex.log if ev == "release"]
    # some cohort started before the first one finished (overlap on the device)
    assert starts[1][0] < min(releases)


def test_latency_matches_single_job_service_time_when_idle():
    j = Job(id=0, arrival=0.0, nsteps=100, faces=10 ** 6, cells=10)
    ex = FakeExecutor(sec_per_face_step=1e-9, setup_s=0.02)
    rep = Server(ex, budget_bytes=10 ** 12).run([j])
    service = 0.02 + 100 * 1e-9 * 10 ** 6
    assert math.isclose(j.t_done - j.arrival, service, rel_tol=1e-6, abs_tol=5e-4)
    assert rep.summary()["p50_latency_s"] == pytest.approx(j.t_done - j.arrival)


def test_cohort_size_cap_and_arrival_order_with_slow_sizing():
    # sizing takes longer for larger jobs, so sizes complete out of arrival order;
    # admission must still follow arrival order, at most two jobs per cohort
    jobs = make_jobs(20)
    ex = FakeExecutor(arrivals=[j.arrival for j in jobs], size_delay=lambda j: j.faces * 2e-8)
    rep = Server(ex, budget_bytes=10 ** 12, max_cohorts=3, depth=2, max_jobs_per_cohort=2).run(jobs)
    starts = [ids for t, ev, ids in ex.log if ev == "start"]
    assert all(len(ids) <= 2 for ids in starts)
    order = sorted(range(len(jobs)), key=lambda i: (jobs[i].arrival, i))
    assert [i for ids in starts for i in ids] == order
    assert rep.summary()["completed"] == len(jobs)
