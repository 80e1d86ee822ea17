"""Throughput of the unsplit geometric VOF step (LSGIR + FMFPA) on one MI355X.

Workloads (--workload):
  batch      the default, the largest single-GPU workload: 256 independent
             problems (seed 2): sides 16..48, Cartesian or distorted
             (interior vertices moved by up to 0.25h per axis) with
             probability 1/2, sphere r ~ U[0.1, 0.2] at U[0.3, 0.7]^3,
             Enright 3D deformation with period T ~ U[1, 3], CFL 0.5; every
             problem advances to its own T with its own time step; one step
             of the batch is one replay of a captured HIP graph.
  jittered   64^3 distorted grid (seed 1), sphere r = 0.15 at 0.35, Enright
             field with T = 3, CFL 0.5.
  cartesian  64^3 Cartesian grid, same body and field.
All arithmetic is FP64.  One step = reconstruction (tags, cut-off, LSGIR,
plane constants) + advection (V_d, FMFPA polyhedra, truncation, update) of
every active problem.  The library receives u0 at faces and vertices
(resident in HBM) and dt cos(pi t^{n+1/2}/T) per problem.

Timed steps.  An untimed pass runs the whole trajectory once and keeps the
volume fractions before K steps spread evenly over it (step s_i =
floor((i + 1/2) S / K)); W untimed warm-up steps follow; then each timed step
restores its saved fractions (outside the timed events) and runs once,
bracketed by HIP events on the library's stream.  So a short run measures
the trajectory as a whole, not its first steps.  `value` = faces of the
active problems summed over the timed steps / the summed event times (all
faces, boundary included; inputs resident in HBM).

Also reported: the same steps as graph replays (single-problem workloads) or
eagerly (batch); the batch's problems advanced one by one (a sample);
per-kernel times over the same steps with their rooflines; the oracle on the
host's cores; the other workloads as sub-records.  Prints one JSON line.
"""
from __future__ import annotations

import argparse
import json
import math
import os
import platform
import sys
import time

import numpy as np

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

FP64_VECTOR_PEAK_TFLOPS = 78.6
HBM_PEAK_GBS = 8000.0


def parse():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=20, help="timed steps, spread evenly over the trajectory")
    ap.add_argument("--warmup", type=int, default=5)
    ap.add_argument("--workload", default="batch", choices=["batch", "jittered", "cartesian"])
    ap.add_argument("--n", type=int, default=64, help="grid side of the single-problem workloads")
    ap.add_argument("--method", default="fmfpa", choices=["fmfpa", "emfpa", "nmfpa"],
                    help="flux polyhedron of the single-problem workloads")
    ap.add_argument("--recon", default="lsgir", choices=["lsgir", "lsfir", "llcir", "elcir", "clcir"],
                    help="interface reconstruction of the single-problem workloads")
    ap.add_argument("--problems", type=int, default=256, help="problems of the batch workload")
    ap.add_argument("--no-sub", action="store_true", help="skip the other workloads' sub-records")
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--cpu-seconds", type=float, default=10.0, help="budget of each CPU baseline run")
    ap.add_argument("--no-probes", action="store_true")
    ap.add_argument("--no-kernels", action="store_true", help="skip the per-kernel timing pass")
    ap.add_argument("--no-autotune", action="store_true")
    ap.add_argument("--launch-config", default=None, help="JSON launch shapes instead of autotuning")
    ap.add_argument("--single-sample", type=int, default=32, help="batch problems timed one by one")
    ap.add_argument("--served", type=int, default=0,
                    help="serve this many jobs of the served workload at --served-load of the capacity measured first "
                         "(the served run alone: no other workload)")
    ap.add_argument("--served-load", type=float, default=0.75, help="offered load, a fraction of the measured capacity")
    ap.add_argument("--served-capacity-jobs", type=int, default=24,
                    help="jobs (all arriving at once) of the capacity run")
    ap.add_argument("--served-budget-gb", type=float, default=200.0)
    ap.add_argument("--served-slots", type=int, default=16)
    ap.add_argument("--copy-probe", type=int, default=0, help="only run a plain copy of this many MiB, 5 times")
    ap.add_argument("--dump-states", default=None,
                    help="directory: save the fractions before each timed step and the launch shapes, per workload")
    ap.add_argument("--load-states", default=None,
                    help="directory written by --dump-states: take the states and shapes from there (no untimed pass, "
                         "no tuning)")
    ap.add_argument("--timed-only", action="store_true",
                    help="run only the warm-up and timed steps of the main workload (for profiler runs that should "
                         "see exactly those dispatches), print their times")
    return ap.parse_args()


# ------------------------------------------------------------------ helpers
def snapshot_steps(S: int, K: int):
    """K steps spread evenly over a trajectory of S steps."""
    return [min(S - 1, int(math.floor((i + 0.5) * S / K))) for i in range(K)]


def cpu_model() -> str:
    try:
        with open("/proc/cpuinfo") as f:
            for line in f:
                if line.startswith("model name"):
                    return line.split(":", 1)[1].strip()
    except OSError:
        pass
    return platform.processor() or "unknown"


class EventPairs:
    """Per-step HIP events on one stream; the summed time of the bracketed work."""

    def __init__(self, torch, n):
        self.a = [torch.cuda.Event(enable_timing=True) for _ in range(n)]
        self.b = [torch.cuda.Event(enable_timing=True) for _ in range(n)]

    def ms(self):
        return [a.elapsed_time(b) for a, b in zip(self.a, self.b)]


def kernel_table(gvof, prof):
    return {k: (v[0] / v[1] if v[1] else 0.0, v[1]) for k, v in prof.items()}


# Work per unit, by workload and kernel, from the rocprofv3 runs summarised in
# profiles/ (paper_2111_01524_amd/profile_summary.py): FP64 FLOPs of the active
# lanes and HBM bytes per unit of the kernel's work (faces that need a flux
# polyhedron, interface cells, or all faces / cells), measured over the same
# timed steps of the same workload.
def load_work_table():
    p = os.path.join(ROOT, "profiles", "work_per_unit.json")
    if os.path.exists(p):
        with open(p) as f:
            return json.load(f)
    return {}


def kernel_sources_digest() -> str:
    """Digest of the kernel sources (the counters in profiles/ hold for the sources they were taken on)."""
    from paper_2111_01524_amd.profile_summary import sources_digest
    return sources_digest()


# kernels whose work is FP64 arithmetic (the flux polyhedra, their truncation, the reconstruction); the others
# are sweeps over faces, cells or vertices, bound by HBM
ALU_KERNELS = {"k_flux_prep", "k_flux_items_box", "k_flux_gen_filter", "k_flux_gen_units", "k_flux_gen_units_deep",
               "k_flux_deep", "k_recon"}


def rooflines(kt, step_ms, counts, table, workload):
    """Rooflines of every kernel taking 10% of the step or more, largest first.  A kernel's achieved rate is its
    work per unit x the units of the timed steps (counted on the device) over its summed launch time over the same
    steps (HIP events around each launch on the library's stream)."""
    out = []
    K = counts["steps"]
    fresh = table.get("sources_digest") == kernel_sources_digest()
    for k, (avg_ms, n) in sorted(kt.items(), key=lambda kv: -kv[1][0] * kv[1][1]):
        if n == 0 or avg_ms <= 0:
            continue
        per_step = avg_ms * n / K
        if per_step < 0.1 * step_ms:
            continue
        ent = {"kernel": k, "avg_launch_ms": avg_ms, "launches": n, "ms_per_step": per_step,
               "share_of_step": per_step / step_ms}
        spec = table.get(workload, {}).get(k)
        if spec:
            units = counts[spec["unit"]]
            secs = avg_ms * n / 1e3
            tf = spec["flops"] * units / secs / 1e12
            gb = spec["bytes"] * units / secs / 1e9
            if k in ALU_KERNELS:
                ent.update(bound="alu", unit="TFLOP/s", peak=FP64_VECTOR_PEAK_TFLOPS, achieved=tf,
                           frac=tf / FP64_VECTOR_PEAK_TFLOPS)
            else:
                ent.update(bound="hbm", unit="GB/s", peak=HBM_PEAK_GBS, achieved=gb, frac=gb / HBM_PEAK_GBS)
            ent.update(counters_match_sources=fresh, flops_per_unit=spec["flops"], issued_flops_per_unit=spec["flops_issued"],
                       hbm_bytes_per_unit=spec["bytes"], hbm_gbs=gb, hbm_frac=gb / HBM_PEAK_GBS,
                       fp64_tflops=tf, unit_of_work=spec["unit"], units_per_launch=units / n,
                       traffic=spec["bytes"] * units / n if fresh else None,
                       profile_avg_launch_ms=spec["avg_launch_ms"],
                       profile_units_per_launch=spec["units_per_launch"], work_source=spec["source"])
            if "valu_issue_frac" in spec:  # the profiled run's VALU issue time over its run time (what binds it)
                ent["profile_valu_issue_frac"] = spec["valu_issue_frac"]
        out.append(ent)
    return out


def dump_states(args, name, steps, snaps, launch_config):
    if not args.dump_states or args.load_states:
        return
    os.makedirs(args.dump_states, exist_ok=True)
    np.savez(os.path.join(args.dump_states, f"{name}.npz"), steps=np.array(steps),
             F=np.stack([x.cpu().numpy() for x in snaps]), launch_config=json.dumps(launch_config))


def load_states(args, name):
    if not args.load_states:
        return None
    with np.load(os.path.join(args.load_states, f"{name}.npz")) as d:
        return {"steps": [int(x) for x in d["steps"]], "F": d["F"], "launch_config": json.loads(str(d["launch_config"]))}


# ------------------------------------------------------------------ single problem
def single_leg(args, kind, dev, K, W):
    import torch

    from paper_2111_01524_amd import gvof, inputs

    n, T_end, cfl = args.n, 3.0, 0.5
    mesh = inputs.cartesian_mesh(n) if kind == "cartesian" else inputs.jittered_mesh(n, seed=1)
    st = torch.cuda.Stream()
    g = gvof.GvofMesh(mesh, dev, stream=st, method=args.method, recon=args.recon)
    scheme = f"{args.recon.upper()}+{args.method.upper()}"
    name = kind if scheme == "LSGIR+FMFPA" else f"{kind}_{args.recon}_{args.method}"
    uf, uv = inputs.velocity_enright(mesh)
    dt = inputs.cfl_dt(mesh, np.abs(uf).max(axis=1), cfl)
    sched = inputs.step_schedule(T_end, dt)
    S = len(sched)
    times = np.concatenate([[0.0], np.cumsum(sched)])
    dteff = [sched[s] * inputs.enright_time_factor(times[s] + 0.5 * sched[s], T_end) for s in range(S)]
    steps = snapshot_steps(S, K)
    loaded = load_states(args, name)
    with torch.cuda.stream(st):
        ufd = torch.from_numpy(uf).to(dev)
        uvd = torch.from_numpy(uv).to(dev)
        F0 = g.init_fraction("sphere", [0.35, 0.35, 0.35, 0.15], 10)
        Fa, Fb = F0.clone(), torch.empty_like(F0)
        snaps = {}
        if loaded is not None:
            steps = loaded["steps"]
            snaps = {s: torch.from_numpy(loaded["F"][i]).to(dev) for i, s in enumerate(steps)}
        else:
            for s in range(S):  # the untimed pass: fractions before each timed step
                if s in steps:
                    snaps[s] = Fa.clone()
                g.reconstruct(Fa)
                g.advect_step(ufd, uvd, dteff[s], Fa, Fb)
                Fa, Fb = Fb, Fa
        st.synchronize()
        g.status()
        tuned = None
        if loaded is not None:
            gvof.gvof_set_launch_config(g.h, gvof.gvof_launch_config(**loaded["launch_config"]))
        elif args.launch_config:
            d = gvof.gvof_get_launch_config(g.h).as_dict()
            d.update(json.loads(args.launch_config))
            gvof.gvof_set_launch_config(g.h, gvof.gvof_launch_config(**d))
        elif not args.no_autotune:  # shapes measured where the interface is most stretched
            sm = steps[len(steps) // 2]
            Fm = snaps[sm].clone()
            dtm = torch.tensor([dteff[sm]], dtype=torch.float64, device=dev)
            act = torch.ones(1, dtype=torch.uint8, device=dev)
            cfg, _ = gvof.gvof_autotune(g.h, ufd, uvd, dtm, act, Fm, Fb, 20)
            tuned = cfg.as_dict()
        dump_states(args, name, steps, [snaps[s] for s in steps], gvof.gvof_get_launch_config(g.h).as_dict())
        Fw, Fo = torch.empty_like(F0), torch.empty_like(F0)

        def one(s):
            g.reconstruct(Fw)
            g.advect_step(ufd, uvd, dteff[s], Fw, Fo)

        for i in range(W):  # warm-up, untimed
            Fw.copy_(snaps[steps[i % K]])
            one(steps[i % K])
        st.synchronize()
        c0, f0 = gvof.gvof_work_totals(g.h)
        ev = EventPairs(torch, K)
        torch.cuda.synchronize()
        t_wall = time.perf_counter()
        for i, s in enumerate(steps):
            Fw.copy_(snaps[s])
            ev.a[i].record(st)
            one(s)
            ev.b[i].record(st)
        torch.cuda.synchronize()
        t_wall = time.perf_counter() - t_wall
        g.status()
        c1, f1 = gvof.gvof_work_totals(g.h)
        ms = ev.ms()
        if args.timed_only:
            g.close()
            return {"workload": f"{kind} {n}^3 Enright T=3, CFL 0.5, {scheme}", "name": name,
                    "ms_per_step": sum(ms) / K, "timed_steps": steps,
                    "interfacial_faces_per_step": (f1 - f0) / K, "interfacial_cells_per_step": (c1 - c0) / K,
                    "faces_per_step": mesh.nf, "cells_per_step": mesh.nc}, None
        # the same steps as replays of a captured step (one graph launch per step)
        dtg = torch.zeros(1, dtype=torch.float64, device=dev)
        actg = torch.ones(1, dtype=torch.uint8, device=dev)
        Fg = torch.empty_like(F0)
        Fg.copy_(snaps[steps[0]])
        gvof.gvof_graph_capture(g.h, ufd, uvd, dtg, actg, Fg)
        dt_rows = torch.tensor([dteff[s] for s in steps], dtype=torch.float64, device=dev)
        evg = EventPairs(torch, K)
        for i, s in enumerate(steps):
            Fg.copy_(snaps[s])
            dtg.copy_(dt_rows[i:i + 1])
            evg.a[i].record(st)
            gvof.gvof_graph_launch(g.h)
            evg.b[i].record(st)
        torch.cuda.synchronize()
        g.status()
        msg = evg.ms()
        # per-kernel times over the same steps (events around every kernel; not in the values above)
        kt, kcounts = None, None
        if not args.no_kernels:
            gvof.gvof_profile_read(g.h)
            k0 = gvof.gvof_work_totals(g.h)
            for i, s in enumerate(steps):
                Fw.copy_(snaps[s])
                gvof.gvof_profile_enable(g.h, (1 << gvof.GVOF_NUM_KERNELS) - 1)
                one(s)
                gvof.gvof_profile_enable(g.h, 0)
            torch.cuda.synchronize()
            kt = kernel_table(gvof, gvof.gvof_profile_read(g.h))
            k1 = gvof.gvof_work_totals(g.h)
            kcounts = {"steps": K, "interfacial_faces": k1[1] - k0[1], "interfacial_cells": k1[0] - k0[0],
                       "faces": mesh.nf * K, "cells": mesh.nc * K}
    tot = sum(ms)
    res = {
        "workload": f"{kind} {n}^3 unit cube, sphere r=0.15 at 0.35, Enright deformation T=3, CFL 0.5, {scheme}, "
                    f"{S} steps per trajectory; timed steps {steps[0]}..{steps[-1]} spread evenly",
        "name": name, "faces": mesh.nf, "cells": mesh.nc, "vertices": mesh.nv, "trajectory_steps": S,
        "timed_steps": steps,
        "value": mesh.nf * K / (tot / 1e3), "unit": "face·steps/s", "ms_per_step": tot / K,
        "value_graph": mesh.nf * K / (sum(msg) / 1e3), "ms_per_step_graph": sum(msg) / K,
        "cells_per_s": mesh.nc * K / (tot / 1e3),
        "interfacial_faces_per_step": (f1 - f0) / K, "interfacial_cells_per_step": (c1 - c0) / K,
        "launch_config": tuned if tuned is not None else gvof.gvof_get_launch_config(g.h).as_dict(),
        "launch_config_autotuned": tuned is not None, "wall_s": t_wall,
    }
    if kt is not None:
        res["kernels_ms_per_launch"] = {k: v[0] for k, v in kt.items() if v[1]}
        res["rooflines"] = rooflines(kt, tot / K, kcounts, load_work_table(), name)
    ctx = dict(mesh=mesh, uf=uf, uv=uv, dteff=dteff, steps=steps, snaps={s: v.cpu().numpy() for s, v in snaps.items()})
    g.close()
    del snaps, Fa, Fb, Fw, Fo, Fg
    torch.cuda.empty_cache()
    return res, ctx


# ------------------------------------------------------------------ batch
def batch_leg(args, problems, dev, K, W):
    import torch

    from paper_2111_01524_amd import gvof
    from paper_2111_01524_amd.runtime import BatchRun

    st = torch.cuda.Stream()
    t0 = time.perf_counter()
    R = BatchRun(problems, dev, st, autotune=False, graph=False)
    setup_s = time.perf_counter() - t0
    S = R.max_steps
    steps = snapshot_steps(S, K)
    print(f"# batch bound: nf={R.B.nf} nc={R.B.nc} setup {setup_s:.1f} s, {S} steps", file=sys.stderr, flush=True)
    snaps = {}
    loaded = load_states(args, "batch")
    with torch.cuda.stream(st):
        if loaded is not None:
            steps = loaded["steps"]
            snaps = {s: torch.from_numpy(loaded["F"][i]).to(dev) for i, s in enumerate(steps)}
        else:
            while not R.done:  # the untimed pass
                if R.s in steps:
                    snaps[R.s] = R.F.clone()
                R.step()
                if R.s % 100 == 0:
                    st.synchronize()
                    print(f"# batch untimed pass: step {R.s}/{S}", file=sys.stderr, flush=True)
        st.synchronize()
        R.status()
        tuned = None
        if loaded is not None:
            gvof.gvof_set_launch_config(R.B.h, gvof.gvof_launch_config(**loaded["launch_config"]))
        elif args.launch_config:
            d = gvof.gvof_get_launch_config(R.B.h).as_dict()
            d.update(json.loads(args.launch_config))
            gvof.gvof_set_launch_config(R.B.h, gvof.gvof_launch_config(**d))
        elif not args.no_autotune:  # shapes measured in the middle of the pass
            sm = steps[len(steps) // 2]
            R.F.copy_(snaps[sm])
            R.dt.copy_(R.dt_tab[sm])
            R.act.copy_(R.act_tab[sm])
            cfg, tms = R.B.autotune(R.uf, R.uv, R.dt, R.act, R.F, reps=2)
            tuned = (cfg.as_dict(), tms)
        dump_states(args, "batch", steps, [snaps[s] for s in steps], gvof.gvof_get_launch_config(R.B.h).as_dict())
        # timed steps: graph replays; with --timed-only (the profiler runs) the same steps launched eagerly,
        # as the per-kernel pass below launches them
        graph = not args.timed_only
        if graph:
            R.B.capture(R.uf, R.uv, R.dt, R.act, R.F)
            R.graph = True

        def one(s):
            R.dt.copy_(R.dt_tab[s])
            R.act.copy_(R.act_tab[s])

        def run():
            if graph:
                R.B.replay()
            else:
                R.B.step(R.uf, R.uv, R.dt, R.act, R.F)

        for i in range(W):
            R.F.copy_(snaps[steps[i % K]])
            one(steps[i % K])
            run()
        st.synchronize()
        ev = EventPairs(torch, K)
        torch.cuda.synchronize()
        c0, f0 = gvof.gvof_work_totals(R.B.h)
        t_wall = time.perf_counter()
        for i, s in enumerate(steps):
            R.F.copy_(snaps[s])
            one(s)
            ev.a[i].record(st)
            run()
            ev.b[i].record(st)
        torch.cuda.synchronize()
        t_wall = time.perf_counter() - t_wall
        R.status()
        c1, f1 = gvof.gvof_work_totals(R.B.h)
        ms = ev.ms()
        fs = sum(R.face_steps(s, s + 1) for s in steps)
        cs = sum(int(R.act_host[s].astype(np.int64) @ R.nc_q) for s in steps)
        if args.timed_only:
            R.close()
            return {"workload": f"batch of {R.nprob} problems (Enright, LSGIR+FMFPA)", "name": "batch",
                    "ms_per_step": sum(ms) / K, "timed_steps": steps, "face_steps_timed": fs,
                    "interfacial_faces_per_step": (f1 - f0) / K, "interfacial_cells_per_step": (c1 - c0) / K,
                    "faces_per_step": fs / K, "cells_per_step": cs / K}, None
        # the same steps eagerly (the kernels launched one by one), then per kernel
        eve = EventPairs(torch, K)
        for i, s in enumerate(steps):
            R.F.copy_(snaps[s])
            one(s)
            eve.a[i].record(st)
            R.B.step(R.uf, R.uv, R.dt, R.act, R.F)
            eve.b[i].record(st)
        torch.cuda.synchronize()
        mse = eve.ms()
        kt, kcounts = None, None
        if not args.no_kernels:
            gvof.gvof_profile_read(R.B.h)
            k0 = gvof.gvof_work_totals(R.B.h)
            for i, s in enumerate(steps):
                R.F.copy_(snaps[s])
                one(s)
                gvof.gvof_profile_enable(R.B.h, (1 << gvof.GVOF_NUM_KERNELS) - 1)
                R.B.step(R.uf, R.uv, R.dt, R.act, R.F)
                gvof.gvof_profile_enable(R.B.h, 0)
            torch.cuda.synchronize()
            kt = kernel_table(gvof, gvof.gvof_profile_read(R.B.h))
            k1 = gvof.gvof_work_totals(R.B.h)
            kcounts = {"steps": K, "interfacial_faces": k1[1] - k0[1], "interfacial_cells": k1[0] - k0[0],
                       "faces": fs, "cells": cs}
    tot = sum(ms)
    res = {
        "workload": f"batch of {R.nprob} problems (seed 2): sides 16..48, Cartesian or distorted (+-0.25h), sphere "
                    f"r~U[0.1,0.2] at U[0.3,0.7]^3, Enright deformation T~U[1,3], CFL 0.5, LSGIR+FMFPA; each problem "
                    f"to its own end time ({S} batch steps); one graph launch per batch step; timed steps "
                    f"{steps[0]}..{steps[-1]} spread evenly",
        "problems": R.nprob, "faces": int(R.B.nf), "cells": int(R.B.nc), "trajectory_steps": S, "timed_steps": steps,
        "value": fs / (tot / 1e3), "unit": "face·steps/s", "ms_per_step": tot / K,
        "value_eager": fs / (sum(mse) / 1e3), "ms_per_step_eager": sum(mse) / K,
        "face_steps_timed": fs, "setup_s": setup_s, "wall_s": t_wall,
        "interfacial_faces_per_step": (f1 - f0) / K, "interfacial_cells_per_step": (c1 - c0) / K,
        "launch_config": tuned[0] if tuned else gvof.gvof_get_launch_config(R.B.h).as_dict(),
        "launch_config_autotuned": tuned is not None,
    }
    if kt is not None:
        res["kernels_ms_per_launch"] = {k: v[0] for k, v in kt.items() if v[1]}
        res["rooflines"] = rooflines(kt, sum(mse) / K, kcounts, load_work_table(), "batch")
    # a sample of the problems one by one (single-problem calls, their own handles), at the same steps
    # from the same states (a problem's fractions in the batch equal its fractions alone, bit for bit)
    sample = list(range(0, R.nprob, max(1, R.nprob // max(1, args.single_sample))))[: args.single_sample]
    tot1, fs1 = 0.0, 0
    with torch.cuda.stream(st):
        for q in sample:
            p = problems[q]
            g = gvof.GvofMesh(p["mesh"], dev, stream=st)
            ufq, uvq = torch.from_numpy(p["uf"]).to(dev), torch.from_numpy(p["uv"]).to(dev)
            Fq, Fo = torch.empty(p["mesh"].nc, dtype=torch.float64, device=dev), None
            Fo = torch.empty_like(Fq)
            act = [s for s in steps if s < p["nsteps"]]
            evq = EventPairs(torch, len(act))
            for j, s in enumerate(act):
                Fq.copy_(snaps[s][R.B.cells(q)])
                evq.a[j].record(st)
                g.reconstruct(Fq)
                g.advect_step(ufq, uvq, p["dt_eff"][s], Fq, Fo)
                evq.b[j].record(st)
            st.synchronize()
            g.status()
            tot1 += sum(evq.ms())
            fs1 += p["mesh"].nf * len(act)
            g.close()
    res["one_by_one"] = {"value": fs1 / (tot1 / 1e3) if tot1 > 0 else None, "unit": "face·steps/s",
                         "sample": f"{len(sample)} of the {R.nprob} problems, each alone through the single-problem "
                                   f"calls at the timed steps where it is active, from the same states"}
    res["speedup_vs_one_by_one"] = res["value"] / res["one_by_one"]["value"] if tot1 > 0 else None
    ctx = dict(problems=problems, steps=steps, cell_off=R.B.cell_off, snaps={s: v.cpu().numpy() for s, v in snaps.items()})
    R.close()
    del snaps
    torch.cuda.empty_cache()
    return res, ctx


# ------------------------------------------------------------------ CPU baseline
def cpu_run(jobs, budget_s, threads):
    """The oracle (as it stands) on (mesh, F, u_f, u_v, dt) jobs until the budget is spent: face-steps/s and the
    reconstruct / advect split."""
    from oracle import oracle as O
    used = O.set_threads(threads)
    rec = adv = 0.0
    fs = done = 0
    t0 = time.perf_counter()
    cache = {}
    for key, mesh, F, uf, uv, dt in jobs:
        om = cache.get(key)
        if om is None:
            om = cache[key] = O.OracleMesh(mesh)
        a = time.perf_counter()
        Fc, Fs, tn, tf, tc, pl = om.reconstruct(F)
        b = time.perf_counter()
        om.advect(pl, tc, tf, uf, uv, dt, Fc)
        c = time.perf_counter()
        rec += b - a
        adv += c - b
        fs += mesh.nf
        done += 1
        if time.perf_counter() - t0 > budget_s:
            break
    return {"value": fs / (rec + adv), "threads": used, "steps": done, "reconstruct_s": rec, "advect_s": adv}


def cpu_baseline(jobs_all, jobs_one, budget_s, what):
    allc = cpu_run(jobs_all, budget_s, int(os.environ.get("OMP_NUM_THREADS", "0") or 0) or (os.cpu_count() or 1))
    one = cpu_run(jobs_one, budget_s, 1)
    return {"value": allc["value"], "unit": "face·steps/s", "cores": allc["threads"], "kind": "oracle",
            "cpu_model": cpu_model(),
            "sample": f"{what}: {allc['steps']} (problem, step) states with all threads in {allc['reconstruct_s'] + allc['advect_s']:.1f} s",
            "reconstruct_s": allc["reconstruct_s"], "advect_s": allc["advect_s"],
            "one_thread": {"value": one["value"], "steps": one["steps"], "reconstruct_s": one["reconstruct_s"],
                           "advect_s": one["advect_s"]}}


def batch_cpu_jobs(ctx):
    """(problem, step) states of the batch's timed steps: problems in a spread order, each at every timed step
    where it is active, so that a bounded run covers problems of every size and kind and the whole trajectory."""
    P, steps, off = ctx["problems"], ctx["steps"], ctx["cell_off"]
    order = sorted(range(len(P)), key=lambda q: (q % 16, q))
    jobs = []
    for q in order:
        for s in steps:
            if s < P[q]["nsteps"]:
                jobs.append((q, P[q]["mesh"], ctx["snaps"][s][off[q]:off[q + 1]], P[q]["uf"], P[q]["uv"],
                             P[q]["dt_eff"][s]))
    return jobs


def single_cpu_jobs(ctx):
    m = ctx["mesh"]
    return [(0, m, ctx["snaps"][s], ctx["uf"], ctx["uv"], ctx["dteff"][s]) for s in ctx["steps"]]


# ------------------------------------------------------------------ main
def main():
    t_start = time.perf_counter()
    args = parse()
    if args.gpus != 1:
        print("bench.py measures one GPU: this build has no multi-GPU path (run with --gpus 1)", file=sys.stderr)
        sys.exit(2)
    if args.copy_probe > 0:
        copy_probe(args.copy_probe)
        return
    K, W = args.steps, args.warmup
    if args.served > 0:
        import torch
        print(json.dumps(served_leg(args, torch.device("cuda:0"))), flush=True)
        return
    problems = None
    if args.workload == "batch":
        from paper_2111_01524_amd import batch_inputs, inputs as _inputs
        t0 = time.perf_counter()
        problems = batch_inputs.generate(_inputs.batch_problem_specs(args.problems))
        print(f"# batch inputs: {len(problems)} problems in {time.perf_counter() - t0:.1f} s", file=sys.stderr,
              flush=True)
    import torch

    dev = torch.device("cuda:0")
    if args.workload == "batch":
        head, ctx = batch_leg(args, problems, dev, K, W)
    else:
        head, ctx = single_leg(args, args.workload, dev, K, W)
    if args.timed_only:
        print(json.dumps(head), flush=True)
        return
    subs = []
    sub_ctx = {}
    if not args.no_sub:
        for kind in ("jittered", "cartesian"):
            if kind != args.workload:
                print(f"# sub-record: {kind}", file=sys.stderr, flush=True)
                r, c = single_leg(args, kind, dev, K, W)
                subs.append(r)
                sub_ctx[r["name"]] = c
    out = {
        "metric": "face·step flux updates/s",
        "value": head["value"],
        "unit": "face·steps/s",
        "n_gpus": 1,
        "steps": K,
        "warmup": W,
        "ms_per_step": head["ms_per_step"],
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "f64",
        "data": "synthetic",
        "config": {k: head[k] for k in ("workload", "faces", "cells") if k in head},
    }
    if "problems" in head:
        out["config"]["problems"] = head["problems"]
    rl = head.get("rooflines") or []
    if rl:
        out["roofline"] = rl[0]
        out["rooflines"] = rl
    for k in head:
        if k not in ("value", "unit", "ms_per_step", "workload", "faces", "cells", "problems", "rooflines"):
            out[k] = head[k]
    if not args.no_probes:
        from paper_2111_01524_amd import probe
        out["probes"] = {"fp64_fma_tflops": probe.measure_fp64_fma(dev), "copy_gbs": probe.measure_copy(dev)}
    if subs:
        out["sub_records"] = subs
    if not args.no_cpu_baseline:
        if args.workload == "batch":
            jobs = batch_cpu_jobs(ctx)
            out["cpu_baseline"] = cpu_baseline(jobs, jobs, args.cpu_seconds,
                                               "the batch's problems at its timed steps, from the same states")
        else:
            jobs = single_cpu_jobs(ctx)
            out["cpu_baseline"] = cpu_baseline(jobs, jobs, args.cpu_seconds, "the timed steps, from the same states")
        for r in subs:  # the sub-records' own baselines, on half the budget
            jobs = single_cpu_jobs(sub_ctx[r["name"]])
            r["cpu_baseline"] = cpu_baseline(jobs, jobs, 0.5 * args.cpu_seconds,
                                             "the timed steps, from the same states")
    print(json.dumps(out), flush=True)
    print(f"# bench done in {time.perf_counter() - t_start:.1f} s", file=sys.stderr, flush=True)


def copy_probe(mib: int):
    """A plain copy of mib MiB (FP64), five launches: reads and writes mib MiB each."""
    import torch
    n = mib * (1 << 20) // 8
    src = torch.arange(n, dtype=torch.float64, device="cuda:0")
    dst = torch.empty_like(src)
    torch.cuda.synchronize()
    for _ in range(5):
        dst.copy_(src)
    torch.cuda.synchronize()
    print(json.dumps({"copy_probe_bytes_per_launch": n * 8, "launches": 5}), flush=True)


def served_specs(n: int, seed: int = 3, seeds_per_side: int = 4):
    """The served workload's first n jobs (Poisson arrivals at 20/s, sides 32..128, half distorted, 50..500
    steps), with the distorted grids drawn from a pool of seeds_per_side jitter seeds per side."""
    from paper_2111_01524_amd import inputs
    specs = inputs.served_job_specs(duration_s=2.0 * n / 20.0 + 10.0, rate=20.0, seed=seed)[:n]
    for s in specs:
        s["jitter_seed"] = 5000 + s["jitter_seed"] % seeds_per_side
    return specs


def served_leg(args, dev):
    """A capacity run (the first jobs all arriving at once), then args.served jobs whose Poisson arrivals are
    slowed so that the offered load is args.served_load x that capacity.  Latency = result ready - arrival."""
    from paper_2111_01524_amd import batch_inputs, inputs, serve

    n_cap, N = args.served_capacity_jobs, args.served
    specs = served_specs(max(N, n_cap))
    t0 = time.perf_counter()
    G = batch_inputs.grids(specs)
    problems = [inputs.problem_inputs(s, grids=G) for s in specs]
    print(f"# served: {len(specs)} jobs on {len(G)} grids, inputs in {time.perf_counter() - t0:.1f} s", file=sys.stderr,
          flush=True)
    budget = int(args.served_budget_gb * 1e9)

    def progress(tag, n):
        cnt = [0]

        def cb(j):
            cnt[0] += 1
            if cnt[0] % 4 == 0 or cnt[0] == n:
                print(f"# served {tag}: {cnt[0]}/{n} done", file=sys.stderr, flush=True)
        return cb

    cap_specs = [dict(s, arrival=0.0) for s in specs[:n_cap]]
    rep = serve.Server(serve.GpuExecutor(dev, workers=6), budget, slots=args.served_slots).run(
        serve.jobs_from_specs(cap_specs, problems[:n_cap]), progress("capacity", n_cap))
    cap = rep.summary(arrival_window=0.0)
    capacity = cap["value"]
    import torch
    torch.cuda.empty_cache()  # the capacity run's cached blocks go back before the sustained run
    fs = [p["mesh"].nf * p["nsteps"] for p in problems[:N]]
    rate = args.served_load * capacity / (sum(fs) / N)  # jobs per second
    sus_specs = [dict(s, arrival=s["arrival"] * 20.0 / rate) for s in specs[:N]]
    jobs = serve.jobs_from_specs(sus_specs, problems[:N])
    rep = serve.Server(serve.GpuExecutor(dev, workers=6), budget, slots=args.served_slots).run(
        jobs, progress("sustained", N))
    window = max(s["arrival"] for s in sus_specs)
    S = rep.summary(arrival_window=window)
    lat = np.array([j.t_done - j.arrival for j in jobs if j.t_done is not None])
    run = np.array([j.t_done - j.t_start for j in jobs if j.t_done is not None])
    return {
        "metric": "served face·steps/s; p50/p99 latency", "unit": "face·steps/s",
        "workload": f"served jobs (seed 3): sides 32/64/96/128, Cartesian or distorted (+-0.25h; 4 jitter seeds per "
                    f"side), sphere r~U[0.1,0.2] at U[0.3,0.7]^3, Enright deformation T~U[1,3], CFL 0.5, 50..500 "
                    f"steps, LSGIR+FMFPA; budget {args.served_budget_gb:g} GB, {args.served_slots} slots",
        "capacity": {"jobs": n_cap, "value": capacity, "makespan_s": cap["makespan_s"],
                     "how": "all jobs arriving at t=0, face·steps / makespan"},
        "target_load": args.served_load, "arrival_rate_jobs_per_s": rate,
        "sustained": S,
        "latency_s": {"p50": S["p50_latency_s"], "p90": float(np.percentile(lat, 90)), "p99": S["p99_latency_s"],
                      "max": float(lat.max())},
        "run_time_s": {"p50": float(np.percentile(run, 50)), "p99": float(np.percentile(run, 99))},
        "offered_vs_capacity": S.get("offered_face_steps_per_s", 0.0) / capacity if capacity else None,
    }


if __name__ == "__main__":
    main()
