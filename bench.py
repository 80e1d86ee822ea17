"""Throughput of the LSGIR + FMFPA (or EMFPA) VOF step on one MI355X.

Workload (default): 64^3 uniform hexahedra on the unit cube, sphere r=0.15 at
(0.35, 0.35, 0.35) initialised by refinement (10 divisions), Enright 3D
deformation field with period T=3, CFL 0.5 (constant dt from the largest face
velocity, last step shortened to land on T), FP64.  One "step" is one pass of
the whole hot path: reconstruction (tags, cut-off, LSGIR, plane constants)
followed by the advection step (face flux volumes, FMFPA flux polyhedra with
truncation, update).  The field is u0(x) cos(pi t/T): the library receives
u0 at faces and vertices (resident in HBM) and dt * cos(pi t^{n+1/2}/T).

Prints one JSON line.  `value` = faces x steps / wall time of the timed steps
(all faces, boundary included), inputs resident in HBM.
"""
from __future__ import annotations

import argparse
import json
import math
import os
import sys
import time

import numpy as np

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

# Algorithmic FP64 operations per face that needs a flux polyhedron (its
# construction + truncation, and the truncation alone, which k_flux_items
# performs), by flux polyhedron method, and per interfacial cell (LSGIR +
# plane constant) on this workload, counted by the FLOP-counting build of the
# CPU reference over a sample of the trajectory (oracle/count_flops.py).
FLOPS_PER_FLUX_FACE = {"fmfpa": 38766.0, "emfpa": 49094.0, "nmfpa": 34525.0}
FLOPS_PER_FLUX_FACE_TRUNCATION = {"fmfpa": 37578.0, "emfpa": 47629.0, "nmfpa": 34030.0}
FLOPS_PER_RECON_CELL = 53202.0
FP64_VECTOR_PEAK_TFLOPS = 78.6
HBM_PEAK_GBS = 8000.0
# HBM bytes per launch of k_flux_items_box on this workload (FETCH_SIZE and
# WRITE_SIZE counters, scaled by the same counters on a plain copy kernel of
# known size; profiles/hbm_traffic_cartesian64_enright.md), valid for the
# kernel sources whose digest is recorded beside it.
ITEMS_BOX_TRAFFIC_BYTES = 2.82545e7
ITEMS_BOX_TRAFFIC_SOURCES = "eb4e382cf8ee7eb5"


def kernel_sources_digest() -> str:
    import hashlib
    h = hashlib.sha256()
    for f in ("gvof_kernels.hip", "clip.h", "gvof_dev.h"):
        with open(os.path.join(ROOT, "paper_2111_01524_amd", "csrc", f), "rb") as fh:
            h.update(fh.read())
    return h.hexdigest()[:16]


def parse():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=748)
    ap.add_argument("--warmup", type=int, default=20)
    ap.add_argument("--n", type=int, default=64)
    ap.add_argument("--kind", default="cartesian", choices=["cartesian", "jittered"])
    ap.add_argument("--method", default="fmfpa", choices=["fmfpa", "emfpa", "nmfpa"],
                    help="flux polyhedra: face-matched (the default workload), edge-matched or non-matched")
    ap.add_argument("--recon", default="lsgir", choices=["lsgir", "lsfir", "llcir", "elcir", "clcir"],
                    help="interface normals: LSGIR (the default workload), LSFIR, LLCIR, ELCIR or CLCIR")
    ap.add_argument("--lsfir-outer", type=int, default=1, help="LSFIR outer passes")
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--no-recon-leg", action="store_true",
                    help="skip the leg that times the reconstruction alone (cells/s)")
    ap.add_argument("--no-probes", action="store_true",
                    help="skip the measured FP64 FMA and copy ceilings (reported beside the published peaks)")
    ap.add_argument("--cpu-seconds", type=float, default=20.0)
    ap.add_argument("--profile-all", action="store_true", help="time every kernel with events (diagnostics)")
    ap.add_argument("--event-every", type=int, default=8,
                    help="bracket the truncation kernel with HIP events on every n-th timed step (each pair of "
                         "event records costs the stream a few microseconds)")
    ap.add_argument("--no-autotune", action="store_true", help="keep the library's default launch shapes")
    ap.add_argument("--launch-config", default=None,
                    help="JSON object of launch-shape fields to set instead of autotuning (others keep their defaults)")
    ap.add_argument("--batch", type=int, default=0,
                    help="also run the batched workload with this many problems (256 = the full batch)")
    ap.add_argument("--batch-steps", type=int, default=10)
    ap.add_argument("--batch-warmup", type=int, default=2)
    ap.add_argument("--single-steps", type=int, default=2, help="timed steps per problem of the one-by-one baseline")
    ap.add_argument("--served", type=int, default=0,
                    help="also serve this many jobs of the served workload (Poisson arrivals at 20/s)")
    ap.add_argument("--served-budget-gb", type=float, default=200.0)
    ap.add_argument("--served-cohort-jobs", type=int, default=2, help="most jobs per admitted cohort (0: no limit)")
    ap.add_argument("--copy-probe", type=int, default=0,
                    help="only run a plain device copy of this many MiB, 5 times (calibrates HBM byte counters)")
    return ap.parse_args()


def main():
    args = parse()
    if args.gpus != 1:
        print("bench.py measures one GPU: this build has no multi-GPU path (run with --gpus 1)", file=sys.stderr)
        sys.exit(2)
    if args.copy_probe > 0:
        copy_probe(args.copy_probe)
        return
    batch_problems = None
    if args.batch > 0:
        # host-side inputs first, in spawned workers, before anything touches the GPU
        from paper_2111_01524_amd import batch_inputs, inputs as _inputs
        t0 = time.perf_counter()
        batch_problems = batch_inputs.generate(_inputs.batch_problem_specs(args.batch))
        batch_gen_s = time.perf_counter() - t0
        print(f"# batch inputs: {args.batch} problems in {batch_gen_s:.1f} s", file=sys.stderr, flush=True)
    served = None
    if args.served > 0:
        from paper_2111_01524_amd import batch_inputs, inputs as _inputs
        t0 = time.perf_counter()
        sspecs = _inputs.served_job_specs()[: args.served]
        served = (sspecs, batch_inputs.generate(sspecs))
        print(f"# served inputs: {args.served} jobs in {time.perf_counter() - t0:.1f} s", file=sys.stderr, flush=True)
    import torch

    from paper_2111_01524_amd import gvof, inputs

    dev = torch.device("cuda:0")
    n, T_end, cfl = args.n, 3.0, 0.5
    mesh = inputs.cartesian_mesh(n) if args.kind == "cartesian" else inputs.jittered_mesh(n, seed=1)
    g = gvof.GvofMesh(mesh, dev, method=args.method, recon=args.recon, lsfir_outer=args.lsfir_outer)
    uf, uv = inputs.velocity_enright(mesh)
    dt = inputs.cfl_dt(mesh, np.abs(uf).max(axis=1), cfl)
    sched = inputs.step_schedule(T_end, dt)
    times = np.concatenate([[0.0], np.cumsum(sched)])
    dteff = [sched[s] * inputs.enright_time_factor(times[s] + 0.5 * sched[s], T_end) for s in range(len(sched))]
    ufd = torch.from_numpy(uf).to(dev)
    uvd = torch.from_numpy(uv).to(dev)
    F0 = g.init_fraction("sphere", [0.35, 0.35, 0.35, 0.15], 10)
    tuned = None
    if args.launch_config:
        d = gvof.gvof_get_launch_config(g.h).as_dict()
        d.update(json.loads(args.launch_config))
        gvof.gvof_set_launch_config(g.h, gvof.gvof_launch_config(**d))
    elif not args.no_autotune:
        # launch shapes measured at the middle of the trajectory, where the
        # interface is most stretched (the timed steps restart from F0)
        s_mid = len(sched) // 2
        Fm, Fn = F0.clone(), torch.empty_like(F0)
        for s in range(s_mid):
            g.reconstruct(Fm)
            g.advect_step(ufd, uvd, dteff[s], Fm, Fn)
            Fm, Fn = Fn, Fm
        dtm = torch.tensor([dteff[s_mid]], dtype=torch.float64, device=dev)
        act0 = torch.ones(1, dtype=torch.uint8, device=dev)
        cfg, tms = gvof.gvof_autotune(g.h, ufd, uvd, dtm, act0, Fm, Fn, 20)
        tuned = cfg.as_dict()
        del Fm, Fn
    torch.cuda.synchronize()
    state = {"s": 0}

    # ping-pong without copies
    bufs = [F0.clone(), torch.empty_like(F0)]

    def step_pp(reconstructs=1):
        s = state["s"]
        if s == len(sched):
            bufs[0].copy_(F0)
            s = 0
        for _ in range(reconstructs):
            g.reconstruct(bufs[0])
        g.advect_step(ufd, uvd, dteff[s], bufs[0], bufs[1])
        bufs[0], bufs[1] = bufs[1], bufs[0]
        state["s"] = s + 1

    for _ in range(args.warmup):
        step_pp()
    torch.cuda.synchronize()
    g.status()
    c0, f0 = gvof.gvof_work_totals(g.h)
    mask = (1 << gvof.GVOF_NUM_KERNELS) - 1 if args.profile_all else (1 << 5)  # k_flux_items_box
    every = 1 if args.profile_all else max(1, args.event_every)
    gvof.gvof_profile_read(g.h)  # clear
    stream = torch.cuda.current_stream(dev)
    e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
    torch.cuda.synchronize()
    t_wall = time.perf_counter()
    e0.record(stream)
    for i in range(args.steps):
        # the kernel's launch time is sampled on every `every`-th step, evenly over the timed region
        if i % every == 0:
            gvof.gvof_profile_enable(g.h, mask)
        step_pp()
        if i % every == 0:
            gvof.gvof_profile_enable(g.h, 0)
    e1.record(stream)
    torch.cuda.synchronize()
    t_wall = time.perf_counter() - t_wall
    ms_total = e0.elapsed_time(e1)
    prof = gvof.gvof_profile_read(g.h)
    gvof.gvof_profile_enable(g.h, 0)
    g.status()
    c1, f1 = gvof.gvof_work_totals(g.h)
    ncells_work, nfaces_work = c1 - c0, f1 - f0
    K = args.steps
    value = mesh.nf * K / (ms_total / 1e3)
    # Reconstruction time: the same warm-up and timed steps again with
    # gvof_reconstruct called twice per step.  The second call sees the
    # fractions it has already cut off and repeats the same work, so the
    # difference of the two timed runs is the reconstruction time.
    recon_ms = None
    if not args.no_recon_leg:
        bufs[0].copy_(F0)
        state["s"] = 0
        for _ in range(args.warmup):
            step_pp()
        torch.cuda.synchronize()
        r0, r1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
        r0.record(stream)
        for _ in range(args.steps):
            step_pp(reconstructs=2)
        r1.record(stream)
        torch.cuda.synchronize()
        g.status()
        recon_ms = (r0.elapsed_time(r1) - ms_total) / args.steps
    flux_ms, flux_n = prof["k_flux_items_box"]
    flux_ms_avg = flux_ms / max(flux_n, 1)
    flops_per_face = FLOPS_PER_FLUX_FACE_TRUNCATION[args.method]
    flux_flops_per_launch = flops_per_face * nfaces_work / K  # one launch per step
    achieved_tflops = flux_flops_per_launch / (flux_ms_avg / 1e3) / 1e12 if flux_ms_avg > 0 else 0.0
    out = {
        "metric": "face·step flux updates/s",
        "value": value,
        "unit": "face·steps/s",
        "n_gpus": 1,
        "steps": K,
        "warmup": args.warmup,
        "ms_per_step": ms_total / K,
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "f64",
        "data": "synthetic",
        "config": {
            "workload": f"{args.kind} {n}^3 unit cube, sphere r=0.15 at 0.35, Enright deformation T=3, CFL 0.5, "
                        f"{args.recon.upper()}{f' ({args.lsfir_outer} outer)' if args.recon == 'lsfir' else ''}"
                        f"+{args.method.upper()}, {len(sched)} steps per trajectory",
            "faces": mesh.nf, "cells": mesh.nc, "vertices": mesh.nv,
        },
        "cells_per_s": (mesh.nc / (recon_ms / 1e3) if recon_ms and recon_ms > 0 else None),
        "reconstruct_ms_per_step": recon_ms,
        "interfacial_faces_steps_per_s": nfaces_work / (ms_total / 1e3),
        "launch_config": tuned if tuned is not None else gvof.gvof_get_launch_config(g.h).as_dict(),
        "launch_config_autotuned": tuned is not None,
        "interfacial_faces_per_step": nfaces_work / K,
        "interfacial_cells_per_step": ncells_work / K,
        "wall_s": t_wall,
        "roofline": {
            "bound": "alu",
            "kernel": "k_flux_items_box",
            "achieved": achieved_tflops,
            "peak": FP64_VECTOR_PEAK_TFLOPS,
            "unit": "TFLOP/s",
            "frac": achieved_tflops / FP64_VECTOR_PEAK_TFLOPS,
            "traffic": (ITEMS_BOX_TRAFFIC_BYTES
                        if kernel_sources_digest() == ITEMS_BOX_TRAFFIC_SOURCES and args.method == "fmfpa"
                        and args.kind == "cartesian" and n == 64 else None),
            "traffic_unit": "bytes per launch (HBM, counters)",
            "avg_launch_ms": flux_ms_avg,
            "flops_per_unit": flops_per_face,
            "unit_of_work": "face needing a flux polyhedron (truncation FLOPs)",
            "units_per_launch": nfaces_work / K,
            "launches_timed": flux_n,
        },
    }
    if not args.no_probes:
        # measured ceilings: an FP64 FMA loop (libgvof_probe) and a plain copy
        from paper_2111_01524_amd import probe
        fma_tflops = probe.measure_fp64_fma(dev)
        out["probes"] = {"fp64_fma_tflops": fma_tflops, "copy_gbs": probe.measure_copy(dev)}
        out["roofline"]["peak_measured"] = fma_tflops
        out["roofline"]["frac_measured"] = achieved_tflops / fma_tflops
    if args.profile_all:
        out["kernels_ms_per_launch"] = {k: (v[0] / v[1] if v[1] else 0.0) for k, v in prof.items()}
    if batch_problems is not None:
        del g, bufs, ufd, uvd
        torch.cuda.empty_cache()
        out["batched"] = batched_leg(args, batch_problems, dev)
    if served is not None:
        torch.cuda.empty_cache()
        out["served"] = served_leg(args, served, dev)
    if not args.no_cpu_baseline:
        out["cpu_baseline"] = cpu_baseline(mesh, uf, uv, sched, dteff, args.cpu_seconds, args.method, args.recon,
                                           args.lsfir_outer)
    print(json.dumps(out), flush=True)


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


def served_leg(args, served, dev):
    """The served workload: the first jobs of the seeded Poisson arrival
    stream (20 jobs/s, sides 32..128, both grid kinds, 50..500 steps), each
    arriving at its own time with its inputs in host memory; admitted under
    the HBM budget into cohorts that run concurrently; latency from arrival to
    the job's fractions in host memory."""
    from paper_2111_01524_amd import serve

    specs, problems = served
    jobs = serve.jobs_from_specs(specs, problems)
    ex = serve.GpuExecutor(dev)
    srv = serve.Server(ex, budget_bytes=int(args.served_budget_gb * 1e9), max_cohorts=4, depth=4,
                       max_jobs_per_cohort=args.served_cohort_jobs or None)
    rep = srv.run(jobs)
    window = max(s["arrival"] for s in specs)
    S = rep.summary(arrival_window=window)
    S["unit"] = "face·steps/s"
    S["workload"] = (f"first {len(specs)} jobs of the Poisson stream (20/s, seed 3), arrivals over {window:.2f} s, "
                     f"sides {sorted(set(s['side'] for s in specs))}, budget {args.served_budget_gb:g} GB, "
                     f"at most 4 cohorts of {args.served_cohort_jobs or 'any number of'} jobs")
    S["latency_includes_queueing"] = True
    return S


def batched_leg(args, problems, dev):
    """The batched workload (independent problems of uneven sizes and grid
    kinds, each with its own sphere, period and time step) advanced together:
    one captured step per graph launch, launch shapes autotuned, against the
    same problems advanced one after another through the single-problem calls."""
    import torch

    from paper_2111_01524_amd import gvof
    from paper_2111_01524_amd.runtime import BatchRun

    st = torch.cuda.Stream()
    t0 = time.perf_counter()
    R = BatchRun(problems, dev, st)
    setup_s = time.perf_counter() - t0
    print(f"# batch bound: nf={R.B.nf} nc={R.B.nc} setup {setup_s:.1f} s tuned {R.tuned}", file=sys.stderr, flush=True)
    W, K = args.batch_warmup, args.batch_steps
    for _ in range(W):
        R.step()
    st.synchronize()
    e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
    e0.record(st)
    for _ in range(K):
        R.step()
    e1.record(st)
    st.synchronize()
    R.status()
    ms = e0.elapsed_time(e1)
    fs = R.face_steps(W, W + K)
    res = {
        "workload": f"{R.nprob} problems, sides 16..48, Cartesian or distorted (+-0.25h), sphere r~U[0.1,0.2], "
                    f"centre~U[0.3,0.7]^3, Enright period T~U[1,3], CFL 0.5; steps {W}..{W + K - 1}",
        "faces": int(R.B.nf), "cells": int(R.B.nc),
        "value": fs / (ms / 1e3), "unit": "face·steps/s", "ms_per_step": ms / K, "steps": K, "warmup": W,
        "launch_config": R.tuned[0] if R.tuned else None, "autotune_ms_per_step": R.tuned[1] if R.tuned else None,
        "setup_s": setup_s,
    }
    R.close()
    del R
    torch.cuda.empty_cache()
    # the same problems one after another, each on its own handle, single-problem calls
    Ks = args.single_steps
    tot_ms, tot_fs = 0.0, 0
    with torch.cuda.stream(st):
        for qi, p in enumerate(problems):
            if qi % 32 == 0:
                print(f"# one-by-one: problem {qi}/{len(problems)}", file=sys.stderr, flush=True)
            g = gvof.GvofMesh(p["mesh"], dev, stream=st)
            ufd, uvd = torch.from_numpy(p["uf"]).to(dev), torch.from_numpy(p["uv"]).to(dev)
            F = g.init_fraction(p["shape"][0], p["shape"][1], 10)
            g.reconstruct(F)
            g.advect_step(ufd, uvd, p["dt_eff"][0], F, F)
            e0.record(st)
            for s in range(1, 1 + Ks):
                g.reconstruct(F)
                g.advect_step(ufd, uvd, p["dt_eff"][min(s, p["nsteps"] - 1)], F, F)
            e1.record(st)
            st.synchronize()
            tot_ms += e0.elapsed_time(e1)
            tot_fs += p["mesh"].nf * Ks
            g.status()
            g.close()
            del g, F, ufd, uvd
    res["one_by_one"] = {"value": tot_fs / (tot_ms / 1e3), "unit": "face·steps/s",
                         "sample": f"every problem alone, steps 1..{Ks} after one untimed step, sum of event times"}
    res["speedup_vs_one_by_one"] = res["value"] / res["one_by_one"]["value"]
    return res


def cpu_baseline(mesh, uf, uv, sched, dteff, budget_s, method, recon, lsfir_outer):
    """The CPU reference (as it stands) on the host cores: the first steps of the same trajectory."""
    from oracle import oracle as O
    threads = O.set_threads(int(os.environ.get("OMP_NUM_THREADS", "0") or 0) or (os.cpu_count() or 1))
    om = O.OracleMesh(mesh, method=method, recon=recon, lsfir_outer=lsfir_outer)
    F = om.init_fraction("sphere", [0.35, 0.35, 0.35, 0.15], 10)
    t0 = time.perf_counter()
    done = 0
    while done < len(sched):
        Fc, Fs, tn, tf, tc, pl = om.reconstruct(F)
        F, Vd, VF, up, bad = om.advect(pl, tc, tf, uf, uv, dteff[done], Fc)
        done += 1
        if time.perf_counter() - t0 > budget_s and done >= 2:
            break
    el = time.perf_counter() - t0
    return {"value": mesh.nf * done / el, "unit": "face·steps/s", "cores": threads, "kind": "oracle",
            "sample": f"first {done} steps of the same trajectory from t=0 on the full mesh ({el:.1f} s)"}


if __name__ == "__main__":
    main()
