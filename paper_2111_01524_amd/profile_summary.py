"""Summaries of rocprofv3 runs of bench.py for profiles/ (tables as text), and
the work-per-unit table bench.py reads for its rooflines.

Each workload is profiled over exactly the timed steps of a bench run: the
states before those steps are saved by `bench.py --dump-states DIR`, and every
profiled run is `bench.py --workload W --load-states DIR --timed-only
--warmup 0`, which restores them and runs only the timed steps, so that the
kernel times and the counters cover the same dispatches.  Per workload:

  <run>/<W>_trace  rocprofv3 --kernel-trace --stats
  <run>/<W>_fetch  rocprofv3 --pmc FETCH_SIZE
  <run>/<W>_write  rocprofv3 --pmc WRITE_SIZE
  <run>/<W>_fp64   rocprofv3 --pmc SQ_INSTS_VALU_ADD_F64 SQ_INSTS_VALU_MUL_F64
                   SQ_INSTS_VALU_FMA_F64 SQ_INSTS_VALU_TRANS_F64 SQ_INSTS_VALU
                   SQ_ACTIVE_INST_VALU SQ_THREAD_CYCLES_VALU SQ_WAVES
  <run>/<W>.json   the timed-only run's output (the units it advanced)

and, for the HBM calibration, <run>/copy_fetch and <run>/copy_write: the same
two counters over `bench.py --copy-probe MIB` (a plain copy of known size).

FLOPs.  The SQ_INSTS_VALU_*_F64 counters count wavefront instructions; the
lane FLOPs they issue are 64 (ADD + MUL + TRANS + 2 FMA).  Lanes that are
masked off still issue, so the FLOPs of the lanes that do work are taken as
that figure times the kernel's active-lane fraction of VALU work,
SQ_THREAD_CYCLES_VALU / (64 SQ_ACTIVE_INST_VALU).  That is the executed FP64
arithmetic of the kernel's live lanes, the basis of bench.py's 'alu'
rooflines; the issued figure is kept beside it.

Usage: python -m paper_2111_01524_amd.profile_summary RUN_DIR [--copy-mib M] [--out profiles]
"""
from __future__ import annotations

import argparse
import csv
import json
import os
import re
from collections import defaultdict

# the library's per-kernel timing slot of each kernel (bench.py's per-kernel table)
SLOT = {"k_flux_gen_runs": "k_flux_gen_filter"}
# the unit each kernel's work is counted per: faces that need a flux polyhedron,
# cells with an interface (tag 0), or every face / cell of the active problems
UNIT = {"k_flux_prep": "interfacial_faces", "k_flux_items_box": "interfacial_faces",
        "k_flux_gen_filter": "interfacial_faces", "k_flux_gen_units": "interfacial_faces",
        "k_flux_gen_units_deep": "interfacial_faces", "k_flux_gen_sum": "interfacial_faces",
        "k_flux_deep": "interfacial_faces", "k_flux_sum": "interfacial_faces", "k_recon": "interfacial_cells",
        "k_face_sweep": "faces", "k_node_tag": "faces", "k_cell_tag": "cells", "k_update": "cells"}


def sources_digest() -> str:
    """Digest of the code of the HIP sources the kernels are built from (comments and whitespace excluded,
    so that editing a comment does not disown the counters taken on the same kernels)."""
    import hashlib
    h = hashlib.sha256()
    d = os.path.join(os.path.dirname(os.path.abspath(__file__)), "csrc")
    for f in sorted(os.listdir(d)):
        if f.endswith((".hip", ".h")):
            with open(os.path.join(d, f)) as fh:
                text = fh.read()
            text = re.sub(r"/\*.*?\*/", " ", text, flags=re.S)
            text = re.sub(r"//[^\n]*", " ", text)
            h.update(f.encode() + b"\0" + " ".join(text.split()).encode())
    return h.hexdigest()[:16]


def base_name(kernel: str) -> str:
    k = kernel.split("(")[0].strip()
    k = re.sub(r"^void\s+", "", k)
    k = re.sub(r"<.*>$", "", k)
    k = k.split("::")[-1]
    return SLOT.get(k, k)


def read_csv(path):
    with open(path, newline="") as f:
        return list(csv.DictReader(f))


def find(dirpath, suffix):
    for root, _, files in os.walk(dirpath):
        for f in files:
            if f.endswith(suffix):
                return os.path.join(root, f)
    raise FileNotFoundError(f"{dirpath}/*{suffix}")


def counters(dirpath):
    """Counter sums per kernel slot and the slot's dispatch count."""
    tot = defaultdict(lambda: defaultdict(float))
    disp = defaultdict(set)
    for r in read_csv(find(dirpath, "counter_collection.csv")):
        k = base_name(r["Kernel_Name"])
        tot[k][r["Counter_Name"]] += float(r["Counter_Value"])
        disp[k].add(r["Dispatch_Id"])
    return tot, {k: len(v) for k, v in disp.items()}


def kernel_times(dirpath):
    """Per slot: dispatches and total ns (kernel trace of the run)."""
    out = defaultdict(lambda: [0, 0.0])
    for r in read_csv(find(dirpath, "kernel_trace.csv")):
        k = base_name(r["Kernel_Name"])
        out[k][0] += 1
        out[k][1] += float(r["End_Timestamp"]) - float(r["Start_Timestamp"])
    return out


def calibration(run, mib):
    """HBM bytes per KiB of FETCH_SIZE and of WRITE_SIZE, from a plain copy of mib MiB (read and written once)."""
    f, nf = counters(os.path.join(run, "copy_fetch"))
    w, nw = counters(os.path.join(run, "copy_write"))
    kf = max(f, key=lambda k: f[k].get("FETCH_SIZE", 0.0))
    kw = max(w, key=lambda k: w[k].get("WRITE_SIZE", 0.0))
    per_f = f[kf]["FETCH_SIZE"] / nf[kf]
    per_w = w[kw]["WRITE_SIZE"] / nw[kw]
    nbytes = mib * (1 << 20)
    return nbytes / per_f, nbytes / per_w, (kf, per_f, per_w)


# VALU issue time of a kernel: its wave64 VALU instructions at 4 cycles each (16 lanes per SIMD), over every
# SIMD of the chip (256 compute units x 4) at the peak engine clock, against its run time
SIMDS = 256 * 4
CLOCK_HZ = 2.4e9
CYCLES_PER_VALU = 4


def summarise(run, workload, cal, out_dir, cmds):
    res = json.load(open(os.path.join(run, f"{workload}.json")))
    K = len(res["timed_steps"])
    units = {"interfacial_faces": res["interfacial_faces_per_step"] * K,
             "interfacial_cells": res["interfacial_cells_per_step"] * K,
             "faces": res["faces_per_step"] * K, "cells": res["cells_per_step"] * K}
    times = kernel_times(os.path.join(run, f"{workload}_trace"))
    fe, _ = counters(os.path.join(run, f"{workload}_fetch"))
    wr, _ = counters(os.path.join(run, f"{workload}_write"))
    fp, fpn = counters(os.path.join(run, f"{workload}_fp64"))
    # the step's kernels: the library's, launched at least once per timed step (not the set-up kernels of the
    # run, nor the copies that restore the saved fractions before each step)
    times = {k: v for k, v in times.items() if k.startswith("k_") and v[0] >= K}
    step_ns = sum(v[1] for v in times.values())
    table = {}
    rows = []
    for k, (n, ns) in sorted(times.items(), key=lambda kv: -kv[1][1]):
        c = fp.get(k, {})
        issued = 64.0 * (c.get("SQ_INSTS_VALU_ADD_F64", 0) + c.get("SQ_INSTS_VALU_MUL_F64", 0)
                         + c.get("SQ_INSTS_VALU_TRANS_F64", 0) + 2 * c.get("SQ_INSTS_VALU_FMA_F64", 0))
        act = c.get("SQ_ACTIVE_INST_VALU", 0.0)
        lanes = c.get("SQ_THREAD_CYCLES_VALU", 0.0) / (64.0 * act) if act > 0 else 0.0
        fp64_share = ((c.get("SQ_INSTS_VALU_ADD_F64", 0) + c.get("SQ_INSTS_VALU_MUL_F64", 0)
                       + c.get("SQ_INSTS_VALU_TRANS_F64", 0) + c.get("SQ_INSTS_VALU_FMA_F64", 0))
                      / c["SQ_INSTS_VALU"]) if c.get("SQ_INSTS_VALU") else 0.0
        live = issued * lanes
        hbm = fe.get(k, {}).get("FETCH_SIZE", 0.0) * cal[0] + wr.get(k, {}).get("WRITE_SIZE", 0.0) * cal[1]
        sec = ns * 1e-9
        valu_issue = CYCLES_PER_VALU * c.get("SQ_INSTS_VALU", 0.0) / (SIMDS * CLOCK_HZ) / sec if sec else 0.0
        row = dict(kernel=k, launches=n, avg_us=ns / n / 1e3, share=ns / step_ns, fp64_issued=issued / n,
                   active_lanes=lanes, fp64_live=live / n, fp64_share=fp64_share, hbm_bytes=hbm / n,
                   tflops_live=live / sec / 1e12 if sec else 0.0, gbs=hbm / sec / 1e9 if sec else 0.0,
                   valu_issue=valu_issue)
        rows.append(row)
        u = UNIT.get(k)
        if u and units[u] > 0:
            table[k] = {"unit": u, "flops": live / units[u], "flops_issued": issued / units[u],
                        "bytes": hbm / units[u], "traffic": hbm / n, "avg_launch_ms": ns / n / 1e6,
                        "units_per_launch": units[u] / n, "active_lanes": lanes, "valu_issue_frac": valu_issue,
                        "source": f"profiles/counters_{workload}.md"}
    name = f"counters_{workload}.md"
    with open(os.path.join(out_dir, name), "w") as f:
        f.write(f"# Kernel times and counters: {res['workload']}\n\n")
        f.write("Commands (from the repository root, on one MI355X; STATES written by the first):\n\n```\n")
        f.write("\n".join(c.replace("{W}", workload) for c in cmds) + "\n```\n\n")
        f.write(f"Timed steps {res['timed_steps'][0]}..{res['timed_steps'][-1]} ({K} steps, spread evenly over the "
                f"trajectory); per step {res['interfacial_faces_per_step']:.1f} faces needing a flux polyhedron, "
                f"{res['interfacial_cells_per_step']:.1f} interface cells, {res['faces_per_step']:.0f} faces; "
                f"the timed-only run measured {res['ms_per_step']:.4f} ms per step with HIP events.\n\n")
        f.write(f"HBM calibration: a plain copy of {cal[2][0]} reads FETCH_SIZE {cal[2][1]:.1f} KiB and writes "
                f"WRITE_SIZE {cal[2][2]:.1f} KiB per launch for its bytes, so HBM bytes = FETCH_SIZE x {cal[0]:.1f} "
                f"+ WRITE_SIZE x {cal[1]:.1f}.\n\n")
        f.write("| kernel | launches | avg µs | share of step | FP64 lane FLOPs issued / launch | active lanes | "
                "FP64 FLOPs of active lanes / launch | FP64 share of VALU | TFLOP/s (active) | HBM bytes / launch "
                "| GB/s | VALU issue time / kernel time |\n|---|---|---|---|---|---|---|---|---|---|---|---|\n")
        for r in rows:
            f.write(f"| {r['kernel']} | {r['launches']} | {r['avg_us']:.2f} | {r['share']:.3f} | "
                    f"{r['fp64_issued']:.4g} | {r['active_lanes']:.3f} | {r['fp64_live']:.4g} | "
                    f"{r['fp64_share']:.2f} | {r['tflops_live']:.2f} | {r['hbm_bytes']:.4g} | {r['gbs']:.0f} | "
                    f"{r['valu_issue']:.2f} |\n")
        f.write("\nWork per unit (what bench.py's rooflines use): FP64 FLOPs of active lanes and HBM bytes per "
                "unit of the kernel's work.\n\n| kernel | unit | FLOPs / unit | issued FLOPs / unit | HBM bytes / "
                "unit |\n|---|---|---|---|---|\n")
        for k, v in table.items():
            f.write(f"| {k} | {v['unit']} | {v['flops']:.1f} | {v['flops_issued']:.1f} | {v['bytes']:.1f} |\n")
    return table


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("run")
    ap.add_argument("--copy-mib", type=int, default=1024)
    ap.add_argument("--out", default="profiles")
    ap.add_argument("--cmds", default=None, help="text file: the commands of the run, {W} for the workload")
    a = ap.parse_args()
    cmds = open(a.cmds).read().strip().splitlines() if a.cmds else []
    cal = calibration(a.run, a.copy_mib)
    table = {}
    names = sorted(f[:-5] for f in os.listdir(a.run)
                   if f.endswith(".json") and os.path.isdir(os.path.join(a.run, f[:-5] + "_trace")))
    for w in names:
        table[w] = summarise(a.run, w, cal, a.out, cmds)
    table["sources_digest"] = sources_digest()
    path = os.path.join(a.out, "work_per_unit.json")
    with open(path, "w") as f:
        json.dump(table, f, indent=1, sort_keys=True)
    print("wrote", path, {w: sorted(t) for w, t in table.items() if isinstance(t, dict)})


if __name__ == "__main__":
    main()
