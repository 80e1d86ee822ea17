"""The profile summary (rocprofv3 CSVs -> work per unit) on synthetic counter
files: kernel names map to the library's timing slots, only the step's
kernels count, the HBM calibration and the active-lane FLOPs follow their
definitions, and bench.py's roofline recomputes from the table."""
from __future__ import annotations

import csv
import json
import os

import pytest

from paper_2111_01524_amd import profile_summary as PS

K = 4
KERNELS = [("void gvof::k_flux_prep<32, 0>(gvof::DevMesh, double const*, double)", 200_000),
           ("gvof::k_flux_gen_runs(gvof::DevMesh)", 2_000_000), ("gvof::k_face_sweep(gvof::DevMesh)", 60_000)]


def _csv(path, rows):
    os.makedirs(os.path.dirname(path), exist_ok=True)
    with open(path, "w", newline="") as f:
        w = csv.DictWriter(f, fieldnames=list(rows[0]))
        w.writeheader()
        w.writerows(rows)


def _pmc(path, counters):
    rows, d = [], 0
    for _ in range(K):
        for k, _ in KERNELS:
            d += 1
            rows += [{"Dispatch_Id": d, "Kernel_Name": k, "Counter_Name": c, "Counter_Value": v} for c, v in counters.items()]
    _csv(path, rows)


@pytest.fixture()
def run(tmp_path):
    r = tmp_path / "run"
    rows = [{"Kernel_Name": k, "Start_Timestamp": 0, "End_Timestamp": ns} for _ in range(K) for k, ns in KERNELS]
    rows += [{"Kernel_Name": "gvof::k_face_geom(gvof::DevMesh)", "Start_Timestamp": 0, "End_Timestamp": 99_999},
             {"Kernel_Name": "__amd_rocclr_copyBuffer", "Start_Timestamp": 0, "End_Timestamp": 10}]
    _csv(str(r / "jittered_trace" / "p_kernel_trace.csv"), rows)
    _pmc(str(r / "jittered_fetch" / "p_counter_collection.csv"), {"FETCH_SIZE": 1000})
    _pmc(str(r / "jittered_write" / "p_counter_collection.csv"), {"WRITE_SIZE": 500})
    _pmc(str(r / "jittered_fp64" / "p_counter_collection.csv"),
         {"SQ_INSTS_VALU_ADD_F64": 10, "SQ_INSTS_VALU_MUL_F64": 10, "SQ_INSTS_VALU_FMA_F64": 20,
          "SQ_INSTS_VALU_TRANS_F64": 1, "SQ_INSTS_VALU": 100, "SQ_ACTIVE_INST_VALU": 100,
          "SQ_THREAD_CYCLES_VALU": 3200, "SQ_WAVES": 5})
    for n, c, v in (("copy_fetch", "FETCH_SIZE", 524288), ("copy_write", "WRITE_SIZE", 1048576)):
        _csv(str(r / n / "p_counter_collection.csv"),
             [{"Dispatch_Id": 1, "Kernel_Name": "__amd_rocclr_copyBuffer", "Counter_Name": c, "Counter_Value": v}])
    (r / "jittered.json").write_text(json.dumps(
        {"workload": "jittered 64^3", "name": "jittered", "ms_per_step": 2.3, "timed_steps": [1, 2, 3, 4],
         "interfacial_faces_per_step": 50000, "interfacial_cells_per_step": 2000, "faces_per_step": 3194880,
         "cells_per_step": 262144}))
    return str(r)


def test_summary_counts_and_definitions(run, tmp_path):
    out = tmp_path / "out"
    out.mkdir()
    cal = PS.calibration(run, 1024)
    assert cal[0] == pytest.approx(2048.0) and cal[1] == pytest.approx(1024.0)  # bytes per KiB of each counter
    t = PS.summarise(run, "jittered", cal, str(out), ["bench.py --workload {W}"])
    assert set(t) == {"k_flux_prep", "k_flux_gen_filter", "k_face_sweep"}  # the run filter maps to its slot
    e = t["k_flux_gen_filter"]
    issued = 64 * (10 + 10 + 1 + 2 * 20)
    assert e["flops_issued"] * 50000 * K == pytest.approx(issued * K)
    assert e["active_lanes"] == pytest.approx(0.5)
    assert e["flops"] == pytest.approx(0.5 * e["flops_issued"])
    assert e["traffic"] == pytest.approx(1000 * 2048.0 + 500 * 1024.0)
    assert e["unit"] == "interfacial_faces" and t["k_face_sweep"]["unit"] == "faces"
    assert e["avg_launch_ms"] == pytest.approx(2.0)
    # 100 VALU instructions a launch at 4 cycles over 1024 SIMDs at 2.4 GHz, against 2 ms a launch
    assert e["valu_issue_frac"] == pytest.approx(4 * 100 / (1024 * 2.4e9) / 2e-3)
    text = (out / "counters_jittered.md").read_text()
    rows = [ln.split("|")[1].strip() for ln in text.splitlines() if ln.startswith("| ")]
    assert "k_face_geom" not in rows and "__amd_rocclr_copyBuffer" not in rows  # set-up kernels, state copies
    assert "bench.py --workload jittered" in text


def test_bench_roofline_recomputes_from_the_table(run, tmp_path):
    import importlib.util
    spec = importlib.util.spec_from_file_location("bench", os.path.join(os.path.dirname(__file__), "..", "bench.py"))
    bench = importlib.util.module_from_spec(spec)
    spec.loader.exec_module(bench)
    out = tmp_path / "out"
    out.mkdir()
    t = PS.summarise(run, "jittered", PS.calibration(run, 1024), str(out), [])
    table = {"jittered": t, "sources_digest": PS.sources_digest()}
    # the bench's own per-kernel times and units over its timed steps
    kt = {"k_flux_gen_filter": (2.0, K), "k_flux_prep": (0.2, K), "k_face_sweep": (0.06, K)}
    counts = {"steps": K, "interfacial_faces": 50000 * K, "interfacial_cells": 2000 * K, "faces": 3194880 * K,
              "cells": 262144 * K}
    rl = bench.rooflines(kt, 2.26, counts, table, "jittered")
    assert [r["kernel"] for r in rl] == ["k_flux_gen_filter"]  # only kernels taking 10% of the step or more
    r = rl[0]
    assert r["bound"] == "alu" and r["unit"] == "TFLOP/s"
    assert r["achieved"] == pytest.approx(t["k_flux_gen_filter"]["flops"] * 50000 * K / (2.0 * K * 1e-3) / 1e12)
    assert r["frac"] == pytest.approx(r["achieved"] / 78.6)
    assert r["traffic"] == pytest.approx(t["k_flux_gen_filter"]["traffic"])
    assert r["profile_valu_issue_frac"] == pytest.approx(t["k_flux_gen_filter"]["valu_issue_frac"])
    table["sources_digest"] = "stale"
    assert bench.rooflines(kt, 2.26, counts, table, "jittered")[0]["traffic"] is None
