"""Parity at the full 64^3 sizes of the measured workloads: every cell and
every face is compared with the oracle, teacher-forced from a common state.

  - 64^3 Cartesian, Enright field with period 3, CFL 0.5: the first two steps
    and step 100 (the oracle runs the trajectory up to there);
  - 64^3 distorted (+-0.25h, seed 1), same field: the first two steps, with
    FMFPA, EMFPA and NMFPA flux polyhedra, and with LSFIR, LLCIR, ELCIR and
    CLCIR normals (library default launch shapes);
  - 64^3 distorted with LSGIR + FMFPA in the middle of the trajectory, where
    the interface is most stretched: the HIP path runs free to the middle
    step, then both sides step from that state, the HIP path under the launch
    shapes the autotuner picks there (what bench.py times), under the
    defaults, and under staging limits that send faces and pairs to the
    overflow and deferred kernels.

Bars as in the small-size parity tests: tags and upwind cells bit for bit,
V_d bit for bit, |dV_F| <= 1e-12 V, |dF| <= 1e-12 per cell.
"""
from __future__ import annotations

import numpy as np
import pytest

from paper_2111_01524_amd import inputs
from tests.gpu_common import host, log, max_abs, to_dev, torch_dev

pytestmark = pytest.mark.gpu

SPHERE = [0.35, 0.35, 0.35, 0.15]


def _step_parity(oracle_mod, g, om, F, uf, uv, ufd, uvd, dts, V, torch, dev, label):
    Fd = to_dev(torch, dev, F)
    g.reconstruct(Fd)
    T = {k: host(v) for k, v in g.tags().items()}
    Fc, Fs, tn, tf, tc, pl = om.reconstruct(F)
    assert np.array_equal(T["cell"], tc) and np.array_equal(T["face"], tf) and np.array_equal(T["node"], tn)
    assert np.array_equal(host(Fd), Fc)
    Fout = torch.empty_like(Fd)
    up_g, vd_g, vf_g = g.advect_step(ufd, uvd, dts, Fd, Fout, want_faces=True)
    F1, Vd, VF, up, bad = om.advect(pl, tc, tf, uf, uv, dts, Fc)
    g.status()
    assert bad == 0
    assert np.array_equal(host(vd_g), Vd)
    assert np.array_equal(host(up_g), up)
    dVF = float(np.abs(host(vf_g) - VF).max() / V.max())
    dF = max_abs(host(Fout), F1)
    log(f"{label}: tag-0 cells {(tc == 0).sum()} faces {(tf == 0).sum()} max|dVF|/V={dVF:.2e} max|dF|={dF:.2e}")
    assert dVF <= 1e-12 and dF <= 1e-12
    return F1


@pytest.mark.parametrize("kind,later,method,recon", [("cartesian", 100, "fmfpa", "lsgir"),
                                                      ("jittered", None, "fmfpa", "lsgir"),
                                                      ("jittered", None, "emfpa", "lsgir"),
                                                      ("jittered", None, "nmfpa", "lsgir"),
                                                      ("jittered", None, "fmfpa", "lsfir"),
                                                      ("jittered", None, "fmfpa", "llcir"),
                                                      ("jittered", None, "fmfpa", "elcir"),
                                                      ("jittered", None, "fmfpa", "clcir")])
def test_full_size_parity(oracle_mod, kind, later, method, recon):
    from paper_2111_01524_amd import gvof
    torch, dev = torch_dev()
    m = inputs.cartesian_mesh(64) if kind == "cartesian" else inputs.jittered_mesh(64, seed=1)
    log(f"full size {kind} 64^3 {method} {recon}: faces {m.nf} cells {m.nc}")
    om = oracle_mod.OracleMesh(m, method=method, recon=recon)
    g = gvof.GvofMesh(m, dev, method=method, recon=recon)
    uf, uv = inputs.velocity_enright(m)
    dt = inputs.cfl_dt(m, np.abs(uf).max(axis=1), 0.5)
    sched = inputs.step_schedule(3.0, dt)
    ufd, uvd = to_dev(torch, dev, uf), to_dev(torch, dev, uv)
    V = om.geometry()["V"]
    ndiv = 10 if kind == "cartesian" else 4
    F = om.init_fraction("sphere", SPHERE, ndiv)
    Fg = host(g.init_fraction("sphere", SPHERE, ndiv))
    assert max_abs(Fg, F) <= 1e-12
    t = 0.0

    def dteff(s, t):
        return sched[s] * inputs.enright_time_factor(t + 0.5 * sched[s], 3.0)

    for s in range(2):
        F = _step_parity(oracle_mod, g, om, F, uf, uv, ufd, uvd, dteff(s, t), V, torch, dev, f"{kind} step {s}")
        t += sched[s]
    if later:
        for s in range(2, later):
            Fc, Fs, tn, tf, tc, pl = om.reconstruct(F)
            F, *_ = om.advect(pl, tc, tf, uf, uv, dteff(s, t), Fc)
            t += sched[s]
        _step_parity(oracle_mod, g, om, F, uf, uv, ufd, uvd, dteff(later, t), V, torch, dev, f"{kind} step {later}")


def test_full_size_distorted_mid_trajectory_launch_shapes(oracle_mod):
    """64^3 distorted, LSGIR + FMFPA: one step from the HIP path's own state at
    the middle of the trajectory, compared with the oracle's step from the
    same state, under the autotuned shapes, the defaults and forced staging
    overflows (faces and pairs that do not fit are computed by the overflow
    and deferred kernels, which must give the same values)."""
    from paper_2111_01524_amd import gvof
    torch, dev = torch_dev()
    m = inputs.jittered_mesh(64, seed=1)
    om = oracle_mod.OracleMesh(m)
    g = gvof.GvofMesh(m, dev)
    uf, uv = inputs.velocity_enright(m)
    dt = inputs.cfl_dt(m, np.abs(uf).max(axis=1), 0.5)
    sched = inputs.step_schedule(3.0, dt)
    times = np.concatenate([[0.0], np.cumsum(sched)])
    dteff = [sched[s] * inputs.enright_time_factor(times[s] + 0.5 * sched[s], 3.0) for s in range(len(sched))]
    ufd, uvd = to_dev(torch, dev, uf), to_dev(torch, dev, uv)
    V = om.geometry()["V"]
    F = g.init_fraction("sphere", SPHERE, 10)
    Fn = torch.empty_like(F)
    s_mid = len(sched) // 2
    for s in range(s_mid):
        g.reconstruct(F)
        g.advect_step(ufd, uvd, dteff[s], F, Fn)
        F, Fn = Fn, F
    g.status()
    F_mid = host(F)
    log(f"distorted 64^3 free run to step {s_mid}")
    dtm = to_dev(torch, dev, np.array([dteff[s_mid]]))
    act = to_dev(torch, dev, np.ones(1, np.uint8))
    cfg, ms = gvof.gvof_autotune(g.h, ufd, uvd, dtm, act, F, Fn, 2)
    tuned = cfg.as_dict()
    log(f"autotuned at step {s_mid}: {tuned} ({ms:.3f} ms/step)")
    assert np.array_equal(host(F), F_mid), "autotune must leave F unchanged"
    Fc, Fs, tn, tf, tc, pl = om.reconstruct(F_mid)
    F1, Vd, VF, up, bad = om.advect(pl, tc, tf, uf, uv, dteff[s_mid], Fc)
    assert bad == 0
    log(f"oracle step {s_mid}: tag-0 cells {(tc == 0).sum()} faces {(tf == 0).sum()}")
    default = gvof.gvof_launch_config(256, 128, 16384, 16, 32, 0, 0, 64, 4).as_dict()
    shapes = [("autotuned", tuned), ("defaults", default),
              ("staging limits", dict(tuned, staged_faces=20000, staged_pairs=256 * 2000)),
              ("tight pair buffer", dict(default, staged_pairs=256 * 200, filter_lanes=16, prep_lanes=32)),
              ("runs filter", dict(default, filter_lanes=0)), ("per-pair filter, 8 lanes", dict(tuned, filter_lanes=8)),
              ("the other unit ranking window", dict(tuned, units_rank=12 - tuned["units_rank"]))]
    first = None
    for name, cfgd in shapes:
        gvof.gvof_set_launch_config(g.h, gvof.gvof_launch_config(**cfgd))
        Fd = to_dev(torch, dev, F_mid)
        g.reconstruct(Fd)
        T = {k: host(v) for k, v in g.tags().items()}
        assert np.array_equal(T["cell"], tc) and np.array_equal(T["face"], tf)
        assert np.array_equal(host(Fd), Fc)
        Fout = torch.empty_like(Fd)
        up_g, vd_g, vf_g = g.advect_step(ufd, uvd, dteff[s_mid], Fd, Fout, want_faces=True)
        g.status()
        assert np.array_equal(host(vd_g), Vd) and np.array_equal(host(up_g), up)
        dVF = float(np.abs(host(vf_g) - VF).max() / V.max())
        dF = max_abs(host(Fout), F1)
        log(f"  {name} {cfgd}: max|dVF|/V={dVF:.2e} max|dF|={dF:.2e}")
        assert dVF <= 1e-12 and dF <= 1e-12
        # every shape (and so every filter and overflow path) gives the same values, bit for bit
        if first is None:
            first = (host(vf_g), host(Fout))
        else:
            assert np.array_equal(host(vf_g), first[0]) and np.array_equal(host(Fout), first[1]), name
