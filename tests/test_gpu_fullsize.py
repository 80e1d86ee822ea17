"""Parity at the full 64^3 sizes of the measured workloads, in the launch
configuration bench.py times (the library defaults): every cell and every
face is compared with the oracle, teacher-forced from the oracle's state.

  - 64^3 Cartesian, Enright field with period 3, CFL 0.5: the first two steps
    and step 100 (the oracle runs the trajectory up to there);
  - 64^3 distorted (+-0.25h, seed 1), same field: the first two steps, with
    FMFPA, EMFPA and NMFPA flux polyhedra, and with LSFIR and CLCIR normals.

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
