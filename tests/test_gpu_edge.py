"""Edge cases of the step on the GPU, through the C interface, against the oracle.

  - general cells bounded by non-planar quadrilaterals (fanned from their
    vertex mean: the polygon paths of the truncation and of the plane
    constant, which the triangulated grid does not reach), with every flux
    polyhedron method and with the LSFIR, LLCIR and CLCIR normals (saddle
    quadrilateral faces send cells back to LSGIR);
  - the smallest meshes (1^3 and 2^3: every cell touches the boundary; a
    single cell has no neighbour for LSFIR's fit or CLCIR's ring);
  - an empty field (no interface: nothing changes, bit for bit);
  - a zero time step (no flux: F after the step equals F after the cut-off to rounding);
  - velocity reversed (negative time step);
  - a ragged batch with a one-cell problem, equal to its problems alone.
"""
from __future__ import annotations

import numpy as np
import pytest

from paper_2111_01524_amd import inputs
from tests.gpu_common import host, log, max_abs, to_dev, torch_dev

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def gv():
    from paper_2111_01524_amd import gvof
    gvof.lib()
    return gvof


def _parity_steps(oracle_mod, gv, m, uf, uv, dts, F, label, method="fmfpa", recon="lsgir"):
    torch, dev = torch_dev()
    om = oracle_mod.OracleMesh(m, method=method, recon=recon, lsfir_outer=2)
    g = gv.GvofMesh(m, dev, method=method, recon=recon, lsfir_outer=2)
    label = f"{label} {method} {recon}"
    ufd, uvd = to_dev(torch, dev, uf), to_dev(torch, dev, uv)
    V = om.geometry()["V"]
    for s, dt in enumerate(dts):
        Fd = to_dev(torch, dev, F)
        tags, planes = g.reconstruct(Fd, want_tags=True, want_planes=True)
        Fc, Fs, tn, tf, tc, pl = om.reconstruct(F)
        assert np.array_equal(host(tags), tc) and np.array_equal(host(Fd), Fc)
        sel = tc == 0
        dpl = float(np.abs(host(planes)[:, sel] - pl[:, sel]).max()) if sel.any() else 0.0
        log(f"{label} step {s}: max|d plane| = {dpl:.2e}")
        # LSFIR with the section's weight |d|^-2.5 amplifies rounding: on this mesh
        # the oracle's own normals move by 1.5e-12 under 4e-16 relative noise in F,
        # so its planes are not held to 1e-12 here (measured up to 7.7e-12); the
        # fractions below are, as for every reconstruction
        if recon != "lsfir":
            assert dpl <= 1e-12
        Fout = torch.empty_like(Fd)
        up_g, vd_g, vf_g = g.advect_step(ufd, uvd, dt, Fd, Fout, want_faces=True)
        F1, Vd, VF, up, bad = om.advect(pl, tc, tf, uf, uv, dt, Fc)
        g.status()
        assert bad == 0
        assert np.array_equal(host(vd_g), Vd) and np.array_equal(host(up_g), up)
        dVF = float(np.abs(host(vf_g) - VF).max() / V.max())
        dF = max_abs(host(Fout), F1)
        log(f"{label} step {s}: tag-0 cells {int(sel.sum())} faces {int((tf == 0).sum())} dVF/V={dVF:.2e} dF={dF:.2e}")
        assert dVF <= 1e-12 and dF <= 1e-12
        F = F1
    return F


@pytest.mark.parametrize("method,recon", [("fmfpa", "lsgir"), ("emfpa", "lsgir"), ("nmfpa", "lsgir"),
                                          ("fmfpa", "lsfir"), ("fmfpa", "llcir"), ("fmfpa", "clcir")])
def test_polygon_face_general_cells(oracle_mod, gv, method, recon):
    m = inputs.jittered_mesh(7, seed=3, split=False)
    assert m.fv_ptr[1] == 4
    uf, uv = inputs.velocity_enright(m)
    dt = inputs.cfl_dt(m, np.abs(uf).max(axis=1), 0.5)
    F = oracle_mod.OracleMesh(m).init_fraction("sphere", [0.45, 0.5, 0.52, 0.27], 4)
    _parity_steps(oracle_mod, gv, m, uf, uv, [dt, dt, -dt], F, "quad-faced distorted 7^3", method, recon)


@pytest.mark.parametrize("kind,n,method,recon", [("cartesian", 1, "fmfpa", "lsgir"), ("cartesian", 2, "fmfpa", "lsgir"),
                                                 ("jittered", 2, "fmfpa", "lsgir"), ("cartesian", 1, "emfpa", "lsgir"),
                                                 ("jittered", 2, "emfpa", "lsgir"), ("jittered", 2, "nmfpa", "lsgir"),
                                                 ("cartesian", 1, "fmfpa", "lsfir"), ("jittered", 2, "fmfpa", "lsfir"),
                                                 ("cartesian", 1, "fmfpa", "clcir"), ("jittered", 2, "fmfpa", "clcir")])
def test_smallest_meshes(oracle_mod, gv, kind, n, method, recon):
    m = inputs.cartesian_mesh(n) if kind == "cartesian" else inputs.jittered_mesh(n, seed=5)
    uf, uv = inputs.velocity_uniform(m, (0.3, 0.2, 0.1))
    dt = inputs.cfl_dt(m, np.abs(uf).max(axis=1), 0.5)
    F = oracle_mod.OracleMesh(m).init_fraction("sphere", [0.4, 0.45, 0.5, 0.3], 6)
    _parity_steps(oracle_mod, gv, m, uf, uv, [dt, dt], F, f"{kind} {n}^3", method, recon)


def test_empty_field_and_zero_step(oracle_mod, gv):
    torch, dev = torch_dev()
    m = inputs.jittered_mesh(6, seed=2)
    uf, uv = inputs.velocity_enright(m)
    dt = inputs.cfl_dt(m, np.abs(uf).max(axis=1), 0.5)
    g = gv.GvofMesh(m, dev)
    ufd, uvd = to_dev(torch, dev, uf), to_dev(torch, dev, uv)
    # empty: no interfacial cell or face, F stays exactly zero
    F = torch.zeros(m.nc, dtype=torch.float64, device=dev)
    g.reconstruct(F)
    g.advect_step(ufd, uvd, dt, F, F)
    assert g.interface_counts() == (0, 0)
    assert not host(F).any()
    # zero step: V_d = 0 exactly, V_F = 0 and F unchanged to rounding (the
    # collapsed flux polyhedra have rounding-level volumes), as in the oracle
    om = oracle_mod.OracleMesh(m)
    F0 = om.init_fraction("sphere", [0.5, 0.5, 0.5, 0.3], 4)
    V = om.geometry()["V"]
    Fd = to_dev(torch, dev, F0)
    g.reconstruct(Fd)
    Fcut = host(Fd)
    up, vd, vf = g.advect_step(ufd, uvd, 0.0, Fd, Fd, want_faces=True)
    assert not host(vd).any()
    assert np.abs(host(vf)).max() <= 1e-15 * V.min()
    assert max_abs(host(Fd), Fcut) <= 1e-14
    g.status()


def test_ragged_batch_with_one_cell_problem(gv):
    torch, dev = torch_dev()
    specs = [dict(side=1, kind="cartesian", radius=0.3, center=(0.5, 0.5, 0.5), period=2.0, jitter_seed=1),
             dict(side=2, kind="jittered", radius=0.3, center=(0.4, 0.5, 0.5), period=2.0, jitter_seed=2),
             dict(side=5, kind="cartesian", radius=0.2, center=(0.45, 0.5, 0.55), period=2.0, jitter_seed=3)]
    P = [inputs.problem_inputs(s) for s in specs]
    for p in P:  # uniform velocity: the deformation field vanishes on every face of a 1^3 grid
        p["uf"], p["uv"] = inputs.velocity_uniform(p["mesh"], (0.3, -0.2, 0.1))
        dt = inputs.cfl_dt(p["mesh"], np.abs(p["uf"]).max(axis=1), 0.5)
        p["dt_eff"] = np.full(3, dt)
    B = gv.GvofBatch([p["mesh"] for p in P], dev)
    uf = to_dev(torch, dev, inputs.concat_soa([p["uf"] for p in P]))
    uv = to_dev(torch, dev, inputs.concat_soa([p["uv"] for p in P]))
    F = B.init_fraction_each([p["shape"] for p in P], 6)
    F0 = host(F)
    act = to_dev(torch, dev, np.ones(len(P), np.uint8))
    for s in range(3):
        B.step(uf, uv, to_dev(torch, dev, np.array([p["dt_eff"][s] for p in P])), act, F)
    Fb = host(F)
    B.status()
    for q, p in enumerate(P):
        g = gv.GvofMesh(p["mesh"], dev)
        Fa = to_dev(torch, dev, F0[B.cells(q)])
        ufa, uva = to_dev(torch, dev, p["uf"]), to_dev(torch, dev, p["uv"])
        for s in range(3):
            g.reconstruct(Fa)
            g.advect_step(ufa, uva, p["dt_eff"][s], Fa, Fa)
        assert np.array_equal(Fb[B.cells(q)], host(Fa)), q
