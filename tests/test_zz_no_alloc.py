"""gvof_advect_step_static, the advection step whose staging lives in the
library's static device array (for callers that cannot allocate), against
gvof_advect_step on the same reconstructed state, through the C interface.

Both calls must give the same bits: V_d, upwind cells, V_F and F.  Two calls
in a row share the array, the second on a smaller mesh; the first is a 64^3
distorted grid in mid-deformation, whose staging does not fit the array, so
most of its faces and pairs go to the overflow and deferred kernels.  A mesh
whose overflow list does not fit is rejected before anything runs.
"""
from __future__ import annotations

import numpy as np
import pytest

from paper_2111_01524_amd import inputs
from tests.gpu_common import host, log, to_dev, torch_dev

pytestmark = pytest.mark.gpu

SPHERE = [0.35, 0.35, 0.35, 0.15]


def _state(g, m, steps, torch, dev):
    """Mesh inputs and the HIP path's own state after `steps` free steps."""
    uf, uv = inputs.velocity_enright(m)
    dt = inputs.cfl_dt(m, np.abs(uf).max(axis=1), 0.5)
    ufd, uvd = to_dev(torch, dev, uf), to_dev(torch, dev, uv)
    F = g.init_fraction("sphere", SPHERE, 6)
    Fn = torch.empty_like(F)
    for s in range(steps):
        g.reconstruct(F)
        g.advect_step(ufd, uvd, dt * inputs.enright_time_factor((s + 0.5) * dt, 3.0), F, Fn)
        F, Fn = Fn, F
    return ufd, uvd, dt * inputs.enright_time_factor((steps + 0.5) * dt, 3.0), F


def _compare(gv, g, ufd, uvd, dt, F, torch, label):
    g.reconstruct(F)
    outs = []
    for fn in (gv.gvof_advect_step, gv.gvof_advect_step_static):
        up = torch.zeros(g.nf, dtype=torch.int32, device=F.device)
        vd = torch.zeros(g.nf, dtype=torch.float64, device=F.device)
        vf = torch.zeros(g.nf, dtype=torch.float64, device=F.device)
        Fo = torch.empty_like(F)
        fn(g.h, ufd, uvd, dt, F, Fo, up, vd, vf)
        g.status()
        outs.append([host(x) for x in (up, vd, vf, Fo)])
    nfaces = g.interface_counts()[1]
    for name, a, b in zip(("upwind", "V_d", "V_F", "F"), outs[0], outs[1]):
        assert np.array_equal(a, b), (label, name, float(np.abs(a.astype(float) - b).max()))
    log(f"{label}: {nfaces} faces with flux polyhedra, static staging equal bit for bit")


def test_static_staging_equals_workspace_staging():
    from paper_2111_01524_amd import gvof as gv
    torch, dev = torch_dev()
    big = inputs.jittered_mesh(64, seed=1)
    g = gv.GvofMesh(big, dev)
    ufd, uvd, dt, F = _state(g, big, 150, torch, dev)
    _compare(gv, g, ufd, uvd, dt, F, torch, "distorted 64^3, step 150")
    # the same step with the staging limited further by the launch shapes
    cfg = gv.gvof_get_launch_config(g.h).as_dict()
    gv.gvof_set_launch_config(g.h, gv.gvof_launch_config(**dict(cfg, staged_faces=300, staged_pairs=256 * 40)))
    _compare(gv, g, ufd, uvd, dt, F, torch, "distorted 64^3, step 150, staging limited")
    del g, F, ufd, uvd
    small = inputs.cartesian_mesh(24)
    g2 = gv.GvofMesh(small, dev)
    ufd, uvd, dt, F = _state(g2, small, 40, torch, dev)
    _compare(gv, g2, ufd, uvd, dt, F, torch, "Cartesian 24^3, step 40 (second call, smaller)")
    # and back to a step of the first kind of mesh, small this time
    mid = inputs.jittered_mesh(12, seed=3)
    g3 = gv.GvofMesh(mid, dev, method="emfpa")
    ufd, uvd, dt, F = _state(g3, mid, 5, torch, dev)
    _compare(gv, g3, ufd, uvd, dt, F, torch, "distorted 12^3 EMFPA, step 5")


def test_static_staging_rejects_a_mesh_beyond_its_size():
    from paper_2111_01524_amd import gvof as gv
    torch, dev = torch_dev()
    m = inputs.jittered_mesh(66, seed=1)
    g = gv.GvofMesh(m, dev)
    ufd, uvd, dt, F = _state(g, m, 0, torch, dev)
    g.reconstruct(F)
    Fo = torch.empty_like(F)
    with pytest.raises(gv.GvofError) as e:
        gv.gvof_advect_step_static(g.h, ufd, uvd, dt, F, Fo)
    assert e.value.code == gv.GVOF_E_LIMIT and "static staging" in str(e.value)
    log(f"{m.nf} faces rejected: {e.value}")
    g.advect_step(ufd, uvd, dt, F, Fo)  # the workspace path takes it
    g.status()
