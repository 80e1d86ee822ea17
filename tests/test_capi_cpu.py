"""The C-ABI library without a GPU: it loads, exports every declared symbol,
and its host-side mesh validation / topology calls behave (no device work)."""
import ctypes as C
import os
import re

import numpy as np
import pytest

from paper_2111_01524_amd import gvof, inputs

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


def declared_functions():
    txt = open(os.path.join(ROOT, "include", "gvof.h")).read()
    txt = re.sub(r"/\*.*?\*/", "", txt, flags=re.S)
    return sorted(set(re.findall(r"\b(gvof_[a-z_]+)\s*\(", txt)))


def test_library_exports_every_declared_symbol():
    lib = gvof.lib()
    names = declared_functions()
    assert len(names) >= 14
    for n in names:
        assert hasattr(lib, n), n
    assert sorted(gvof.exported_symbols()) == names


def test_params_default():
    p = gvof.gvof_params_default()
    assert p.eps == 1e-12 and p.beta == 1.5 and p.fmfpa_degen == 1e-12


def test_mesh_create_topology_and_workspace():
    m = inputs.cartesian_mesh(4)
    h = gvof.gvof_mesh_create(*m.arrays(), m.nc)
    try:
        nv, nf, nc, maxnb = gvof.gvof_mesh_sizes(h)
        assert (nv, nf, nc) == (m.nv, m.nf, m.nc)
        assert maxnb == 26
        ws = gvof.gvof_mesh_workspace_bytes(h)
        assert ws > 8 * (3 * nv + 6 * nf + 10 * nc)
    finally:
        gvof.gvof_mesh_destroy(h)


@pytest.mark.parametrize("breaker,code", [
    (lambda a: a["owner"].__setitem__(0, 10 ** 6), gvof.GVOF_E_MESH),
    (lambda a: a["neigh"].__setitem__(a["owner"].shape[0] // 2, int(a["owner"][a["owner"].shape[0] // 2])), gvof.GVOF_E_MESH),
    (lambda a: a["fv_idx"].__setitem__(3, -5), gvof.GVOF_E_MESH),
    (lambda a: a["vx"].__setitem__(2, np.nan), gvof.GVOF_E_MESH),
])
def test_mesh_create_rejects_bad_meshes(breaker, code):
    m = inputs.cartesian_mesh(3)
    a = dict(vx=m.vx.copy(), vy=m.vy.copy(), vz=m.vz.copy(), fv_ptr=m.fv_ptr.copy(), fv_idx=m.fv_idx.copy(),
             owner=m.owner.copy(), neigh=m.neigh.copy())
    breaker(a)
    with pytest.raises(gvof.GvofError) as e:
        gvof.gvof_mesh_create(a["vx"], a["vy"], a["vz"], a["fv_ptr"], a["fv_idx"], a["owner"], a["neigh"], m.nc)
    assert e.value.code == code
    assert gvof.gvof_last_error(None)


def test_face_with_too_many_vertices_is_rejected():
    m = inputs.cartesian_mesh(2)
    fv_ptr = m.fv_ptr.copy()
    # pretend face 0 has 9 vertices by shifting pointers (vertex ids stay valid)
    fv_ptr = np.concatenate([[0], fv_ptr[1:] + 5])
    fv_idx = np.concatenate([m.fv_idx[:5], m.fv_idx])
    with pytest.raises(gvof.GvofError) as e:
        gvof.gvof_mesh_create(m.vx, m.vy, m.vz, fv_ptr, fv_idx, m.owner, m.neigh, m.nc)
    assert e.value.code == gvof.GVOF_E_MESH


def test_calls_before_bind_fail_cleanly():
    m = inputs.cartesian_mesh(2)
    h = gvof.gvof_mesh_create(*m.arrays(), m.nc)
    try:
        code = gvof.lib().gvof_reconstruct(h, None, None, None)
        assert code == gvof.GVOF_E_ARG
        assert "not bound" in gvof.gvof_last_error(h)
        code = gvof.lib().gvof_advect_step(h, None, None, C.c_double(0.1), None, None, None, None, None)
        assert code == gvof.GVOF_E_ARG
    finally:
        gvof.gvof_mesh_destroy(h)
