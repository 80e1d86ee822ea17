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


def test_probe_library_exports_every_declared_symbol():
    from paper_2111_01524_amd import probe
    txt = open(os.path.join(ROOT, "include", "gvof_probe.h")).read()
    txt = re.sub(r"/\*.*?\*/", "", txt, flags=re.S)
    names = sorted(set(re.findall(r"\b(gvof_[a-z0-9_]+)\s*\(", txt)))
    assert names == sorted(probe.exported_symbols())
    L = probe.lib()
    for n in names:
        assert hasattr(L, n), n


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


def _concat(meshes):
    """Disjoint union of meshes in the batch numbering (test-side reference)."""
    vo = np.cumsum([0] + [m.nv for m in meshes])
    co = np.cumsum([0] + [m.nc for m in meshes])
    fvo = np.cumsum([0] + [m.fv_idx.size for m in meshes])
    vx = np.concatenate([m.vx for m in meshes]); vy = np.concatenate([m.vy for m in meshes])
    vz = np.concatenate([m.vz for m in meshes])
    fv_ptr = np.concatenate([[0]] + [m.fv_ptr[1:] + fvo[q] for q, m in enumerate(meshes)])
    fv_idx = np.concatenate([m.fv_idx + vo[q] for q, m in enumerate(meshes)])
    owner = np.concatenate([m.owner + co[q] for q, m in enumerate(meshes)])
    neigh = np.concatenate([np.where(m.neigh >= 0, m.neigh + co[q], -1) for q, m in enumerate(meshes)])
    return vx, vy, vz, fv_ptr, fv_idx, owner, neigh, int(co[-1])


def test_batch_create_is_the_disjoint_union():
    ms = [inputs.cartesian_mesh(3), inputs.jittered_mesh(2, seed=1), inputs.cartesian_mesh(2)]
    parts = [gvof.gvof_mesh_create(*m.arrays(), m.nc) for m in ms]
    try:
        h = gvof.gvof_batch_create(parts)
    finally:
        for p in parts:
            gvof.gvof_mesh_destroy(p)
    try:
        vo, fo, co = gvof.gvof_batch_offsets(h)
        assert list(vo) == list(np.cumsum([0] + [m.nv for m in ms]))
        assert list(fo) == list(np.cumsum([0] + [m.nf for m in ms]))
        assert list(co) == list(np.cumsum([0] + [m.nc for m in ms]))
        u = gvof.gvof_mesh_create(*_concat(ms))
        try:
            assert gvof.gvof_mesh_sizes(h) == gvof.gvof_mesh_sizes(u)
            # the batch carries three problem-id arrays and a shape table on top of the union's workspace
            extra = gvof.gvof_mesh_workspace_bytes(h) - gvof.gvof_mesh_workspace_bytes(u)
            assert 4 * (vo[-1] + fo[-1] + co[-1]) <= extra <= 4 * (vo[-1] + fo[-1] + co[-1]) + 8 * 256
        finally:
            gvof.gvof_mesh_destroy(u)
        with pytest.raises(gvof.GvofError):  # a batch is not a part
            gvof.gvof_batch_create([h])
    finally:
        gvof.gvof_mesh_destroy(h)


def test_batch_create_rejects_mixed_parameters():
    m = inputs.cartesian_mesh(2)
    p2 = gvof.gvof_params_default()
    p2.beta = 2.0
    a = gvof.gvof_mesh_create(*m.arrays(), m.nc)
    b = gvof.gvof_mesh_create(*m.arrays(), m.nc, p2)
    try:
        with pytest.raises(gvof.GvofError):
            gvof.gvof_batch_create([a, b])
        with pytest.raises(gvof.GvofError):
            gvof.gvof_batch_create([])
    finally:
        gvof.gvof_mesh_destroy(a)
        gvof.gvof_mesh_destroy(b)


def test_launch_config_validation_without_gpu():
    m = inputs.cartesian_mesh(2)
    h = gvof.gvof_mesh_create(*m.arrays(), m.nc)
    try:
        c = gvof.gvof_get_launch_config(h)
        assert c.as_dict() == dict(sweep_threads=256, recon_threads=128, prep_blocks=16384,
                                   pair_blocks_per_region=16, filter_lanes=0, staged_faces=0,
                                   staged_pairs=0, prep_lanes=64, units_rank=4)
        for bad in (dict(sweep_threads=96), dict(recon_threads=256), dict(prep_blocks=0),
                    dict(pair_blocks_per_region=300), dict(filter_lanes=12), dict(staged_faces=-1),
                    dict(staged_pairs=-1), dict(prep_lanes=16), dict(units_rank=6)):
            d = c.as_dict()
            d.update(bad)
            with pytest.raises(gvof.GvofError):
                gvof.gvof_set_launch_config(h, gvof.gvof_launch_config(**d))
        d = c.as_dict()
        for fl, ur in ((64, 8), (8, 4), (0, 8)):  # the per-pair filter's lane counts and 0, the runs filter
            d.update(sweep_threads=512, filter_lanes=fl, prep_lanes=32, units_rank=ur)
            gvof.gvof_set_launch_config(h, gvof.gvof_launch_config(**d))
            assert gvof.gvof_get_launch_config(h).as_dict() == d
        with pytest.raises(gvof.GvofError):  # not bound
            gvof.gvof_graph_launch(h)
    finally:
        gvof.gvof_mesh_destroy(h)


def test_unit_buffer_only_for_meshes_with_general_cells():
    """The general-cell unit buffer is sized on the host from the cells that
    are not axis-aligned boxes (the device's box test, redone on the host):
    none for a Cartesian grid, at least 4 Mi entries (16 B each, plus the
    deep-unit list) once one interior vertex moves and its 8 cells become
    general."""
    def ws(m):
        h = gvof.gvof_mesh_create(*m.arrays(), m.nc)
        try:
            return gvof.gvof_mesh_workspace_bytes(h)
        finally:
            gvof.gvof_mesh_destroy(h)

    m = inputs.cartesian_mesh(6)
    base = ws(m)
    v = (3 * 7 + 3) * 7 + 3  # an interior vertex of the 7^3 lattice
    m.vx[v] += 0.01
    moved = ws(m)
    grown = ((4 << 20) - 256) * (16 + 4)  # all boxes: a minimal buffer of 256 entries
    assert moved - base >= grown
    assert ws(inputs.jittered_mesh(6, seed=2)) - base >= grown


def test_flags_select_the_flux_polyhedron_method():
    """GVOF_FLAG_EMFPA and GVOF_FLAG_NMFPA select the method: EMFPA slots hold the
    lateral centres and the pair buffer is sized for 5I flux tets per face
    (larger workspace), NMFPA sizes as FMFPA; both together, two
    reconstruction flags, or any other bit, is an argument error; a batch of
    mixed methods is rejected."""
    m = inputs.cartesian_mesh(4)
    pe = gvof.gvof_params_default()
    pe.flags = gvof.GVOF_FLAG_EMFPA
    pn = gvof.gvof_params_default()
    pn.flags = gvof.GVOF_FLAG_NMFPA
    a = gvof.gvof_mesh_create(*m.arrays(), m.nc)
    b = gvof.gvof_mesh_create(*m.arrays(), m.nc, pe)
    c = gvof.gvof_mesh_create(*m.arrays(), m.nc, pn)
    try:
        assert gvof.gvof_mesh_workspace_bytes(b) > gvof.gvof_mesh_workspace_bytes(a)
        assert gvof.gvof_mesh_workspace_bytes(c) == gvof.gvof_mesh_workspace_bytes(a)
        for pair in ([a, b], [a, c], [b, c]):
            with pytest.raises(gvof.GvofError):
                gvof.gvof_batch_create(pair)
    finally:
        gvof.gvof_mesh_destroy(a)
        gvof.gvof_mesh_destroy(b)
        gvof.gvof_mesh_destroy(c)
    for bad in (128, 0x80000000, 3, 4 | 8, 8 | 32, 16 | 32):
        p = gvof.gvof_params_default()
        p.flags = bad
        with pytest.raises(gvof.GvofError) as e:
            gvof.gvof_mesh_create(*m.arrays(), m.nc, p)
        assert e.value.code == gvof.GVOF_E_ARG


def test_lsfir_settings():
    """GVOF_FLAG_LSFIR takes 1..GVOF_MAX_LSFIR_OUTER outer passes and a finite
    tolerance >= 0 (by default the paper's test settings, 4 passes and
    1e-3 rad: Sec. "Test programs and performance analysis"), adds the
    PLIC-centre and fitted-normal buffers to the workspace, and combines with
    any flux polyhedron method and with the optional weight floor; batches
    need equal settings."""
    m = inputs.cartesian_mesh(4)
    d = gvof.gvof_params_default()
    assert d.lsfir_outer == 4 and d.lsfir_tol == 1e-3
    base = gvof.gvof_mesh_create(*m.arrays(), m.nc)
    handles = [base]
    try:
        for flags in (gvof.GVOF_FLAG_LSFIR, gvof.GVOF_FLAG_LSFIR | gvof.GVOF_FLAG_EMFPA,
                      gvof.GVOF_FLAG_LSFIR | gvof.GVOF_FLAG_NMFPA,
                      gvof.GVOF_FLAG_LSFIR | gvof.GVOF_FLAG_LSFIR_CAP):
            p = gvof.gvof_params_default()
            p.flags = flags
            p.lsfir_outer = gvof.GVOF_MAX_LSFIR_OUTER
            h = gvof.gvof_mesh_create(*m.arrays(), m.nc, p)
            handles.append(h)
            assert gvof.gvof_mesh_workspace_bytes(h) >= gvof.gvof_mesh_workspace_bytes(base) + 48 * m.nc
        with pytest.raises(gvof.GvofError):
            gvof.gvof_batch_create([base, handles[1]])
        for outer, tol in ((0, 0.0), (gvof.GVOF_MAX_LSFIR_OUTER + 1, 0.0), (1, -1e-3), (1, float("nan")),
                           (1, float("inf"))):
            p = gvof.gvof_params_default()
            p.flags = gvof.GVOF_FLAG_LSFIR
            p.lsfir_outer, p.lsfir_tol = outer, tol
            with pytest.raises(gvof.GvofError) as e:
                gvof.gvof_mesh_create(*m.arrays(), m.nc, p)
            assert e.value.code == gvof.GVOF_E_ARG
    finally:
        for h in handles:
            gvof.gvof_mesh_destroy(h)


def test_isosurface_reconstruction_flags():
    """LLCIR, ELCIR and CLCIR each add the isosurface and PLIC-centre buffers,
    combine with any flux polyhedron method, and take any mesh whose cells
    have at most 32 faces (the distorted grid's cells have 24)."""
    m = inputs.jittered_mesh(3, seed=1)
    base = gvof.gvof_mesh_create(*m.arrays(), m.nc)
    handles = [base]
    try:
        for flags in (gvof.GVOF_FLAG_LLCIR, gvof.GVOF_FLAG_ELCIR | gvof.GVOF_FLAG_EMFPA,
                      gvof.GVOF_FLAG_CLCIR | gvof.GVOF_FLAG_NMFPA):
            p = gvof.gvof_params_default()
            p.flags = flags
            h = gvof.gvof_mesh_create(*m.arrays(), m.nc, p)
            handles.append(h)
            assert gvof.gvof_mesh_workspace_bytes(h) >= gvof.gvof_mesh_workspace_bytes(base) + 97 * m.nc
    finally:
        for h in handles:
            gvof.gvof_mesh_destroy(h)
