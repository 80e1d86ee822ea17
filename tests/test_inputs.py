"""The seeded input generators: published splitmix64 values, mesh orientation, fields."""
import numpy as np

from paper_2111_01524_amd import inputs


def test_splitmix64_published_values():
    # splitmix64 from seed 0: 0xe220a8397b1dcdaf, 0x6e789e6aa1b965f4, 0x06c45d188009454f
    u = inputs.splitmix64_uniform(0, 3)
    ref = [0xe220a8397b1dcdaf, 0x6e789e6aa1b965f4, 0x06c45d188009454f]
    assert np.array_equal(u, np.array([(r >> 11) / 2.0 ** 53 for r in ref]))


def _signed_volumes(m):
    # divergence theorem on triangulated faces: sum over faces of x_f . S_f / 3
    vol = np.zeros(m.nc)
    for f in range(m.nf):
        vs = m.fv_idx[m.fv_ptr[f]:m.fv_ptr[f + 1]]
        P = np.stack([m.vx[vs], m.vy[vs], m.vz[vs]], 1)
        c = P.mean(0)
        A = 0.5 * sum(np.cross(P[i] - c, P[(i + 1) % len(vs)] - c) for i in range(len(vs)))
        vol[m.owner[f]] += c @ A / 3
        if m.neigh[f] >= 0:
            vol[m.neigh[f]] -= c @ A / 3
    return vol


def test_meshes_are_outward_oriented():
    for m in (inputs.cartesian_mesh(3), inputs.jittered_mesh(3, seed=2)):
        v = _signed_volumes(m)
        assert (v > 0).all()
        assert abs(v.sum() - 1.0) < 1e-13
        assert m.nf == (3 * 3 * 3 * 4 if m.kind == "cartesian" else 4 * 3 * 3 * 3 * 4)


def test_jitter_is_bounded_and_interior_only():
    n = 6
    base = inputs.cartesian_mesh(n)
    m = inputs.jittered_mesh(n, seed=1)
    d = np.stack([m.vx[:base.nv] - base.vx, m.vy[:base.nv] - base.vy, m.vz[:base.nv] - base.vz])
    assert np.abs(d).max() <= 0.25 / n + 1e-15
    on_wall = (np.isclose(base.vx, 0) | np.isclose(base.vx, 1) | np.isclose(base.vy, 0) | np.isclose(base.vy, 1)
               | np.isclose(base.vz, 0) | np.isclose(base.vz, 1))
    assert np.abs(d[:, on_wall]).max() == 0.0


def test_enright_solenoidal_projection():
    m = inputs.jittered_mesh(5, seed=1)
    uf, uv = inputs.velocity_enright(m)
    tri = m.fv_idx.reshape(-1, 3)
    x = [np.stack([m.vx[tri[:, k]], m.vy[tri[:, k]], m.vz[tri[:, k]]]) for k in range(3)]
    S = 0.5 * np.cross((x[1] - x[0]).T, (x[2] - x[0]).T).T
    flux = (uf * S).sum(0)
    net = np.zeros(m.nc)
    np.add.at(net, m.owner, flux)
    inner = m.neigh >= 0
    np.add.at(net, m.neigh[inner], -flux[inner])
    assert np.abs(net).max() < 1e-16
    # walls carry no flux
    assert np.abs(flux[~inner]).max() < 1e-17


def test_cfl_and_schedule():
    m = inputs.cartesian_mesh(64)
    uf, uv = inputs.velocity_enright(m)
    dt = inputs.cfl_dt(m, np.abs(uf).max(axis=1), 0.5)
    assert abs(dt - 0.5 / 64 / 2) < 1e-5
    dts = inputs.step_schedule(3.0, dt)
    assert abs(sum(dts) - 3.0) < 1e-12 and dts[-1] <= dt
