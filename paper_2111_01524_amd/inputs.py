"""Seeded synthetic inputs for the unsplit geometric VOF path.

This module is shared by the HIP path's tests/bench and by the CPU oracle's
tests.  It builds meshes, samples velocity fields and picks time steps; it
holds none of the method's own arithmetic (no face area vectors for the
method, no tags, no reconstruction, no flux polyhedra).

Workloads follow the paper's test programs:
  * grids: uniform Cartesian hexahedra and "distorted cubic" non-convex
    hexahedra (Sec. "Test programs", grid list).  The distorted grid here moves
    every interior vertex by an independent uniform offset of at most h/4 per
    axis (seeded splitmix64) and triangulates every quadrilateral through its
    vertex mean, which gives the paper's 14-vertex / 24-triangle cells;
  * velocity: the 3D deformation field of Enright (Sec. "3D deformation
    test"), uniform translation (Sec. "Translation test");
  * time step: Eq. (cfl).

Mesh format (OpenFOAM-like, Sec. "Grid construction"): vertices, faces as a
CSR list of vertex indices ordered counter-clockwise seen from outside the
owner cell, owner and neighbour per face (-1 on the boundary).
"""
from __future__ import annotations

import dataclasses
import math

import numpy as np

__all__ = [
    "Mesh", "splitmix64_uniform", "cartesian_mesh", "jittered_mesh",
    "enright_u0", "enright_vector_potential", "face_sample_points",
    "velocity_uniform", "velocity_enright", "cfl_dt", "step_schedule",
    "enright_time_factor", "batch_problem_specs", "served_job_specs",
]

MASK64 = (1 << 64) - 1


def splitmix64_uniform(seed: int, n: int) -> np.ndarray:
    """n uniform doubles in [0,1) from the splitmix64 sequence started at `seed`.

    splitmix64 (Steele, Lea, Flood 2014): state += 0x9E3779B97F4A7C15, then the
    finaliser z ^= z>>30; z *= 0xBF58476D1CE4E5B9; z ^= z>>27;
    z *= 0x94D049BB133111EB; z ^= z>>31.  The top 53 bits give the double.
    """
    out = np.empty(n, dtype=np.float64)
    state = seed & MASK64
    # vectorised in blocks of uint64 arithmetic (wraps mod 2^64)
    idx = np.arange(1, n + 1, dtype=np.uint64)
    with np.errstate(over="ignore"):
        z = (np.uint64(state) + idx * np.uint64(0x9E3779B97F4A7C15))
        z = (z ^ (z >> np.uint64(30))) * np.uint64(0xBF58476D1CE4E5B9)
        z = (z ^ (z >> np.uint64(27))) * np.uint64(0x94D049BB133111EB)
        z = z ^ (z >> np.uint64(31))
    out[:] = (z >> np.uint64(11)).astype(np.float64) * (1.0 / 9007199254740992.0)
    return out


@dataclasses.dataclass
class Mesh:
    """Polyhedral mesh in the paper's owner/neighbour form."""
    vx: np.ndarray          # (nv,) float64
    vy: np.ndarray
    vz: np.ndarray
    fv_ptr: np.ndarray      # (nf+1,) int32
    fv_idx: np.ndarray      # (fv_ptr[-1],) int32
    owner: np.ndarray       # (nf,) int32
    neigh: np.ndarray       # (nf,) int32, -1 on the boundary
    nc: int
    kind: str = "cartesian"
    n: int = 0              # cells per side for structured generators

    @property
    def nv(self) -> int:
        return int(self.vx.shape[0])

    @property
    def nf(self) -> int:
        return int(self.owner.shape[0])

    def arrays(self):
        return (self.vx, self.vy, self.vz, self.fv_ptr, self.fv_idx, self.owner, self.neigh)


def _structured_quads(n: int):
    """Quadrilateral faces of an n^3 block on the (n+1)^3 vertex lattice.

    Returns (quads[nq,4] vertex ids, owner[nq], neigh[nq]); each quad is
    counter-clockwise seen from outside its owner.
    """
    m = n + 1

    def vid(i, j, k):
        return i + m * (j + m * k)

    def cid(i, j, k):
        return i + n * (j + n * k)

    quads, own, nei = [], [], []
    # x-normal faces at lattice plane i: vertices (i,j,k),(i,j+1,k),(i,j+1,k+1),(i,j,k+1) -> +x
    ii, jj, kk = np.meshgrid(np.arange(m), np.arange(n), np.arange(n), indexing="ij")
    ii, jj, kk = ii.ravel(), jj.ravel(), kk.ravel()
    q = np.stack([vid(ii, jj, kk), vid(ii, jj + 1, kk), vid(ii, jj + 1, kk + 1), vid(ii, jj, kk + 1)], 1)
    o = np.where(ii > 0, cid(ii - 1, jj, kk), cid(np.minimum(ii, n - 1), jj, kk))
    nb = np.where((ii > 0) & (ii < n), cid(np.minimum(ii, n - 1), jj, kk), -1)
    flip = ii == 0            # boundary at x=0: owner is cell 0, outward is -x
    q[flip] = q[flip][:, ::-1]
    quads.append(q); own.append(o); nei.append(nb)
    # y-normal faces: (i,j,k),(i,j,k+1),(i+1,j,k+1),(i+1,j,k) -> +y
    ii, jj, kk = np.meshgrid(np.arange(n), np.arange(m), np.arange(n), indexing="ij")
    ii, jj, kk = ii.ravel(), jj.ravel(), kk.ravel()
    q = np.stack([vid(ii, jj, kk), vid(ii, jj, kk + 1), vid(ii + 1, jj, kk + 1), vid(ii + 1, jj, kk)], 1)
    o = np.where(jj > 0, cid(ii, jj - 1, kk), cid(ii, np.minimum(jj, n - 1), kk))
    nb = np.where((jj > 0) & (jj < n), cid(ii, np.minimum(jj, n - 1), kk), -1)
    flip = jj == 0
    q[flip] = q[flip][:, ::-1]
    quads.append(q); own.append(o); nei.append(nb)
    # z-normal faces: (i,j,k),(i+1,j,k),(i+1,j+1,k),(i,j+1,k) -> +z
    ii, jj, kk = np.meshgrid(np.arange(n), np.arange(n), np.arange(m), indexing="ij")
    ii, jj, kk = ii.ravel(), jj.ravel(), kk.ravel()
    q = np.stack([vid(ii, jj, kk), vid(ii + 1, jj, kk), vid(ii + 1, jj + 1, kk), vid(ii, jj + 1, kk)], 1)
    o = np.where(kk > 0, cid(ii, jj, kk - 1), cid(ii, jj, np.minimum(kk, n - 1)))
    nb = np.where((kk > 0) & (kk < n), cid(ii, jj, np.minimum(kk, n - 1)), -1)
    flip = kk == 0
    q[flip] = q[flip][:, ::-1]
    quads.append(q); own.append(o); nei.append(nb)
    return (np.concatenate(quads).astype(np.int64), np.concatenate(own).astype(np.int64),
            np.concatenate(nei).astype(np.int64))


def _lattice(n: int, lo=(0.0, 0.0, 0.0), hi=(1.0, 1.0, 1.0)):
    m = n + 1
    # vertex id = i + m*(j + m*k)
    i = np.arange(m)
    xs = lo[0] + (hi[0] - lo[0]) * i / n
    ys = lo[1] + (hi[1] - lo[1]) * i / n
    zs = lo[2] + (hi[2] - lo[2]) * i / n
    X = np.broadcast_to(xs[None, None, :], (m, m, m)).ravel().copy()
    Y = np.broadcast_to(ys[None, :, None], (m, m, m)).ravel().copy()
    Z = np.broadcast_to(zs[:, None, None], (m, m, m)).ravel().copy()
    return X, Y, Z


def cartesian_mesh(n: int, lo=(0.0, 0.0, 0.0), hi=(1.0, 1.0, 1.0)) -> Mesh:
    """Uniform n^3 hexahedral grid on the box [lo, hi]."""
    X, Y, Z = _lattice(n, lo, hi)
    quads, own, nei = _structured_quads(n)
    nq = quads.shape[0]
    fv_ptr = (np.arange(nq + 1) * 4).astype(np.int32)
    return Mesh(X, Y, Z, fv_ptr, quads.ravel().astype(np.int32), own.astype(np.int32),
                nei.astype(np.int32), n ** 3, "cartesian", n)


def jittered_mesh(n: int, seed: int = 1, amp: float = 0.25, split: bool = True) -> Mesh:
    """Non-convex hexahedral grid on the unit cube.

    Interior lattice vertices are moved by (2U-1)*amp*h per axis, U drawn from
    splitmix64(seed) in lexicographic vertex order (x, y, z draws per vertex).
    Every quadrilateral is then split into 4 triangles through the mean of its
    four corners, which becomes a new mesh vertex.  With split=False the
    (non-planar) quadrilaterals are kept as faces.
    """
    h = 1.0 / n
    X, Y, Z = _lattice(n)
    m = n + 1
    k, j, i = np.unravel_index(np.arange(m ** 3), (m, m, m))
    interior = (i > 0) & (i < n) & (j > 0) & (j < n) & (k > 0) & (k < n)
    nin = int(interior.sum())
    U = splitmix64_uniform(seed, 3 * nin).reshape(nin, 3)
    X[interior] += (2.0 * U[:, 0] - 1.0) * amp * h
    Y[interior] += (2.0 * U[:, 1] - 1.0) * amp * h
    Z[interior] += (2.0 * U[:, 2] - 1.0) * amp * h
    quads, own, nei = _structured_quads(n)
    if not split:
        fv_ptr = (np.arange(quads.shape[0] + 1) * 4).astype(np.int32)
        return Mesh(X, Y, Z, fv_ptr, quads.ravel().astype(np.int32), own.astype(np.int32), nei.astype(np.int32),
                    n ** 3, "jittered-quad", n)
    nq = quads.shape[0]
    nv0 = X.shape[0]
    cx = (X[quads[:, 0]] + X[quads[:, 1]] + X[quads[:, 2]] + X[quads[:, 3]]) / 4.0
    cy = (Y[quads[:, 0]] + Y[quads[:, 1]] + Y[quads[:, 2]] + Y[quads[:, 3]]) / 4.0
    cz = (Z[quads[:, 0]] + Z[quads[:, 1]] + Z[quads[:, 2]] + Z[quads[:, 3]]) / 4.0
    cid = nv0 + np.arange(nq)
    tris = np.empty((nq, 4, 3), dtype=np.int64)
    for e in range(4):
        tris[:, e, 0] = quads[:, e]
        tris[:, e, 1] = quads[:, (e + 1) % 4]
        tris[:, e, 2] = cid
    tris = tris.reshape(-1, 3)
    own4 = np.repeat(own, 4)
    nei4 = np.repeat(nei, 4)
    fv_ptr = (np.arange(tris.shape[0] + 1) * 3).astype(np.int32)
    return Mesh(np.concatenate([X, cx]), np.concatenate([Y, cy]), np.concatenate([Z, cz]),
                fv_ptr, tris.ravel().astype(np.int32), own4.astype(np.int32), nei4.astype(np.int32),
                n ** 3, "jittered", n)


# ----------------------------------------------------------------------------- fields

def enright_u0(x, y, z):
    """Enright 3D deformation field without its time factor cos(pi t / T)."""
    px, py, pz = math.pi * x, math.pi * y, math.pi * z
    u = 2.0 * np.sin(px) ** 2 * np.sin(2 * py) * np.sin(2 * pz)
    v = -np.sin(2 * px) * np.sin(py) ** 2 * np.sin(2 * pz)
    w = -np.sin(2 * px) * np.sin(2 * py) * np.sin(pz) ** 2
    return u, v, w


def enright_vector_potential(x, y, z):
    """A with curl A = enright_u0 (checked symbolically):
    A = (0, -sin^2(pi x) sin(2 pi y) sin^2(pi z)/pi, sin^2(pi x) sin^2(pi y) sin(2 pi z)/pi)."""
    px, py, pz = math.pi * x, math.pi * y, math.pi * z
    ay = -np.sin(px) ** 2 * np.sin(2 * py) * np.sin(pz) ** 2 / math.pi
    az = np.sin(px) ** 2 * np.sin(py) ** 2 * np.sin(2 * pz) / math.pi
    return np.zeros_like(ay), ay, az


def face_sample_points(mesh: Mesh):
    """Where face velocities are sampled: the mean of each face's vertices."""
    cnt = np.diff(mesh.fv_ptr)
    fid = np.repeat(np.arange(mesh.nf), cnt)
    sx = np.bincount(fid, mesh.vx[mesh.fv_idx], mesh.nf) / cnt
    sy = np.bincount(fid, mesh.vy[mesh.fv_idx], mesh.nf) / cnt
    sz = np.bincount(fid, mesh.vz[mesh.fv_idx], mesh.nf) / cnt
    return sx, sy, sz


def velocity_uniform(mesh: Mesh, u=(1.0, 1.0, 1.0)):
    """(u_face[3,nf], u_vert[3,nv]) for a uniform translation."""
    uf = np.empty((3, mesh.nf)); uv = np.empty((3, mesh.nv))
    for a in range(3):
        uf[a] = u[a]; uv[a] = u[a]
    return uf, uv


_GL_X = np.array([-0.9061798459386640, -0.5384693101056831, 0.0, 0.5384693101056831, 0.9061798459386640])
_GL_W = np.array([0.2369268850561891, 0.4786286704993665, 0.5688888888888889, 0.4786286704993665,
                  0.2369268850561891])


def velocity_enright(mesh: Mesh, solenoidal_projection: bool | None = None):
    """Enright field u0 (time factor excluded) at faces and vertices.

    Vertex velocities are exact samples.  Face velocities are exact samples at
    the face vertex mean.  On triangulated (distorted) grids face sampling is not
    discretely divergence free, so with `solenoidal_projection` the face
    velocity is shifted along the triangle normal until its flux equals the
    circulation of the vector potential around the face (Stokes), computed
    once per edge with 5-point Gauss-Legendre quadrature.  Shared edges then
    cancel exactly between faces, so every closed cell has zero net flux up to
    summation round-off.  Cartesian face sampling is already divergence free
    (sin^2(a+b) - sin^2(a-b) = sin 2a sin 2b).
    """
    if solenoidal_projection is None:
        solenoidal_projection = mesh.kind == "jittered"
    sx, sy, sz = face_sample_points(mesh)
    uf = np.stack(enright_u0(sx, sy, sz))
    uv = np.stack(enright_u0(mesh.vx, mesh.vy, mesh.vz))
    if solenoidal_projection:
        cnt = np.diff(mesh.fv_ptr)
        if not np.all(cnt == 3):
            raise ValueError("solenoidal projection implemented for triangle faces only")
        tri = mesh.fv_idx.reshape(-1, 3).astype(np.int64)
        # unique undirected edges, circulation along the low->high id direction
        ea = np.concatenate([tri[:, 0], tri[:, 1], tri[:, 2]])
        eb = np.concatenate([tri[:, 1], tri[:, 2], tri[:, 0]])
        lo, hi = np.minimum(ea, eb), np.maximum(ea, eb)
        key = lo * (mesh.nv + 1) + hi
        ukey, inv = np.unique(key, return_inverse=True)
        ulo, uhi = ukey // (mesh.nv + 1), ukey % (mesh.nv + 1)
        P0 = np.stack([mesh.vx[ulo], mesh.vy[ulo], mesh.vz[ulo]])
        P1 = np.stack([mesh.vx[uhi], mesh.vy[uhi], mesh.vz[uhi]])
        d = P1 - P0
        circ = np.zeros(ukey.shape[0])
        for xq, wq in zip(_GL_X, _GL_W):
            t = 0.5 * (xq + 1.0)
            p = P0 + t * d
            A = enright_vector_potential(p[0], p[1], p[2])
            circ += 0.5 * wq * (A[0] * d[0] + A[1] * d[1] + A[2] * d[2])
        sign = np.where(ea < eb, 1.0, -1.0)
        ce = (circ[inv] * sign).reshape(3, -1)
        Q = (ce[0] + ce[1]) + ce[2]
        x0 = np.stack([mesh.vx[tri[:, 0]], mesh.vy[tri[:, 0]], mesh.vz[tri[:, 0]]])
        x1 = np.stack([mesh.vx[tri[:, 1]], mesh.vy[tri[:, 1]], mesh.vz[tri[:, 1]]])
        x2 = np.stack([mesh.vx[tri[:, 2]], mesh.vy[tri[:, 2]], mesh.vz[tri[:, 2]]])
        nrm = 0.5 * np.cross((x1 - x0).T, (x2 - x0).T).T
        flux = (uf * nrm).sum(0)
        uf = uf + ((Q - flux) / (nrm * nrm).sum(0)) * nrm
    return np.ascontiguousarray(uf), np.ascontiguousarray(uv)


def enright_time_factor(t: float, period: float) -> float:
    return math.cos(math.pi * t / period)


# ----------------------------------------------------------------------------- time step

def cell_bbox_min_sizes(mesh: Mesh):
    """Smallest axis extent of the enclosing box over all cells (Eq. cfl's h)."""
    own, nei = mesh.owner.astype(np.int64), mesh.neigh.astype(np.int64)
    cnt = np.diff(mesh.fv_ptr)
    fid = np.repeat(np.arange(mesh.nf), cnt)
    lo = np.full((3, mesh.nc), np.inf); hi = np.full((3, mesh.nc), -np.inf)
    V = (mesh.vx, mesh.vy, mesh.vz)
    for side in (own, nei):
        c = side[fid]
        ok = c >= 0
        for a in range(3):
            np.minimum.at(lo[a], c[ok], V[a][mesh.fv_idx][ok])
            np.maximum.at(hi[a], c[ok], V[a][mesh.fv_idx][ok])
    return (hi - lo).min(axis=1)


def cfl_dt(mesh: Mesh, u_face_max: np.ndarray, cfl: float) -> float:
    """Eq. (cfl): dt = CFL * min over axes of (min cell extent / max |face velocity|)."""
    h = cell_bbox_min_sizes(mesh)
    r = [h[a] / u_face_max[a] for a in range(3) if u_face_max[a] > 0]
    return cfl * min(r)


def step_schedule(t_end: float, dt: float):
    """Constant dt, with the last step shortened to land on t_end."""
    n = max(1, int(math.ceil(t_end / dt - 1e-12)))
    dts = [dt] * n
    dts[-1] = t_end - dt * (n - 1)
    return dts


# ----------------------------------------------------------------------------- batch / served workloads

def batch_problem_specs(count: int = 256, seed: int = 2, side_lo: int = 16, side_hi: int = 48):
    """Per-problem parameters of the batched workload: side, grid kind, sphere, period."""
    U = splitmix64_uniform(seed, 8 * count).reshape(count, 8)
    specs = []
    for p in range(count):
        side = side_lo + min(int(U[p, 0] * (side_hi - side_lo + 1)), side_hi - side_lo)
        specs.append(dict(
            side=side, kind="jittered" if U[p, 1] < 0.5 else "cartesian",
            radius=0.1 + 0.1 * U[p, 2],
            center=(0.3 + 0.4 * U[p, 3], 0.3 + 0.4 * U[p, 4], 0.3 + 0.4 * U[p, 5]),
            period=1.0 + 2.0 * U[p, 6], jitter_seed=1000 + p))
    return specs


def served_job_specs(duration_s: float = 60.0, rate: float = 20.0, seed: int = 3,
                     sides=(32, 64, 96, 128), steps=(50, 500)):
    """Poisson arrivals with the served workload's job parameters."""
    nmax = int(rate * duration_s * 3 + 64)
    U = splitmix64_uniform(seed, 10 * nmax).reshape(nmax, 10)
    t = 0.0
    jobs = []
    for p in range(nmax):
        t += -math.log(1.0 - U[p, 0]) / rate
        if t > duration_s:
            break
        jobs.append(dict(
            arrival=t, side=sides[min(int(U[p, 1] * len(sides)), len(sides) - 1)],
            kind="jittered" if U[p, 2] < 0.5 else "cartesian",
            radius=0.1 + 0.1 * U[p, 3],
            center=(0.3 + 0.4 * U[p, 4], 0.3 + 0.4 * U[p, 5], 0.3 + 0.4 * U[p, 6]),
            period=1.0 + 2.0 * U[p, 7],
            steps=steps[0] + min(int(U[p, 8] * (steps[1] - steps[0] + 1)), steps[1] - steps[0]),
            jitter_seed=5000 + p))
    return jobs


def grid_key(spec: dict):
    """What a problem's grid and velocity field depend on."""
    return (int(spec["side"]), spec["kind"], int(spec["jitter_seed"]) if spec["kind"] == "jittered" else 0)


def grid_inputs(spec: dict, cfl: float = 0.5):
    """A problem's grid, the Enright field u0 at its faces and vertices, and its CFL time step."""
    n = int(spec["side"])
    mesh = cartesian_mesh(n) if spec["kind"] == "cartesian" else jittered_mesh(n, seed=int(spec["jitter_seed"]))
    uf, uv = velocity_enright(mesh)
    return mesh, uf, uv, cfl_dt(mesh, np.abs(uf).max(axis=1), cfl)


def problem_inputs(spec: dict, cfl: float = 0.5, steps: int | None = None, grids: dict | None = None) -> dict:
    """Inputs of one batched or served problem: its grid, the Enright field
    u0 at faces and vertices, the body, and the effective time step of every
    step, dt_s * cos(pi t_{s+1/2} / T) (the field's time factor folded into dt).
    The problem runs to its own period T, or for `steps` steps (served jobs,
    spec["steps"]) of the CFL time step.  `grids` (grid_key -> grid_inputs)
    lends grids already built; problems then share their arrays."""
    g = grids.get(grid_key(spec)) if grids is not None else None
    mesh, uf, uv, dt = g if g is not None else grid_inputs(spec, cfl)
    T = float(spec["period"])
    nsteps = steps if steps is not None else spec.get("steps")
    sched = step_schedule(T, dt) if nsteps is None else [dt] * int(nsteps)
    t, eff = 0.0, []
    for d in sched:
        eff.append(d * enright_time_factor(t + 0.5 * d, T))
        t += d
    c = spec["center"]
    return dict(mesh=mesh, uf=uf, uv=uv, dt=dt, dt_eff=np.array(eff), nsteps=len(eff),
                shape=("sphere", [float(c[0]), float(c[1]), float(c[2]), float(spec["radius"])]))


def concat_soa(arrays):
    """Batch layout of per-problem SoA arrays (3 x n_q each): 3 x sum n_q, problems in order."""
    return np.ascontiguousarray(np.concatenate(arrays, axis=1))
