"""ctypes front end of the CPU oracle (test infrastructure only).

Only the tests, the smoke check and the benchmark's CPU-baseline leg use this
module.  Arrays of vectors are structure-of-arrays numpy arrays of shape
(3, n) or (4, n).
"""
from __future__ import annotations

import ctypes as C
import os

import numpy as np

HERE = os.path.dirname(os.path.abspath(__file__))
_libs: dict[str, C.CDLL] = {}

_d = C.POINTER(C.c_double)
_i = C.POINTER(C.c_int)
_b = C.POINTER(C.c_int8)


def _lib(counting: bool = False) -> C.CDLL:
    name = "liboracle_count.so" if counting else "liboracle.so"
    if name not in _libs:
        path = os.path.join(HERE, name)
        if not os.path.exists(path):
            raise FileNotFoundError(f"{path} missing: run oracle/build_oracle.py")
        lib = C.CDLL(path)
        lib.orc_mesh_new.restype = C.c_void_p
        lib.orc_mesh_new.argtypes = [C.c_int, _d, _d, _d, C.c_int, _i, _i, _i, _i, C.c_int]
        lib.orc_mesh_free.argtypes = [C.c_void_p]
        lib.orc_mesh_set_method.argtypes = [C.c_void_p, C.c_int]
        lib.orc_mesh_set_method.restype = C.c_int
        lib.orc_mesh_set_recon.argtypes = [C.c_void_p, C.c_int, C.c_int, C.c_double, C.c_int]
        lib.orc_mesh_set_recon.restype = C.c_int
        lib.orc_plic_centres.argtypes = [C.c_void_p, _b, _d, _d, _i]
        lib.orc_lsfir_fit.argtypes = [C.c_void_p, _b, _d, _d, _d, _i]
        lib.orc_iso_polygon.argtypes = [C.c_void_p, C.c_int, _d, C.c_int, _d, _i]
        lib.orc_iso_polygon.restype = C.c_int
        lib.orc_iso_planes.argtypes = [C.c_void_p, _d, _d, _b, C.c_int, _d, _b]
        lib.orc_geometry.argtypes = [C.c_void_p, _d, _d, _d, _d, _d, _d, _b]
        lib.orc_neighbours.argtypes = [C.c_void_p, _i, _i]
        lib.orc_neighbours.restype = C.c_int
        lib.orc_tags.argtypes = [C.c_void_p, _d, C.c_double, _d, _b, _b, _b]
        lib.orc_lsgir.argtypes = [C.c_void_p, _d, _b, C.c_double, _d]
        lib.orc_plane_constant.argtypes = [C.c_void_p, _d, _b, _d, _d]
        lib.orc_cell_cut_volume.argtypes = [C.c_void_p, C.c_int, C.c_double, C.c_double, C.c_double, C.c_double]
        lib.orc_cell_cut_volume.restype = C.c_double
        lib.orc_reconstruct.argtypes = [C.c_void_p, _d, C.c_double, C.c_double, _d, _b, _b, _b, _d]
        lib.orc_face_flux.argtypes = [C.c_void_p, _d, _b, _b, _d, _d, C.c_double, C.c_double, C.c_int, _i, _d, _d,
                                      _i]
        lib.orc_face_flux.restype = C.c_int
        lib.orc_advect.argtypes = [C.c_void_p, _d, _b, _b, _d, _d, C.c_double, C.c_double, _d, _d, _d, _d, _i]
        lib.orc_advect.restype = C.c_int
        lib.orc_update.argtypes = [C.c_void_p, _d, _d, _d, _d]
        lib.orc_flux_coverage.argtypes = [C.c_void_p, _b, _d, _d, C.c_double, C.c_double, _b]
        lib.orc_flux_coverage.restype = C.c_int
        lib.orc_flux_polyhedron.argtypes = [C.c_void_p, C.c_int, _d, _d, C.c_double, C.c_double, C.c_double, _d,
                                            _d]
        lib.orc_flux_polyhedron.restype = C.c_int
        lib.orc_tet_clip_volume.argtypes = [_d, C.c_int, _d]
        lib.orc_tet_clip_volume.restype = C.c_double
        lib.orc_box_clip_volume.argtypes = [_d, _d, C.c_int, _d]
        lib.orc_box_clip_volume.restype = C.c_double
        lib.orc_tet_cell_volume.argtypes = [C.c_void_p, _d, C.c_int, C.c_int, C.c_double, C.c_double, C.c_double,
                                            C.c_double]
        lib.orc_tet_cell_volume.restype = C.c_double
        lib.orc_init_fraction.argtypes = [C.c_void_p, C.c_int, _d, C.c_int, _d]
        lib.orc_set_threads.argtypes = [C.c_int]
        lib.orc_set_threads.restype = C.c_int
        lib.orc_flops_get.restype = C.c_longlong
        lib.orc_counting_build.restype = C.c_int
        _libs[name] = lib
    return _libs[name]


def _p(a, t):
    return a.ctypes.data_as(t)


def _dbl(a):
    return np.ascontiguousarray(a, dtype=np.float64)


def _int(a):
    return np.ascontiguousarray(a, dtype=np.int32)


def _i8(a):
    return np.ascontiguousarray(a, dtype=np.int8)


def set_threads(n: int = 0, counting: bool = False) -> int:
    return _lib(counting).orc_set_threads(n)


class OracleMesh:
    """The oracle's view of a mesh: topology and geometry built on the CPU.

    method selects the flux polyhedra: "fmfpa" (Sec. "Face-matched flux
    polyhedron"), "emfpa" (Sec. "Edge-matched flux polyhedron") or "nmfpa"
    (Sec. "Non-matched flux polyhedron").  recon selects the normals:
    "lsgir" (Sec. LSGIR), "lsfir" (Sec. "Least squares fit interface
    reconstruction", at most lsfir_outer outer iterations, stopping once no
    normal turns by lsfir_tol radians or more; the paper's test settings 4
    and 1e-3 by default; lsfir_cap floors the weight at |d| = 0.05 h, an
    option the paper does not have), or "llcir" / "elcir" /
    "clcir" (Sec. "Isosurface based interface reconstruction").
    """

    METHODS = {"fmfpa": 0, "emfpa": 1, "nmfpa": 2}
    RECONS = {"lsgir": 0, "lsfir": 1, "llcir": 2, "elcir": 3, "clcir": 4}

    def __init__(self, mesh, counting: bool = False, method: str = "fmfpa", recon: str = "lsgir",
                 lsfir_outer: int = 4, lsfir_tol: float = 1e-3, lsfir_cap: bool = False):
        if method not in self.METHODS:
            raise ValueError(f"unknown flux polyhedron method {method!r}")
        self.lib = _lib(counting)
        self.counting = counting
        self.method = method
        self.mesh = mesh
        self.nv, self.nf, self.nc = mesh.nv, mesh.nf, mesh.nc
        self._keep = [_dbl(mesh.vx), _dbl(mesh.vy), _dbl(mesh.vz), _int(mesh.fv_ptr), _int(mesh.fv_idx),
                      _int(mesh.owner), _int(mesh.neigh)]
        vx, vy, vz, fp, fi, ow, ne = self._keep
        self.h = self.lib.orc_mesh_new(self.nv, _p(vx, _d), _p(vy, _d), _p(vz, _d), self.nf, _p(fp, _i),
                                       _p(fi, _i), _p(ow, _i), _p(ne, _i), self.nc)
        if self.lib.orc_mesh_set_method(self.h, self.METHODS[method]) != 0:
            raise RuntimeError("oracle rejected the flux polyhedron method")
        if recon not in self.RECONS:
            raise ValueError(f"unknown reconstruction {recon!r}")
        self.recon = recon
        if self.lib.orc_mesh_set_recon(self.h, self.RECONS[recon], int(lsfir_outer), float(lsfir_tol),
                                       int(bool(lsfir_cap))):
            raise ValueError("oracle rejected the reconstruction settings")

    def __del__(self):
        h = getattr(self, "h", None)
        if h:
            self.lib.orc_mesh_free(h)
            self.h = None

    # -- geometry / topology
    def geometry(self):
        S = np.zeros((3, self.nf)); fc = np.zeros((3, self.nf)); V = np.zeros(self.nc)
        cc = np.zeros((3, self.nc)); lo = np.zeros((3, self.nc)); hi = np.zeros((3, self.nc))
        box = np.zeros(self.nc, np.int8)
        self.lib.orc_geometry(self.h, _p(S, _d), _p(fc, _d), _p(V, _d), _p(cc, _d), _p(lo, _d), _p(hi, _d),
                              _p(box, _b))
        return dict(S=S, fc=fc, V=V, cc=cc, bbmin=lo, bbmax=hi, isbox=box)

    def neighbours(self):
        n = self.lib.orc_neighbours(self.h, None, None)
        ptr = np.zeros(self.nc + 1, np.int32); idx = np.zeros(max(n, 1), np.int32)
        self.lib.orc_neighbours(self.h, _p(ptr, _i), _p(idx, _i))
        return ptr, idx[:n]

    # -- reconstruction
    def tags(self, F, eps=1e-12):
        F = _dbl(F)
        Fs = np.zeros(self.nv); tn = np.zeros(self.nv, np.int8); tf = np.zeros(self.nf, np.int8)
        tc = np.zeros(self.nc, np.int8)
        self.lib.orc_tags(self.h, _p(F, _d), eps, _p(Fs, _d), _p(tn, _b), _p(tf, _b), _p(tc, _b))
        return Fs, tn, tf, tc

    def lsgir(self, F, tcell, beta=1.5):
        F = _dbl(F); tc = _i8(tcell); n = np.zeros((3, self.nc))
        self.lib.orc_lsgir(self.h, _p(F, _d), _p(tc, _b), beta, _p(n, _d))
        return n

    def plane_constant(self, F, tcell, n):
        F = _dbl(F); tc = _i8(tcell); n = _dbl(n); Cc = np.zeros(self.nc)
        self.lib.orc_plane_constant(self.h, _p(F, _d), _p(tc, _b), _p(n, _d), _p(Cc, _d))
        return Cc

    def iso_polygon(self, c, node_values):
        """The isosurface F* = 1/2 of cell c: (points (k, 3) in loop order, faces of the polygon edges),
        or None when the cell has no usable isosurface."""
        fs = _dbl(node_values); pts = np.zeros(3 * 64); fc = np.zeros(64, np.int32)
        n = self.lib.orc_iso_polygon(self.h, int(c), _p(fs, _d), 64, _p(pts, _d), _p(fc, _i))
        if n < 0:
            return None
        return pts[: 3 * n].reshape(-1, 3), fc[:n]

    def iso_planes(self, node_values, F, tcell, planes, level):
        """Isosurface planes (level "llcir" / "elcir" / "clcir") from given node values, F after the
        cut-off, tags and LSGIR planes: (planes (4, nc), has-isosurface flags)."""
        fs = _dbl(node_values); Fc = _dbl(F); tc = _i8(tcell); pl = _dbl(planes).copy()
        ok = np.zeros(self.nc, np.int8)
        self.lib.orc_iso_planes(self.h, _p(fs, _d), _p(Fc, _d), _p(tc, _b), self.RECONS[level], _p(pl, _d),
                                _p(ok, _b))
        return pl, ok

    def plic_centres(self, tcell, planes):
        """Vertex means of the PLIC polygons of the tag-0 cells (3, nc) and their vertex counts."""
        tc = _i8(tcell); pl = _dbl(planes); out = np.zeros((3, self.nc)); cnt = np.zeros(self.nc, np.int32)
        self.lib.orc_plic_centres(self.h, _p(tc, _b), _p(pl, _d), _p(out, _d), _p(cnt, _i))
        return out, cnt

    def lsfir_fit(self, tcell, normals, centres):
        """One LSFIR fit per tag-0 cell: fitted normals (3, nc) and valid-neighbour counts."""
        tc = _i8(tcell); nr = _dbl(normals); xc = _dbl(centres)
        out = np.zeros((3, self.nc)); nv = np.zeros(self.nc, np.int32)
        self.lib.orc_lsfir_fit(self.h, _p(tc, _b), _p(nr, _d), _p(xc, _d), _p(out, _d), _p(nv, _i))
        return out, nv

    def cell_cut_volume(self, c, n, Cst):
        return self.lib.orc_cell_cut_volume(self.h, int(c), float(n[0]), float(n[1]), float(n[2]), float(Cst))

    def reconstruct(self, F, eps=1e-12, beta=1.5):
        """Returns (F_cut, Fstar, tag_node, tag_face, tag_cell, planes[4,nc])."""
        Fc = _dbl(F).copy()
        Fs = np.zeros(self.nv); tn = np.zeros(self.nv, np.int8); tf = np.zeros(self.nf, np.int8)
        tc = np.zeros(self.nc, np.int8); pl = np.zeros((4, self.nc))
        self.lib.orc_reconstruct(self.h, _p(Fc, _d), eps, beta, _p(Fs, _d), _p(tn, _b), _p(tf, _b), _p(tc, _b),
                                 _p(pl, _d))
        return Fc, Fs, tn, tf, tc, pl

    # -- advection
    def face_flux(self, planes, tcell, tface, u_face, u_vert, dt, faces=None, degen=1e-12):
        pl = _dbl(planes); tc = _i8(tcell); tf = _i8(tface); uf = _dbl(u_face); uv = _dbl(u_vert)
        if faces is None:
            n, sel = -1, None
            m = self.nf
        else:
            sel = _int(faces); n = m = sel.shape[0]
        Vd = np.zeros(m); VF = np.zeros(m); up = np.zeros(m, np.int32)
        bad = self.lib.orc_face_flux(self.h, _p(pl, _d), _p(tc, _b), _p(tf, _b), _p(uf, _d), _p(uv, _d), float(dt),
                                     degen, n, None if sel is None else _p(sel, _i), _p(Vd, _d), _p(VF, _d),
                                     _p(up, _i))
        return Vd, VF, up, bad

    def advect(self, planes, tcell, tface, u_face, u_vert, dt, F_in, degen=1e-12):
        """Returns (F_out, Vd, VF, upwind, n_degenerate)."""
        pl = _dbl(planes); tc = _i8(tcell); tf = _i8(tface); uf = _dbl(u_face); uv = _dbl(u_vert)
        Fin = _dbl(F_in); Fout = np.zeros(self.nc); Vd = np.zeros(self.nf); VF = np.zeros(self.nf)
        up = np.zeros(self.nf, np.int32)
        bad = self.lib.orc_advect(self.h, _p(pl, _d), _p(tc, _b), _p(tf, _b), _p(uf, _d), _p(uv, _d), float(dt),
                                  degen, _p(Fin, _d), _p(Fout, _d), _p(Vd, _d), _p(VF, _d), _p(up, _i))
        return Fout, Vd, VF, up, bad

    def coverage(self, tface, u_face, u_vert, dt, degen=1e-12):
        """Per face, 1 where the face builds a flux polyhedron that leaves the
        enclosing boxes of its candidate cells (inside the domain's box), else 0."""
        tf = _i8(tface); uf = _dbl(u_face); uv = _dbl(u_vert); out = np.zeros(self.nf, np.int8)
        self.lib.orc_flux_coverage(self.h, _p(tf, _b), _p(uf, _d), _p(uv, _d), float(dt), degen, _p(out, _b))
        return out

    def update(self, Vd, VF, F_in):
        Vd = _dbl(Vd); VF = _dbl(VF); Fin = _dbl(F_in); Fout = np.zeros(self.nc)
        self.lib.orc_update(self.h, _p(Vd, _d), _p(VF, _d), _p(Fin, _d), _p(Fout, _d))
        return Fout

    def flux_polyhedron(self, face, u_vert, dt, Vd, degen=1e-12, u_face=None):
        """(points, signed volume of the tet fan, apex degenerate).

        Points: x_0..x_{I-1}, b_0..b_{I-1}, apex (NMFPA: b_0), then for EMFPA
        the lateral-face centres m_0..m_{I-1}.  NMFPA reads u_face (3, nf),
        the others u_vert (3, nv).
        """
        uv = _dbl(u_vert) if u_vert is not None else np.zeros((3, self.nv))
        uf = _dbl(u_face) if u_face is not None else np.zeros((3, self.nf))
        pts = np.zeros(3 * (3 * 8 + 1)); vol = np.zeros(1)
        I = self.lib.orc_flux_polyhedron(self.h, int(face), _p(uf, _d), _p(uv, _d), float(dt), float(Vd), degen,
                                         _p(pts, _d), _p(vol, _d))
        k = abs(I)
        npts = 3 * k + 1 if self.method == "emfpa" else 2 * k + 1
        return pts[: 3 * npts].reshape(-1, 3), float(vol[0]), I < 0

    def tet_cell_volume(self, tet, c, plane=None):
        t = _dbl(tet).ravel()
        if plane is None:
            return self.lib.orc_tet_cell_volume(self.h, _p(t, _d), int(c), 0, 0.0, 0.0, 0.0, 0.0)
        return self.lib.orc_tet_cell_volume(self.h, _p(t, _d), int(c), 1, float(plane[0]), float(plane[1]),
                                            float(plane[2]), float(plane[3]))

    def init_fraction(self, shape: str, params, n_div: int = 10):
        kind = {"sphere": 0, "plane": 1}[shape]
        sp = _dbl(params); F = np.zeros(self.nc)
        self.lib.orc_init_fraction(self.h, kind, _p(sp, _d), int(n_div), _p(F, _d))
        return F

    # -- flop counting (counting build only)
    def flops_reset(self):
        self.lib.orc_flops_reset()

    def flops(self) -> int:
        return int(self.lib.orc_flops_get())


def tet_clip_volume(tet, planes):
    t = _dbl(tet).ravel(); pl = _dbl(planes).ravel()
    return _lib().orc_tet_clip_volume(_p(t, _d), pl.shape[0] // 4, _p(pl, _d))


def box_clip_volume(lo, hi, planes):
    a = _dbl(lo); b = _dbl(hi); pl = _dbl(planes).ravel()
    return _lib().orc_box_clip_volume(_p(a, _d), _p(b, _d), pl.shape[0] // 4, _p(pl, _d))
