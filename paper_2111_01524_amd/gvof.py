"""Python binding of libgvof.so (argument marshalling only).

The functions named gvof_* mirror the C interface of include/gvof.h one to
one; `GvofMesh` wraps a handle together with the torch-allocated device
workspace it lives in.  Every computation runs in the HIP kernels of
libgvof.so; when the library is missing this module raises instead of
falling back to anything else.
"""
from __future__ import annotations

import ctypes as C
import os

import numpy as np

HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.environ.get("GVOF_LIB_PATH") or os.path.join(HERE, "libgvof.so")

GVOF_OK, GVOF_E_ARG, GVOF_E_MESH, GVOF_E_NOMEM, GVOF_E_HIP, GVOF_E_GEOM, GVOF_E_LIMIT = 0, -1, -2, -3, -4, -5, -6
GVOF_SHAPE_SPHERE, GVOF_SHAPE_PLANE = 0, 1
GVOF_FLAG_NONE, GVOF_FLAG_EMFPA, GVOF_FLAG_NMFPA, GVOF_FLAG_LSFIR = 0, 1, 2, 4
GVOF_FLAG_LLCIR, GVOF_FLAG_ELCIR, GVOF_FLAG_CLCIR = 8, 16, 32
GVOF_FLAG_LSFIR_CAP = 64
RECON_FLAGS = {"lsgir": 0, "lsfir": GVOF_FLAG_LSFIR, "llcir": GVOF_FLAG_LLCIR, "elcir": GVOF_FLAG_ELCIR,
               "clcir": GVOF_FLAG_CLCIR}
GVOF_MAX_LSFIR_OUTER = 32
METHOD_FLAGS = {"fmfpa": GVOF_FLAG_NONE, "emfpa": GVOF_FLAG_EMFPA, "nmfpa": GVOF_FLAG_NMFPA}


class GvofError(RuntimeError):
    def __init__(self, code, msg):
        super().__init__(f"gvof error {code}: {msg}")
        self.code = code


class gvof_params(C.Structure):
    _fields_ = [("eps", C.c_double), ("beta", C.c_double), ("fmfpa_degen", C.c_double), ("flags", C.c_uint32),
                ("lsfir_outer", C.c_int32), ("lsfir_tol", C.c_double)]


class gvof_shape(C.Structure):
    _fields_ = [("kind", C.c_int32), ("p", C.c_double * 4)]


class gvof_launch_config(C.Structure):
    _fields_ = [("sweep_threads", C.c_int32), ("recon_threads", C.c_int32), ("prep_blocks", C.c_int32),
                ("pair_blocks_per_region", C.c_int32), ("filter_lanes", C.c_int32), ("staged_faces", C.c_int32),
                ("staged_pairs", C.c_int32), ("prep_lanes", C.c_int32), ("units_rank", C.c_int32)]

    def as_dict(self):
        return {k: getattr(self, k) for k, _ in self._fields_}


_lib = None
_vp = C.c_void_p


def lib() -> C.CDLL:
    global _lib
    if _lib is None:
        # One HIP runtime per process: torch ships its own libamdhip64 (SONAME
        # libamdhip64.so.7).  Loading torch first makes the dynamic linker bind
        # this library to that same runtime, so torch's device pointers and
        # streams are valid here.
        import torch  # noqa: F401
        if not os.path.exists(LIB_PATH):
            raise RuntimeError(f"{LIB_PATH} is not built: run `python -m paper_2111_01524_amd.build`")
        L = C.CDLL(LIB_PATH)
        L.gvof_params_default.argtypes = [C.POINTER(gvof_params)]
        L.gvof_params_default.restype = None
        L.gvof_mesh_create.argtypes = [C.POINTER(_vp), C.c_int32, _vp, _vp, _vp, C.c_int32, _vp, _vp, _vp, _vp,
                                       C.c_int32, C.POINTER(gvof_params)]
        L.gvof_mesh_workspace_bytes.argtypes = [_vp, C.POINTER(C.c_size_t)]
        L.gvof_mesh_bind.argtypes = [_vp, _vp, C.c_size_t, _vp]
        L.gvof_set_stream.argtypes = [_vp, _vp]
        L.gvof_mesh_destroy.argtypes = [_vp]
        L.gvof_mesh_destroy.restype = None
        L.gvof_mesh_sizes.argtypes = [_vp] + [C.POINTER(C.c_int32)] * 4
        L.gvof_get_geometry.argtypes = [_vp] * 8
        L.gvof_init_fraction.argtypes = [_vp, C.POINTER(gvof_shape), C.c_int32, _vp]
        L.gvof_reconstruct.argtypes = [_vp, _vp, _vp, _vp]
        L.gvof_get_tags.argtypes = [_vp] * 5
        L.gvof_advect_step.argtypes = [_vp, _vp, _vp, C.c_double, _vp, _vp, _vp, _vp, _vp]
        L.gvof_advect_step_static.argtypes = [_vp, _vp, _vp, C.c_double, _vp, _vp, _vp, _vp, _vp]
        L.gvof_interface_counts.argtypes = [_vp, C.POINTER(C.c_int32), C.POINTER(C.c_int32)]
        L.gvof_status.argtypes = [_vp]
        L.gvof_last_error.argtypes = [_vp]
        L.gvof_last_error.restype = C.c_char_p
        L.gvof_work_totals.argtypes = [_vp, C.POINTER(C.c_int64), C.POINTER(C.c_int64)]
        L.gvof_profile_enable.argtypes = [_vp, C.c_uint32]
        L.gvof_profile_read.argtypes = [_vp, C.c_int32, C.POINTER(C.c_double), C.POINTER(C.c_int64)]
        L.gvof_kernel_name.argtypes = [C.c_int32]
        L.gvof_kernel_name.restype = C.c_char_p
        L.gvof_batch_create.argtypes = [C.POINTER(_vp), C.c_int32, C.POINTER(_vp)]
        L.gvof_batch_offsets.argtypes = [_vp, C.POINTER(C.c_int32), _vp, _vp, _vp]
        L.gvof_batch_init_fraction.argtypes = [_vp, C.POINTER(gvof_shape), C.c_int32, _vp]
        L.gvof_batch_step.argtypes = [_vp] * 6
        L.gvof_graph_capture.argtypes = [_vp] * 6
        L.gvof_graph_launch.argtypes = [_vp]
        L.gvof_get_launch_config.argtypes = [_vp, C.POINTER(gvof_launch_config)]
        L.gvof_set_launch_config.argtypes = [_vp, C.POINTER(gvof_launch_config)]
        L.gvof_autotune.argtypes = [_vp] * 7 + [C.c_int32, C.POINTER(gvof_launch_config), C.POINTER(C.c_double)]
        for name in ("gvof_mesh_create", "gvof_mesh_workspace_bytes", "gvof_mesh_bind", "gvof_set_stream",
                     "gvof_mesh_sizes", "gvof_get_geometry", "gvof_init_fraction", "gvof_reconstruct",
                     "gvof_get_tags", "gvof_advect_step", "gvof_advect_step_static", "gvof_interface_counts",
                     "gvof_status", "gvof_work_totals", "gvof_profile_enable", "gvof_profile_read", "gvof_batch_create",
                     "gvof_batch_offsets", "gvof_batch_init_fraction", "gvof_batch_step", "gvof_graph_capture",
                     "gvof_graph_launch", "gvof_get_launch_config", "gvof_set_launch_config", "gvof_autotune"):
            getattr(L, name).restype = C.c_int
        _lib = L
    return _lib


def exported_symbols():
    """Names of every function include/gvof.h declares (for the load check)."""
    return ["gvof_params_default", "gvof_mesh_create", "gvof_mesh_workspace_bytes", "gvof_mesh_bind",
            "gvof_set_stream", "gvof_mesh_destroy", "gvof_mesh_sizes", "gvof_get_geometry", "gvof_init_fraction",
            "gvof_reconstruct", "gvof_get_tags", "gvof_advect_step", "gvof_interface_counts", "gvof_status",
            "gvof_last_error", "gvof_work_totals", "gvof_profile_enable", "gvof_profile_read", "gvof_kernel_name",
            "gvof_batch_create", "gvof_batch_offsets", "gvof_batch_init_fraction", "gvof_batch_step",
            "gvof_graph_capture", "gvof_graph_launch", "gvof_get_launch_config", "gvof_set_launch_config",
            "gvof_autotune", "gvof_advect_step_static"]


def _check(code, handle=None):
    if code != GVOF_OK:
        msg = lib().gvof_last_error(handle)
        raise GvofError(code, msg.decode() if msg else "")


def _ptr(t):
    """Device pointer of a torch tensor (None -> NULL)."""
    if t is None:
        return None
    if not t.is_contiguous():
        raise ValueError("tensor must be contiguous")
    return t.data_ptr()


def _np_ptr(a, dtype):
    a = np.ascontiguousarray(a, dtype=dtype)
    return a, a.ctypes.data


# ------------------------------------------------------------------ C-named wrappers
def gvof_params_default() -> gvof_params:
    p = gvof_params()
    lib().gvof_params_default(C.byref(p))
    return p


def gvof_mesh_create(vx, vy, vz, fv_ptr, fv_idx, owner, neigh, nc, params: gvof_params | None = None):
    keep = []
    args = []
    for a, dt in ((vx, np.float64), (vy, np.float64), (vz, np.float64), (fv_ptr, np.int32), (fv_idx, np.int32),
                  (owner, np.int32), (neigh, np.int32)):
        arr, p = _np_ptr(a, dt)
        keep.append(arr)
        args.append(p)
    h = _vp()
    nv, nf = keep[0].shape[0], keep[5].shape[0]
    prm = params if params is not None else gvof_params_default()
    code = lib().gvof_mesh_create(C.byref(h), nv, args[0], args[1], args[2], nf, args[3], args[4], args[5], args[6],
                                  int(nc), C.byref(prm))
    _check(code, None)
    return h


def gvof_mesh_workspace_bytes(h) -> int:
    n = C.c_size_t()
    _check(lib().gvof_mesh_workspace_bytes(h, C.byref(n)), h)
    return int(n.value)


def gvof_mesh_bind(h, workspace, stream_ptr):
    _check(lib().gvof_mesh_bind(h, _ptr(workspace), workspace.numel(), stream_ptr), h)


def gvof_set_stream(h, stream_ptr):
    _check(lib().gvof_set_stream(h, stream_ptr), h)


def gvof_mesh_destroy(h):
    lib().gvof_mesh_destroy(h)


def gvof_mesh_sizes(h):
    v = [C.c_int32() for _ in range(4)]
    _check(lib().gvof_mesh_sizes(h, *[C.byref(x) for x in v]), h)
    return tuple(x.value for x in v)


def gvof_get_geometry(h, S=None, fc=None, V=None, cc=None, bbmin=None, bbmax=None, isbox=None):
    _check(lib().gvof_get_geometry(h, _ptr(S), _ptr(fc), _ptr(V), _ptr(cc), _ptr(bbmin), _ptr(bbmax), _ptr(isbox)), h)


def gvof_init_fraction(h, kind: int, params, n_div: int, F_out):
    sh = gvof_shape()
    sh.kind = kind
    for i in range(4):
        sh.p[i] = float(params[i])
    _check(lib().gvof_init_fraction(h, C.byref(sh), int(n_div), _ptr(F_out)), h)


def gvof_reconstruct(h, F_inout, cell_tag_out=None, plane_out=None):
    _check(lib().gvof_reconstruct(h, _ptr(F_inout), _ptr(cell_tag_out), _ptr(plane_out)), h)


def gvof_get_tags(h, node_value=None, node_tag=None, face_tag=None, cell_tag=None):
    _check(lib().gvof_get_tags(h, _ptr(node_value), _ptr(node_tag), _ptr(face_tag), _ptr(cell_tag)), h)


def gvof_advect_step(h, u_face, u_vert, dt, F_in, F_out, upwind_out=None, vd_out=None, vf_out=None):
    _check(lib().gvof_advect_step(h, _ptr(u_face), _ptr(u_vert), float(dt), _ptr(F_in), _ptr(F_out),
                                  _ptr(upwind_out), _ptr(vd_out), _ptr(vf_out)), h)


def gvof_advect_step_static(h, u_face, u_vert, dt, F_in, F_out, upwind_out=None, vd_out=None, vf_out=None):
    _check(lib().gvof_advect_step_static(h, _ptr(u_face), _ptr(u_vert), float(dt), _ptr(F_in), _ptr(F_out),
                                         _ptr(upwind_out), _ptr(vd_out), _ptr(vf_out)), h)


def gvof_interface_counts(h):
    a, b = C.c_int32(), C.c_int32()
    _check(lib().gvof_interface_counts(h, C.byref(a), C.byref(b)), h)
    return a.value, b.value


def gvof_status(h):
    code = lib().gvof_status(h)
    _check(code, h)
    return code


GVOF_NUM_KERNELS = 18


def gvof_work_totals(h):
    a, b = C.c_int64(), C.c_int64()
    _check(lib().gvof_work_totals(h, C.byref(a), C.byref(b)), h)
    return a.value, b.value


def gvof_profile_enable(h, mask: int):
    _check(lib().gvof_profile_enable(h, mask), h)


def gvof_profile_read(h):
    ms = (C.c_double * GVOF_NUM_KERNELS)()
    n = (C.c_int64 * GVOF_NUM_KERNELS)()
    _check(lib().gvof_profile_read(h, GVOF_NUM_KERNELS, ms, n), h)
    return {gvof_kernel_name(k): (ms[k], n[k]) for k in range(GVOF_NUM_KERNELS)}


def gvof_kernel_name(k: int) -> str:
    return lib().gvof_kernel_name(k).decode()


def gvof_batch_create(parts):
    arr = (_vp * len(parts))(*[p.value if isinstance(p, _vp) else p for p in parts])
    h = _vp()
    _check(lib().gvof_batch_create(C.byref(h), len(parts), arr), None)
    return h


def gvof_batch_offsets(h):
    n = C.c_int32()
    _check(lib().gvof_batch_offsets(h, C.byref(n), None, None, None), h)
    vo, fo, co = (np.zeros(n.value + 1, np.int32) for _ in range(3))
    _check(lib().gvof_batch_offsets(h, C.byref(n), vo.ctypes.data, fo.ctypes.data, co.ctypes.data), h)
    return vo, fo, co


def gvof_batch_init_fraction(h, shapes, n_div: int, F_out):
    """shapes: list of (kind, (p0, p1, p2, p3)), one per problem."""
    arr = (gvof_shape * len(shapes))()
    for i, (kind, prm) in enumerate(shapes):
        arr[i].kind = kind
        for j in range(4):
            arr[i].p[j] = float(prm[j])
    _check(lib().gvof_batch_init_fraction(h, arr, int(n_div), _ptr(F_out)), h)


def gvof_batch_step(h, u_face, u_vert, dt, active, F):
    _check(lib().gvof_batch_step(h, _ptr(u_face), _ptr(u_vert), _ptr(dt), _ptr(active), _ptr(F)), h)


def gvof_graph_capture(h, u_face, u_vert, dt, active, F):
    _check(lib().gvof_graph_capture(h, _ptr(u_face), _ptr(u_vert), _ptr(dt), _ptr(active), _ptr(F)), h)


def gvof_graph_launch(h):
    _check(lib().gvof_graph_launch(h), h)


def gvof_get_launch_config(h) -> gvof_launch_config:
    c = gvof_launch_config()
    _check(lib().gvof_get_launch_config(h, C.byref(c)), h)
    return c


def gvof_set_launch_config(h, cfg: gvof_launch_config):
    _check(lib().gvof_set_launch_config(h, C.byref(cfg)), h)


def gvof_autotune(h, u_face, u_vert, dt, active, F, F_save, reps: int):
    c = gvof_launch_config()
    ms = C.c_double()
    _check(lib().gvof_autotune(h, _ptr(u_face), _ptr(u_vert), _ptr(dt), _ptr(active), _ptr(F), _ptr(F_save),
                               int(reps), C.byref(c), C.byref(ms)), h)
    return c, ms.value


def gvof_last_error(h=None) -> str:
    m = lib().gvof_last_error(h)
    return m.decode() if m else ""


# ------------------------------------------------------------------ convenience wrapper
def _with_method(params, method: str, recon: str = "lsgir", lsfir_outer: int | None = None,
                 lsfir_tol: float | None = None, lsfir_cap: bool = False):
    """params with the flags of a flux polyhedron method and of a
    reconstruction set ("fmfpa" / "lsgir": unchanged); lsfir_outer and
    lsfir_tol, when given, set the LSFIR outer passes and stopping angle;
    lsfir_cap sets GVOF_FLAG_LSFIR_CAP."""
    if method not in METHOD_FLAGS:
        raise ValueError(f"unknown flux polyhedron method {method!r}")
    if recon not in RECON_FLAGS:
        raise ValueError(f"unknown reconstruction {recon!r}")
    if method == "fmfpa" and recon == "lsgir":
        return params
    params = params if params is not None else gvof_params_default()
    params.flags |= METHOD_FLAGS[method] | RECON_FLAGS[recon]
    if recon == "lsfir":
        if lsfir_outer is not None:
            params.lsfir_outer = int(lsfir_outer)
        if lsfir_tol is not None:
            params.lsfir_tol = float(lsfir_tol)
        if lsfir_cap:
            params.flags |= GVOF_FLAG_LSFIR_CAP
    return params


class GvofMesh:
    """A mesh handle bound to a torch-allocated device workspace.

    method "emfpa" / "nmfpa" sets GVOF_FLAG_EMFPA / GVOF_FLAG_NMFPA in the
    parameters (the flux polyhedron method), recon "lsfir" / "llcir" /
    "elcir" / "clcir" sets that reconstruction's flag (LSFIR with lsfir_outer
    passes, lsfir_tol and the optional weight floor lsfir_cap when given);
    "fmfpa" and "lsgir" leave the flags as given.
    """

    def __init__(self, mesh, device="cuda", params: gvof_params | None = None, stream=None, handle=None,
                 method: str = "fmfpa", recon: str = "lsgir", lsfir_outer: int | None = None,
                 lsfir_tol: float | None = None, lsfir_cap: bool = False):
        import torch
        params = _with_method(params, method, recon, lsfir_outer, lsfir_tol, lsfir_cap)
        self.torch = torch
        self.device = torch.device(device)
        self.mesh = mesh
        if handle is None:
            handle = gvof_mesh_create(mesh.vx, mesh.vy, mesh.vz, mesh.fv_ptr, mesh.fv_idx, mesh.owner, mesh.neigh,
                                      mesh.nc, params)
        self.h = handle
        self.nv, self.nf, self.nc, _ = gvof_mesh_sizes(self.h)
        self.ws_bytes = gvof_mesh_workspace_bytes(self.h)
        self.workspace = torch.empty(self.ws_bytes + 256, dtype=torch.uint8, device=self.device)
        off = (-self.workspace.data_ptr()) % 256
        self.ws_view = self.workspace[off:off + self.ws_bytes]
        self.stream = stream if stream is not None else torch.cuda.current_stream(self.device)
        gvof_mesh_bind(self.h, self.ws_view, self.stream.cuda_stream)

    def close(self):
        if getattr(self, "h", None):
            gvof_mesh_destroy(self.h)
            self.h = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass

    # -- helpers
    def dzeros(self, *shape, dtype=None):
        return self.torch.zeros(*shape, dtype=dtype or self.torch.float64, device=self.device)

    def geometry(self):
        t = self.torch
        out = dict(S=self.dzeros(3, self.nf), fc=self.dzeros(3, self.nf), V=self.dzeros(self.nc),
                   cc=self.dzeros(3, self.nc), bbmin=self.dzeros(3, self.nc), bbmax=self.dzeros(3, self.nc),
                   isbox=self.dzeros(self.nc, dtype=t.int8))
        gvof_get_geometry(self.h, out["S"], out["fc"], out["V"], out["cc"], out["bbmin"], out["bbmax"], out["isbox"])
        return out

    def init_fraction(self, shape: str, params, n_div: int = 10, F_out=None):
        F = F_out if F_out is not None else self.dzeros(self.nc)
        gvof_init_fraction(self.h, {"sphere": GVOF_SHAPE_SPHERE, "plane": GVOF_SHAPE_PLANE}[shape], params, n_div, F)
        return F

    def reconstruct(self, F, want_tags=False, want_planes=False):
        t = self.torch
        tags = self.dzeros(self.nc, dtype=t.int8) if want_tags else None
        planes = self.dzeros(4, self.nc) if want_planes else None
        gvof_reconstruct(self.h, F, tags, planes)
        return tags, planes

    def tags(self):
        t = self.torch
        out = dict(node_value=self.dzeros(self.nv), node=self.dzeros(self.nv, dtype=t.int8),
                   face=self.dzeros(self.nf, dtype=t.int8), cell=self.dzeros(self.nc, dtype=t.int8))
        gvof_get_tags(self.h, out["node_value"], out["node"], out["face"], out["cell"])
        return out

    def advect_step(self, u_face, u_vert, dt, F_in, F_out, want_faces=False):
        t = self.torch
        up = vd = vf = None
        if want_faces:
            up = self.dzeros(self.nf, dtype=t.int32)
            vd = self.dzeros(self.nf)
            vf = self.dzeros(self.nf)
        gvof_advect_step(self.h, u_face, u_vert, dt, F_in, F_out, up, vd, vf)
        return up, vd, vf

    def advect_step_static(self, u_face, u_vert, dt, F_in, F_out, up=None, vd=None, vf=None):
        """gvof_advect_step_static: the step with its staging in the library's
        static array; optional outputs are caller-allocated device tensors."""
        gvof_advect_step_static(self.h, u_face, u_vert, dt, F_in, F_out, up, vd, vf)

    def interface_counts(self):
        return gvof_interface_counts(self.h)

    def status(self):
        return gvof_status(self.h)


class GvofBatch(GvofMesh):
    """Independent problems advanced together: the handle of their disjoint
    union (gvof_batch_create), bound to one torch-allocated workspace.
    `offsets` gives each problem's vertex / face / cell ranges."""

    def __init__(self, meshes, device="cuda", params: gvof_params | None = None, stream=None, parts=None,
                 method: str = "fmfpa", recon: str = "lsgir", lsfir_outer: int | None = None):
        """parts: optional handles already made by gvof_mesh_create for these
        meshes (taken over and destroyed here).  method, recon and lsfir_outer
        as for GvofMesh."""
        params = _with_method(params, method, recon, lsfir_outer)
        parts = list(parts) if parts is not None else []
        try:
            for m in meshes[len(parts):]:
                parts.append(gvof_mesh_create(m.vx, m.vy, m.vz, m.fv_ptr, m.fv_idx, m.owner, m.neigh, m.nc, params))
            h = gvof_batch_create(parts)
        finally:
            for p in parts:
                gvof_mesh_destroy(p)
        super().__init__(None, device, params, stream, handle=h)
        self.nprob = len(meshes)
        self.vert_off, self.face_off, self.cell_off = gvof_batch_offsets(self.h)

    def init_fraction_each(self, shapes, n_div: int = 10, F_out=None):
        """shapes: one ("sphere" | "plane", params) per problem."""
        F = F_out if F_out is not None else self.dzeros(self.nc)
        kinds = {"sphere": GVOF_SHAPE_SPHERE, "plane": GVOF_SHAPE_PLANE}
        gvof_batch_init_fraction(self.h, [(kinds[k], p) for k, p in shapes], n_div, F)
        return F

    def step(self, u_face, u_vert, dt, active, F):
        gvof_batch_step(self.h, u_face, u_vert, dt, active, F)

    def capture(self, u_face, u_vert, dt, active, F):
        gvof_graph_capture(self.h, u_face, u_vert, dt, active, F)

    def replay(self):
        gvof_graph_launch(self.h)

    def autotune(self, u_face, u_vert, dt, active, F, reps: int = 3):
        scratch = self.torch.empty_like(F)
        return gvof_autotune(self.h, u_face, u_vert, dt, active, F, scratch, reps)

    def cells(self, q):
        return slice(int(self.cell_off[q]), int(self.cell_off[q + 1]))
