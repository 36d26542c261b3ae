"""ctypes front of the oracle library (test infrastructure only).

Arrays on this side are numpy float64 of shape (ncell, nvel), the oracle's
own layout (cell index fastest in x, velocity index fastest in p1).
"""
from __future__ import annotations

import ctypes as C

import numpy as np

from . import build as _build

_BODY = {"none": 0, "circle": 1, "ellipse": 2, "cavity": 3, "halfplane": 4, "sphere": 5, "vane": 6}
_MOTION = {"fixed": 0, "free_rotation": 1, "imposed": 2}


class OracleError(RuntimeError):
    pass


class _Cfg(C.Structure):
    _fields_ = [("dim", C.c_int), ("n", C.c_int * 3), ("lo", C.c_double * 3),
                ("hi", C.c_double * 3), ("nv", C.c_int), ("vmin", C.c_double),
                ("vmax", C.c_double), ("kn", C.c_double), ("lref", C.c_double),
                ("cfl", C.c_double), ("dt", C.c_double), ("inflow", C.c_double * 5),
                ("body_kind", C.c_int), ("center", C.c_double * 3),
                ("axes", C.c_double * 3), ("theta", C.c_double), ("t_wall", C.c_double),
                ("mass", C.c_double), ("inertia", C.c_double), ("motion", C.c_int),
                ("vel", C.c_double * 3), ("omega", C.c_double), ("maxwellian", C.c_int),
                ("scheme", C.c_int), ("model", C.c_int), ("prandtl", C.c_double),
                ("amr_depth", C.c_int), ("amr_band", C.c_double)]


def cfg_struct(cfg) -> _Cfg:
    b = cfg.body
    s = _Cfg()
    s.dim = cfg.dim
    s.n[:] = list(cfg.n)
    s.lo[:] = list(cfg.lo)
    s.hi[:] = list(cfg.hi)
    s.nv = cfg.nv
    s.vmin, s.vmax = cfg.vmin, cfg.vmax
    s.kn, s.lref, s.cfl, s.dt = cfg.kn, cfg.lref, cfg.cfl, cfg.dt
    s.inflow[:] = list(cfg.inflow)
    s.body_kind = _BODY[b.kind]
    s.center[:] = list(b.center)
    s.axes[:] = list(b.axes)
    s.theta, s.t_wall, s.mass, s.inertia = b.theta, b.t_wall, b.mass, b.inertia
    s.motion = _MOTION[b.motion]
    s.vel[:] = list(b.vel)
    s.omega = b.omega
    s.maxwellian = {"direct": 0, "conservative": 1}[getattr(cfg, "maxwellian", "direct")]
    s.scheme = {"explicit": 0, "imex": 1}[getattr(cfg, "scheme", "explicit")]
    s.model = {"bgk": 0, "shakhov": 1}[getattr(cfg, "model", "bgk")]
    s.prandtl = getattr(cfg, "prandtl", 2.0 / 3.0)
    s.amr_depth = getattr(cfg, "amr_depth", 0)
    s.amr_band = getattr(cfg, "amr_band", 0.0)
    return s


_lib = None


def lib():
    global _lib
    if _lib is None:
        _lib = C.CDLL(_build.ensure_built())
        P = C.c_void_p
        _lib.orc2d_create.argtypes = [C.POINTER(_Cfg), C.POINTER(P)]
        _lib.orc2d_destroy.argtypes = [P]
        _lib.orc2d_dt.argtypes = [P]
        _lib.orc2d_dt.restype = C.c_double
        for name in ("orc2d_velocity", "orc2d_body_state"):
            getattr(_lib, name).argtypes = [P, P]
        _lib.orc2d_geometry.argtypes = [P] + [P] * 13
        _lib.orc2d_init.argtypes = [P, P, P]
        _lib.orc2d_merge.argtypes = [P, P, P]
        _lib.orc2d_update_cells.argtypes = [P, P, P, P, C.c_int, P, P]
        _lib.orc2d_step.argtypes = [P, P, P, P, P, P]
        _lib.orc2d_force.argtypes = [P, P, P, P]
        _lib.orc2d_moments.argtypes = [P, P, P, P]
        _lib.orc_threads.restype = C.c_int
        _lib.orc_set_threads.argtypes = [C.c_int]
        _lib.orc_set_threads.restype = None
        _lib.orc2d_adjoint.argtypes = [P, C.c_int, C.c_int, P]
        _lib.orc2d_equilibrium.argtypes = [P, P, P, P]
        _lib.orc2d_equilibrium_values.argtypes = [P, P, P, P, P]
    return _lib


def threads() -> int:
    return lib().orc_threads()


def set_threads(n: int) -> None:
    lib().orc_set_threads(int(n))


def _p(a):
    return a.ctypes.data_as(C.c_void_p)


class Oracle2D:
    """Reduced 2D model: state (f, g), each (ncell, N*N) float64."""

    def __init__(self, cfg):
        assert cfg.dim == 2
        self.cfg = cfg
        self._s = cfg_struct(cfg)
        h = C.c_void_p()
        st = lib().orc2d_create(C.byref(self._s), C.byref(h))
        if st != 0:
            raise OracleError(f"oracle create failed with status {st}")
        self._h = h
        self.nx, self.ny = cfg.n[0], cfg.n[1]
        self.ncell = self.nx * self.ny
        self.N = cfg.nv
        self.nvel = cfg.nv * cfg.nv

    def __del__(self):
        h = getattr(self, "_h", None)
        if h is not None and h.value:
            lib().orc2d_destroy(h)
            self._h = None

    @property
    def dt(self) -> float:
        return lib().orc2d_dt(self._h)

    def velocity(self):
        v = np.zeros(self.N)
        lib().orc2d_velocity(self._h, _p(v))
        return v

    def body_state(self):
        s = np.zeros(6)
        lib().orc2d_body_state(self._h, _p(s))
        return s

    def geometry(self):
        n = self.ncell
        out = {"type": np.zeros(n, np.int32), "master": np.zeros(n, np.int32)}
        names = ["lxm", "lxp", "lym", "lyp", "lw", "nwx", "nwy", "rwx", "rwy", "sbar", "scv"]
        for k in names:
            out[k] = np.zeros(n)
        lib().orc2d_geometry(self._h, _p(out["type"]), _p(out["master"]),
                             *[_p(out[k]) for k in names])
        return out

    def _zeros(self):
        return np.zeros((self.ncell, self.nvel))

    def init(self):
        f, g = self._zeros(), self._zeros()
        lib().orc2d_init(self._h, _p(f), _p(g))
        return f, g

    def merge(self, f, g):
        f = np.ascontiguousarray(f, dtype=np.float64).copy()
        g = np.ascontiguousarray(g, dtype=np.float64).copy()
        lib().orc2d_merge(self._h, _p(f), _p(g))
        return f, g

    def update_cells(self, fm, gm, cells):
        cells = np.ascontiguousarray(cells, dtype=np.int32)
        fo = np.zeros((cells.size, self.nvel))
        go = np.zeros((cells.size, self.nvel))
        lib().orc2d_update_cells(self._h, _p(np.ascontiguousarray(fm)),
                                 _p(np.ascontiguousarray(gm)), _p(cells),
                                 int(cells.size), _p(fo), _p(go))
        return fo, go

    def step(self, f, g):
        """One step; returns (f1, g1, diag) with diag = (Fx, Fy, torque, mass) of f^n."""
        f = np.ascontiguousarray(f, dtype=np.float64)
        g = np.ascontiguousarray(g, dtype=np.float64)
        fo, go = self._zeros(), self._zeros()
        d = np.zeros(4)
        st = lib().orc2d_step(self._h, _p(f), _p(g), _p(fo), _p(go), _p(d))
        if st != 0:
            raise OracleError(f"oracle step failed with status {st}")
        return fo, go, d

    def run(self, f, g, nsteps):
        diags = []
        for _ in range(nsteps):
            f, g, d = self.step(f, g)
            diags.append(d)
        return f, g, np.array(diags).reshape(-1, 4)

    def force(self, fm, gm):
        d = np.zeros(4)
        lib().orc2d_force(self._h, _p(np.ascontiguousarray(fm)), _p(np.ascontiguousarray(gm)), _p(d))
        return d

    def adjoint(self, nsteps, objective="drag"):
        """J and dJ/d(T_w, Kn, u_x, u_y) after nsteps from the inflow Maxwellian."""
        out = np.zeros(5)
        st = lib().orc2d_adjoint(self._h, int(nsteps), 0 if objective == "drag" else 1, _p(out))
        if st != 0:
            raise OracleError(f"oracle adjoint failed with status {st}")
        return out[0], out[1:]

    def equilibrium(self, f1, g1):
        """(rho, ux, uy, T) of the relaxation for one cell's (f, g) and the
        Newton iterations taken (0: direct moments)."""
        out = np.zeros(4)
        it = lib().orc2d_equilibrium(self._h, _p(np.ascontiguousarray(f1, dtype=np.float64)),
                                     _p(np.ascontiguousarray(g1, dtype=np.float64)), _p(out))
        return out, it

    def equilibrium_values(self, f1, g1):
        """(f_eq, g_eq) of one cell's (f, g) at every velocity."""
        fe, ge = np.zeros(self.nvel), np.zeros(self.nvel)
        lib().orc2d_equilibrium_values(self._h, _p(np.ascontiguousarray(f1, dtype=np.float64)),
                                       _p(np.ascontiguousarray(g1, dtype=np.float64)), _p(fe), _p(ge))
        return fe, ge

    def moments(self, f, g):
        out = np.zeros((self.ncell, 9))
        lib().orc2d_moments(self._h, _p(np.ascontiguousarray(f)), _p(np.ascontiguousarray(g)), _p(out))
        return out


def _lib3():
    L = lib()
    if not getattr(L, "_has3", False):
        P = C.c_void_p
        L.orc3d_create.argtypes = [C.POINTER(_Cfg), C.POINTER(P)]
        L.orc3d_destroy.argtypes = [P]
        L.orc3d_dt.argtypes = [P]
        L.orc3d_dt.restype = C.c_double
        L.orc3d_velocity.argtypes = [P, P]
        L.orc3d_geometry.argtypes = [P] + [P] * 8
        L.orc3d_init.argtypes = [P, P]
        L.orc3d_merge.argtypes = [P, P]
        L.orc3d_update_cells.argtypes = [P, P, P, C.c_int, P]
        L.orc3d_step.argtypes = [P, P, P, P]
        L.orc3d_force.argtypes = [P, P, P]
        L.orc3d_moments.argtypes = [P, P, P]
        L.orc3d_equilibrium.argtypes = [P, P, P]
        L.orc3d_equilibrium_values.argtypes = [P, P, P]
        L._has3 = True
    return L


class Oracle3D:
    """Three-dimensional model: state F of shape (ncell, N**3)."""

    def __init__(self, cfg):
        assert cfg.dim == 3
        self.cfg = cfg
        self._s = cfg_struct(cfg)
        h = C.c_void_p()
        st = _lib3().orc3d_create(C.byref(self._s), C.byref(h))
        if st != 0:
            raise OracleError(f"oracle create failed with status {st}")
        self._h = h
        self.nx, self.ny, self.nz = cfg.n
        self.ncell = self.nx * self.ny * self.nz
        self.N = cfg.nv
        self.nvel = cfg.nv ** 3

    def __del__(self):
        h = getattr(self, "_h", None)
        if h is not None and h.value:
            _lib3().orc3d_destroy(h)
            self._h = None

    @property
    def dt(self) -> float:
        return _lib3().orc3d_dt(self._h)

    def velocity(self):
        v = np.zeros(self.N)
        _lib3().orc3d_velocity(self._h, _p(v))
        return v

    def geometry(self):
        n = self.ncell
        out = {"type": np.zeros(n, np.int32), "master": np.zeros(n, np.int32),
               "S": np.zeros((n, 6)), "sw": np.zeros(n), "nw": np.zeros((n, 3)),
               "rw": np.zeros((n, 3)), "vbar": np.zeros(n), "vcv": np.zeros(n)}
        _lib3().orc3d_geometry(self._h, *[_p(out[k]) for k in
                                          ("type", "master", "S", "sw", "nw", "rw", "vbar", "vcv")])
        return out

    def init(self):
        F = np.zeros((self.ncell, self.nvel))
        _lib3().orc3d_init(self._h, _p(F))
        return F

    def merge(self, F):
        F = np.ascontiguousarray(F, dtype=np.float64).copy()
        _lib3().orc3d_merge(self._h, _p(F))
        return F

    def update_cells(self, Fm, cells):
        cells = np.ascontiguousarray(cells, dtype=np.int32)
        out = np.zeros((cells.size, self.nvel))
        _lib3().orc3d_update_cells(self._h, _p(np.ascontiguousarray(Fm)), _p(cells),
                                   int(cells.size), _p(out))
        return out

    def step(self, F):
        """One step; returns (F1, diag) with diag = (Fx, Fy, Fz, mass) of F^n."""
        F = np.ascontiguousarray(F, dtype=np.float64)
        Fo = np.zeros_like(F)
        d = np.zeros(4)
        st = _lib3().orc3d_step(self._h, _p(F), _p(Fo), _p(d))
        if st != 0:
            raise OracleError(f"oracle step failed with status {st}")
        return Fo, d

    def run(self, F, nsteps):
        diags = []
        for _ in range(nsteps):
            F, d = self.step(F)
            diags.append(d)
        return F, np.array(diags).reshape(-1, 4)

    def force(self, Fm):
        d = np.zeros(4)
        _lib3().orc3d_force(self._h, _p(np.ascontiguousarray(Fm)), _p(d))
        return d

    def equilibrium(self, F1):
        """(rho, ux, uy, uz, T) of the relaxation for one cell's F and the
        Newton iterations taken (0: direct moments)."""
        out = np.zeros(5)
        it = _lib3().orc3d_equilibrium(self._h, _p(np.ascontiguousarray(F1, dtype=np.float64)), _p(out))
        return out, it

    def equilibrium_values(self, F1):
        """F_eq of one cell's F at every velocity."""
        Fe = np.zeros(self.nvel)
        _lib3().orc3d_equilibrium_values(self._h, _p(np.ascontiguousarray(F1, dtype=np.float64)), _p(Fe))
        return Fe

    def moments(self, F):
        out = np.zeros((self.ncell, 14))
        _lib3().orc3d_moments(self._h, _p(np.ascontiguousarray(F)), _p(out))
        return out


def _lib3a():
    L = _lib3()
    if not getattr(L, "_has3a", False):
        P = C.c_void_p
        L.orc3a_create.argtypes = [C.POINTER(_Cfg), C.POINTER(P)]
        L.orc3a_destroy.argtypes = [P]
        L.orc3a_dt.argtypes = [P]
        L.orc3a_dt.restype = C.c_double
        L.orc3a_nleaf.argtypes = [P]
        L.orc3a_nface.argtypes = [P]
        L.orc3a_velocity.argtypes = [P, P]
        L.orc3a_leaves.argtypes = [P] + [P] * 8
        L.orc3a_faces.argtypes = [P] + [P] * 4
        L.orc3a_init.argtypes = [P, P]
        L.orc3a_merge.argtypes = [P, P]
        L.orc3a_step.argtypes = [P, P, P, P]
        L.orc3a_adapt.argtypes = [P]
        L.orc3a_remap.argtypes = [P, P, P]
        L.orc3a_body.argtypes = [P, P]
        L.orc3a_levelset.argtypes = [P] + [C.c_double] * 4
        L.orc3a_levelset.restype = C.c_double
        L._has3a = True
    return L


class Oracle3A:
    """3D octree mesh (Section 5.1): state F of shape (nleaf, N**3), leaves in
    Z-order.  With a turning body the mesh follows the body: every step
    returns the state on the mesh of the new angle (nleaf may change)."""

    def __init__(self, cfg):
        assert cfg.dim == 3
        self.cfg = cfg
        self._s = cfg_struct(cfg)
        h = C.c_void_p()
        st = _lib3a().orc3a_create(C.byref(self._s), C.byref(h))
        if st != 0:
            raise OracleError(f"oracle create failed with status {st}")
        self._h = h
        self.nleaf = _lib3a().orc3a_nleaf(h)
        self.nface = _lib3a().orc3a_nface(h)
        self.N = cfg.nv
        self.nvel = cfg.nv ** 3

    def __del__(self):
        h = getattr(self, "_h", None)
        if h is not None and h.value:
            _lib3a().orc3a_destroy(h)
            self._h = None

    @property
    def dt(self) -> float:
        return _lib3a().orc3a_dt(self._h)

    def velocity(self):
        v = np.zeros(self.N)
        _lib3a().orc3a_velocity(self._h, _p(v))
        return v

    def leaves(self):
        n = self.nleaf
        out = {"lvl": np.zeros(n, np.int32), "ijk": np.zeros((n, 3), np.int32),
               "type": np.zeros(n, np.int32), "master": np.zeros(n, np.int32),
               "vbar": np.zeros(n), "vcv": np.zeros(n), "sw": np.zeros(n), "S": np.zeros((n, 6))}
        _lib3a().orc3a_leaves(self._h, *[_p(out[k]) for k in
                                         ("lvl", "ijk", "type", "master", "vbar", "vcv", "sw", "S")])
        return out

    def faces(self):
        out = {"ptr": np.zeros(self.nleaf + 1, np.int32), "nb": np.zeros(self.nface, np.int32),
               "dir": np.zeros(self.nface, np.int32), "area": np.zeros(self.nface)}
        _lib3a().orc3a_faces(self._h, *[_p(out[k]) for k in ("ptr", "nb", "dir", "area")])
        return out

    def init(self):
        F = np.zeros((self.nleaf, self.nvel))
        _lib3a().orc3a_init(self._h, _p(F))
        return F

    def merge(self, F):
        F = np.ascontiguousarray(F, dtype=np.float64).copy()
        _lib3a().orc3a_merge(self._h, _p(F))
        return F

    @property
    def moving(self) -> bool:
        return self.cfg.body.motion != "fixed" and self.cfg.body.kind != "none"

    def body(self):
        """(angle, angular velocity) of the body."""
        out = np.zeros(2)
        _lib3a().orc3a_body(self._h, _p(out))
        return out

    def levelset(self, th, x, y, z) -> float:
        """Signed distance to the body turned by th (gas side positive)."""
        return _lib3a().orc3a_levelset(self._h, th, x, y, z)

    def step_on_mesh(self, F):
        """Section 5 steps 1-7 on the current mesh (no adaptation): the state
        at t^{n+1} on the same leaves, and diag."""
        F = np.ascontiguousarray(F, dtype=np.float64)
        Fo = np.zeros_like(F)
        d = np.zeros(4)
        st = _lib3a().orc3a_step(self._h, _p(F), _p(Fo), _p(d))
        if st != 0:
            raise OracleError(f"oracle step failed with status {st}")
        return Fo, d

    def adapt(self, F):
        """Rebuild the mesh for the current body angle and carry F over."""
        st = _lib3a().orc3a_adapt(self._h)
        if st != 0:
            raise OracleError(f"oracle mesh adaptation failed with status {st}")
        self.nleaf = _lib3a().orc3a_nleaf(self._h)
        self.nface = _lib3a().orc3a_nface(self._h)
        F = np.ascontiguousarray(F, dtype=np.float64)
        F1 = np.zeros((self.nleaf, self.nvel))
        _lib3a().orc3a_remap(self._h, _p(F), _p(F1))
        return F1

    def step(self, F):
        """One step; returns (F1, diag) with diag = (Fx, Fy, Fz, mass) of F^n
        (turning body: (Fx, Fy, torque about z, mass), and F1 on the mesh
        adapted to the new angle)."""
        Fo, d = self.step_on_mesh(F)
        if self.moving:
            Fo = self.adapt(Fo)
        return Fo, d

    def run(self, F, nsteps):
        diags = []
        for _ in range(nsteps):
            F, d = self.step(F)
            diags.append(d)
        return F, np.array(diags).reshape(-1, 4)
