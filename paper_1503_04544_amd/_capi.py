"""ctypes declarations of the C-ABI in include/ccdvm.h (argument marshalling only)."""
from __future__ import annotations

import ctypes as C
import os

HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(HERE, "libccdvm.so")

CC_STATUS = {0: "CC_OK", -1: "CC_EINVAL", -2: "CC_ENOMEM", -3: "CC_EGEOM", -4: "CC_ECFL",
             -5: "CC_EHIP", -6: "CC_ESTATE"}
BODY = {"none": 0, "circle": 1, "ellipse": 2, "cavity": 3, "halfplane": 4, "sphere": 5, "vane": 6}
MOTION = {"fixed": 0, "free_rotation": 1, "imposed": 2}


class CCError(RuntimeError):
    def __init__(self, status, msg=""):
        super().__init__(f"{CC_STATUS.get(status, status)}: {msg}")
        self.status = status


class cc_config(C.Structure):
    _fields_ = [("dim", C.c_int), ("n", C.c_int * 3), ("lo", C.c_double * 3),
                ("hi", C.c_double * 3), ("nv", C.c_int), ("vmin", C.c_double),
                ("vmax", C.c_double), ("kn", C.c_double), ("lref", C.c_double),
                ("cfl", C.c_double), ("dt", C.c_double), ("inflow", C.c_double * 5),
                ("maxwellian", C.c_int), ("scheme", C.c_int), ("model", C.c_int),
                ("prandtl", C.c_double), ("amr_depth", C.c_int), ("amr_band", C.c_double),
                ("cfl_strict", C.c_int)]


class cc_body(C.Structure):
    _fields_ = [("kind", C.c_int), ("center", C.c_double * 3), ("axes", C.c_double * 3),
                ("theta", C.c_double), ("t_wall", C.c_double), ("mass", C.c_double),
                ("inertia", C.c_double), ("motion", C.c_int), ("vel", C.c_double * 3),
                ("omega", C.c_double)]


SYMBOLS = {
    # name: (restype, argtypes)
    "cc_create": (C.c_int, [C.POINTER(cc_config), C.POINTER(cc_body), C.POINTER(C.c_void_p)]),
    "cc_destroy": (None, [C.c_void_p]),
    "cc_last_error": (C.c_char_p, [C.c_void_p]),
    "cc_workspace_bytes": (C.c_int, [C.c_void_p, C.POINTER(C.c_size_t), C.POINTER(C.c_size_t),
                                     C.POINTER(C.c_size_t)]),
    "cc_bind": (C.c_int, [C.c_void_p] + [C.c_void_p] * 5),
    "cc_bind_noalloc": (C.c_int, [C.c_void_p] + [C.c_void_p] * 4),
    "cc_cfl_number": (C.c_int, [C.c_void_p, C.POINTER(C.c_double)]),
    "cc_init_maxwellian": (C.c_int, [C.c_void_p]),
    "cc_load_state": (C.c_int, [C.c_void_p, C.c_void_p, C.c_void_p]),
    "cc_store_state": (C.c_int, [C.c_void_p, C.c_void_p, C.c_void_p]),
    "cc_step": (C.c_int, [C.c_void_p, C.c_int, C.c_void_p]),
    "cc_moments": (C.c_int, [C.c_void_p, C.c_void_p]),
    "cc_body_force": (C.c_int, [C.c_void_p, C.POINTER(C.c_double)]),
    "cc_body_state": (C.c_int, [C.c_void_p, C.POINTER(C.c_double)]),
    "cc_rigid_update": (C.c_int, [C.c_void_p, C.POINTER(C.c_double), C.c_double]),
    "cc_dt": (C.c_int, [C.c_void_p, C.POINTER(C.c_double)]),
    "cc_geometry_export": (C.c_int, [C.c_void_p] + [C.c_void_p] * 13),
    "cc_geometry_export3d": (C.c_int, [C.c_void_p] + [C.c_void_p] * 17),
    "cc_geometry_counts": (C.c_int, [C.c_void_p] + [C.POINTER(C.c_int)] * 3),
    "cc_amr_counts": (C.c_int, [C.c_void_p] + [C.POINTER(C.c_int)] * 2),
    "cc_amr_export": (C.c_int, [C.c_void_p] * 9),
    "cc_amr_faces": (C.c_int, [C.c_void_p] * 5),
    "cc_set_tile_rows": (C.c_int, [C.c_void_p, C.c_int]),
    "cc_profile_enable": (C.c_int, [C.c_void_p, C.c_int]),
    "cc_profile_read": (C.c_int, [C.c_void_p, C.c_int, C.POINTER(C.c_double), C.POINTER(C.c_int)]),
    "cc_adjoint_workspace_bytes": (C.c_int, [C.c_void_p, C.c_int, C.c_int, C.POINTER(C.c_size_t)]),
    "cc_adjoint": (C.c_int, [C.c_void_p, C.c_int, C.c_int, C.c_int, C.c_void_p, C.POINTER(C.c_double)]),
    "cc_batch_create": (C.c_int, [C.POINTER(C.c_void_p), C.c_int, C.POINTER(C.c_void_p)]),
    "cc_batch_workspace_bytes": (C.c_int, [C.c_void_p, C.POINTER(C.c_size_t)]),
    "cc_batch_bind": (C.c_int, [C.c_void_p, C.c_void_p]),
    "cc_batch_autotune": (C.c_int, [C.c_void_p, C.c_int, C.POINTER(C.c_int)]),
    "cc_batch_groups": (C.c_int, [C.c_void_p, C.POINTER(C.c_int), C.POINTER(C.c_int), C.POINTER(C.c_int)]),
    "cc_batch_step": (C.c_int, [C.c_void_p, C.c_int]),
    "cc_batch_adjoint_workspace_bytes": (C.c_int, [C.c_void_p, C.c_int, C.c_int, C.POINTER(C.c_size_t)]),
    "cc_batch_adjoint": (C.c_int, [C.c_void_p, C.c_int, C.c_int, C.c_int, C.c_void_p, C.POINTER(C.c_double)]),
    "cc_batch_last_error": (C.c_char_p, [C.c_void_p]),
    "cc_batch_destroy": (None, [C.c_void_p]),
}

_lib = None


def lib():
    """Load libccdvm.so; raises if it has not been built (there is no fallback)."""
    global _lib
    if _lib is None:
        if not os.path.exists(LIB_PATH):
            raise ImportError(f"{LIB_PATH} is missing: build it with "
                              "`python -c 'import __graft_entry__ as g; g.build()'`")
        L = C.CDLL(LIB_PATH)
        for name, (res, args) in SYMBOLS.items():
            fn = getattr(L, name)
            fn.restype = res
            fn.argtypes = args
        _lib = L
    return _lib


def make_config(cfg) -> cc_config:
    c = cc_config()
    c.dim = cfg.dim
    c.n[:] = list(cfg.n)
    c.lo[:] = [float(x) for x in cfg.lo]
    c.hi[:] = [float(x) for x in cfg.hi]
    c.nv = cfg.nv
    c.vmin, c.vmax = cfg.vmin, cfg.vmax
    c.kn, c.lref, c.cfl, c.dt = cfg.kn, cfg.lref, cfg.cfl, cfg.dt
    c.inflow[:] = [float(x) for x in cfg.inflow]
    c.maxwellian = {"direct": 0, "conservative": 1}[getattr(cfg, "maxwellian", "direct")]
    c.scheme = {"explicit": 0, "imex": 1}[getattr(cfg, "scheme", "explicit")]
    c.model = {"bgk": 0, "shakhov": 1}[getattr(cfg, "model", "bgk")]
    c.prandtl = getattr(cfg, "prandtl", 2.0 / 3.0)
    c.amr_depth = getattr(cfg, "amr_depth", 0)
    c.amr_band = getattr(cfg, "amr_band", 0.0)
    c.cfl_strict = int(getattr(cfg, "cfl_strict", 0))
    return c


def make_body(b) -> cc_body:
    s = cc_body()
    s.kind = BODY[b.kind]
    s.center[:] = [float(x) for x in b.center]
    s.axes[:] = [float(x) for x in b.axes]
    s.theta, s.t_wall, s.mass, s.inertia = b.theta, b.t_wall, b.mass, b.inertia
    s.motion = MOTION[b.motion]
    s.vel[:] = [float(x) for x in b.vel]
    s.omega = b.omega
    return s
