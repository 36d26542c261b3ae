"""The library's octree builder (host side of cc_create) against the
oracle's: leaves, types, masters and face lists identical, areas and
volumes to 1e-13; rejected configurations."""
import ctypes as C

import numpy as np
import pytest

from ccdvm_inputs import Body, small_3d, workload
from oracle.oracle import Oracle3A

SPH = Body("sphere", (0.5, 0.25, 0.25), (0.1,) * 3)


def case(n=(16, 8, 8), nv=4, depth=1, **kw):
    kw.setdefault("body", SPH)
    return small_3d(*n, nv=nv, kn=0.1, mach=0.5, amr_depth=depth, lo=(0.0, 0.0, 0.0),
                    hi=(1.0, 0.5, 0.5), **kw)


def create(cfg):
    from paper_1503_04544_amd._capi import lib, make_body, make_config
    c, b = make_config(cfg), make_body(cfg.body)
    h = C.c_void_p()
    st = lib().cc_create(C.byref(c), C.byref(b), C.byref(h))
    return st, h


def export(h):
    from paper_1503_04544_amd._capi import lib
    nl, nf = C.c_int(), C.c_int()
    assert lib().cc_amr_counts(h, C.byref(nl), C.byref(nf)) == 0
    n, m = nl.value, nf.value
    L = {"lvl": np.zeros(n, np.int32), "ijk": np.zeros((n, 3), np.int32), "type": np.zeros(n, np.int32),
         "master": np.zeros(n, np.int32), "vbar": np.zeros(n), "vcv": np.zeros(n), "sw": np.zeros(n),
         "S": np.zeros((n, 6))}
    F = {"ptr": np.zeros(n + 1, np.int32), "nb": np.zeros(m, np.int32), "dir": np.zeros(m, np.int32),
         "area": np.zeros(m)}
    P = lambda a: a.ctypes.data_as(C.c_void_p)
    assert lib().cc_amr_export(h, *[P(L[k]) for k in ("lvl", "ijk", "type", "master", "vbar", "vcv", "sw", "S")]) == 0
    assert lib().cc_amr_faces(h, *[P(F[k]) for k in ("ptr", "nb", "dir", "area")]) == 0
    return L, F


def close(a, b):
    return np.max(np.abs(a - b)) <= 1e-13 * max(np.max(np.abs(b)), 1e-300)


@pytest.mark.parametrize("n,depth,nv", [((16, 8, 8), 1, 4), ((16, 8, 8), 2, 4), ((8, 4, 4), 3, 6),
                                        ((32, 16, 16), 2, 16)])
def test_builder_equals_oracle(n, depth, nv):
    cfg = case(n=n, depth=depth, nv=nv)
    st, h = create(cfg)
    assert st == 0
    try:
        L, F = export(h)
    finally:
        from paper_1503_04544_amd._capi import lib
        lib().cc_destroy(h)
    o = Oracle3A(cfg)
    Lo, Fo = o.leaves(), o.faces()
    for k in ("lvl", "ijk", "type", "master"):
        assert np.array_equal(L[k], Lo[k]), k
    for k in ("vbar", "vcv", "sw", "S"):
        assert close(L[k], Lo[k]), k
    for k in ("ptr", "nb", "dir"):
        assert np.array_equal(F[k], Fo[k]), k
    assert close(F["area"], Fo["area"])


def test_octree_configurations_rejected():
    from paper_1503_04544_amd._capi import lib
    for bad in (case(model="shakhov"), case(scheme="imex"), case(maxwellian="conservative"), case(depth=9)):
        st, h = create(bad)
        assert st != 0 and not h.value
    st, h = create(case(depth=1, amr_band=0.3))   # band narrower than a cell: cut cells above the finest depth
    assert st == -3 and not h.value
    st, h = create(case(depth=0))
    assert st == 0
    nl = C.c_int()
    assert lib().cc_amr_counts(h, C.byref(nl), None) != 0   # a uniform grid is no octree
    lib().cc_destroy(h)


VANE = Body("vane", (0.5, 0.5, 0.25), (0.2, 0.06, 0.12), theta=0.0, inertia=0.01,
            motion="free_rotation", omega=20.0)


@pytest.mark.parametrize("theta", [0.0, 0.3927, 1.1, 2.0, -0.7])
def test_builder_equals_oracle_for_the_vane(theta):
    from ccdvm_inputs.configs import Config, _inflow
    body = Body("vane", VANE.center, VANE.axes, theta=theta, inertia=0.01, motion="free_rotation", omega=20.0)
    cfg = Config(dim=3, n=(8, 8, 4), lo=(0.0, 0.0, 0.0), hi=(1.0, 1.0, 0.5), nv=4, kn=0.1, inflow=_inflow(0.5),
                 body=body, amr_depth=2)
    st, h = create(cfg)
    assert st == 0
    try:
        L, F = export(h)
    finally:
        from paper_1503_04544_amd._capi import lib
        lib().cc_destroy(h)
    o = Oracle3A(cfg)
    Lo, Fo = o.leaves(), o.faces()
    for k in ("lvl", "ijk", "type", "master"):
        assert np.array_equal(L[k], Lo[k]), k
    for k in ("vbar", "vcv", "sw", "S"):
        assert close(L[k], Lo[k]), k
    for k in ("ptr", "nb", "dir"):
        assert np.array_equal(F[k], Fo[k]), k
    assert close(F["area"], Fo["area"])
    assert np.sum(Lo["type"] == 1) > 50


def test_turning_configurations():
    from ccdvm_inputs.configs import Config, _inflow
    from paper_1503_04544_amd._capi import lib

    def cfg(**b):
        kw = dict(center=VANE.center, axes=VANE.axes, inertia=0.01, motion="free_rotation", omega=1.0)
        kw.update(b)
        return Config(dim=3, n=(8, 8, 4), lo=(0.0, 0.0, 0.0), hi=(1.0, 1.0, 0.5), nv=4, kn=0.1,
                      inflow=_inflow(0.5), body=Body("vane", **kw), amr_depth=2)
    # a turning body runs on the octree, also at depth 0 (the uniform grid)
    for c in (cfg(), cfg().with_(amr_depth=0, n=(32, 32, 16))):
        st, h = create(c)
        assert st == 0
        nl = C.c_int()
        assert lib().cc_amr_counts(h, C.byref(nl), None) == 0 and nl.value > 0
        lib().cc_destroy(h)
    for bad in (cfg(vel=(0.1, 0.0, 0.0)), cfg(inertia=0.0), cfg(axes=(0.2, 0.0, 0.1)),
                cfg().with_(model="shakhov"), cfg().with_(scheme="imex")):
        st, h = create(bad)
        assert st != 0 and not h.value
