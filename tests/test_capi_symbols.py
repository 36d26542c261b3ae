"""The C-ABI library loads and exports every symbol include/ccdvm.h declares,
and host-side validation rejects bad set-ups without touching a GPU."""
import ctypes as C
import os
import re

import pytest

from ccdvm_inputs import Body, small_2d, workload

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


def declared_symbols():
    text = open(os.path.join(ROOT, "include", "ccdvm.h")).read()
    text = re.sub(r"/\*.*?\*/", "", text, flags=re.S)
    return sorted(set(re.findall(r"\b(cc_[a-z0-9_]+)\s*\(", text)))


def test_library_exports_declared_symbols():
    from paper_1503_04544_amd._capi import SYMBOLS, lib
    L = lib()
    names = declared_symbols()
    assert len(names) >= 15
    for n in names:
        assert hasattr(L, n), n
        assert n in SYMBOLS, f"{n} not marshalled by the binding"


def _create(cfg):
    from paper_1503_04544_amd._capi import lib, make_body, make_config
    h = C.c_void_p()
    st = lib().cc_create(C.byref(make_config(cfg)), C.byref(make_body(cfg.body)), C.byref(h))
    return st, h


def test_create_and_dt_on_host():
    from paper_1503_04544_amd._capi import lib
    st, h = _create(workload("cyl32"))
    assert st == 0
    d = C.c_double()
    assert lib().cc_dt(h, C.byref(d)) == 0
    assert d.value == pytest.approx(0.5 / (2 * 5.625 * 32), rel=1e-15)
    sb, gb, xb = C.c_size_t(), C.c_size_t(), C.c_size_t()
    lib().cc_workspace_bytes(h, C.byref(sb), C.byref(gb), C.byref(xb))
    assert sb.value == 32 * 32 * 256 * 16
    # stepping before binding buffers is an ordering error, not a crash
    assert lib().cc_step(h, 1, None) == -6
    lib().cc_destroy(h)


@pytest.mark.parametrize("bad", [
    dict(nv=0), dict(nv=65), dict(vmin=1.0, vmax=1.0), dict(cfl=0.0),
    dict(n=(0, 4, 1)), dict(inflow=(0.0, 0, 0, 0, 1.0)),
])
def test_create_rejects_bad_config(bad):
    cfg = small_2d(8, 8, 8).with_(**bad)
    st, h = _create(cfg)
    assert st == -1 and not h.value


def test_create_rejects_bad_body():
    st, _ = _create(small_2d(8, 8, 8, body=Body("ellipse", axes=(0.1, 0.0, 0.0))))
    assert st == -1
    st, _ = _create(small_2d(8, 8, 8, body=Body("sphere")))
    assert st == -1


def test_create_validates_maxwellian_mode():
    from paper_1503_04544_amd._capi import lib, make_body, make_config
    cfg = small_2d(8, 8, 8)
    c = make_config(cfg)
    c.maxwellian = 2
    h = C.c_void_p()
    assert lib().cc_create(C.byref(c), C.byref(make_body(cfg.body)), C.byref(h)) == -1
    moving = small_2d(8, 8, 8, body=Body("ellipse", (0.5, 0.5, 0), (0.2, 0.05, 0), motion="free_rotation",
                                         inertia=0.01), maxwellian="conservative")
    st, h = _create(moving)
    assert st == -1 and not h.value
    st, h = _create(small_2d(8, 8, 8, maxwellian="conservative"))
    assert st == 0
    from paper_1503_04544_amd._capi import lib as L
    L().cc_destroy(h)


def test_create_validates_scheme():
    from paper_1503_04544_amd._capi import lib, make_body, make_config
    cfg = small_2d(8, 8, 8)
    c = make_config(cfg)
    c.scheme = 2
    h = C.c_void_p()
    assert lib().cc_create(C.byref(c), C.byref(make_body(cfg.body)), C.byref(h)) == -1
    moving = small_2d(8, 8, 8, body=Body("ellipse", (0.5, 0.5, 0), (0.2, 0.05, 0), motion="free_rotation",
                                         inertia=0.01), scheme="imex")
    st, h = _create(moving)
    assert st == -1 and not h.value
    st, h = _create(small_2d(8, 8, 8, scheme="imex"))
    assert st == 0
    lib().cc_destroy(h)


def test_create_validates_model():
    from paper_1503_04544_amd._capi import lib, make_body, make_config
    cfg = small_2d(8, 8, 8)
    for model, pr in ((2, 0.5), (1, 0.0), (1, float("nan"))):
        c = make_config(cfg)
        c.model, c.prandtl = model, pr
        h = C.c_void_p()
        assert lib().cc_create(C.byref(c), C.byref(make_body(cfg.body)), C.byref(h)) == -1
        assert not h.value
    st, h = _create(small_2d(8, 8, 8, model="shakhov"))
    assert st == 0
    lib().cc_destroy(h)


def test_noalloc_bind_rejects_a_setup_larger_than_the_static_scratch():
    """cc_bind_noalloc checks the scratch size of the set-up against its
    static array before it touches a device: the 3D sphere workload needs
    far more than 32 MiB and is refused with CC_EINVAL."""
    from paper_1503_04544_amd._capi import lib
    st, h = _create(workload("sphere128"))
    assert st == 0
    sb, gb, xb = C.c_size_t(), C.c_size_t(), C.c_size_t()
    assert lib().cc_workspace_bytes(h, C.byref(sb), C.byref(gb), C.byref(xb)) == 0
    assert xb.value > 32 << 20
    dummy = C.c_void_p(1 << 20)   # never dereferenced: the size check comes first
    assert lib().cc_bind_noalloc(h, dummy, dummy, dummy, None) == -1
    assert b"static array" in lib().cc_last_error(h)
    lib().cc_destroy(h)
