"""The positivity number of eq. eq-CFL (Section 3.4.1) that cc_bind
evaluates on the device geometry, against closed forms:

* without a body every control volume is a full cell, phi / S =
  sum_d |v_d| / dx_d, largest at the extreme velocity nodes, and dt was set
  from exactly that sum: the transport part equals the CFL number (2D, 3D);
* a half-plane wall x = x0 that leaves 0.6 of a column of cells in the gas
  (centres in the gas, no merging): the cut cell's outflow is
  dy |v_1| (left face or wall) + 0.6 dx |v_2| over the area 0.6 dx dy, so
  the transport part is CFL (1/0.6 + 1) / 2 on a square grid;
* the collision part is dt rho_in / tau(Kn) (mean free path over mean speed);
* strict mode refuses a set-up above 1 with CC_ECFL, otherwise it binds.
"""
import math

import numpy as np
import pytest

from ccdvm_inputs import Body, Config, small_2d, small_3d, workload

pytestmark = pytest.mark.gpu
torch = pytest.importorskip("torch")


@pytest.fixture(scope="module", autouse=True)
def _gpu():
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    from paper_1503_04544_amd.solver import Solver  # noqa: F401 (fails loudly if unbuilt)


def number(cfg):
    import ctypes as C
    from paper_1503_04544_amd._capi import lib
    from paper_1503_04544_amd.solver import Solver
    s = Solver(cfg, device="cuda:0")
    out = (C.c_double * 3)()
    assert lib().cc_cfl_number(s._h, out) == 0
    dt = s.dt
    s.close()
    return np.array(out[:]), dt


def cbar():
    from scipy.integrate import quad
    v, _ = quad(lambda c: 4.0 * math.pi * c ** 3 * math.exp(-0.5 * c * c) / (2.0 * math.pi) ** 1.5, 0, math.inf)
    return v


def test_no_body_is_the_cfl_number():
    n2, dt = number(small_2d(12, 9, 8, kn=0.2, mach=0.5, body=Body("none")))
    assert n2[0] == pytest.approx(0.5, rel=1e-14)
    assert n2[1] == pytest.approx(dt * cbar() / 0.2, rel=1e-12)
    n3, _ = number(small_3d(6, 5, 4, nv=4, kn=0.0, body=Body("none")))
    assert n3[0] == pytest.approx(0.5, rel=1e-14) and n3[1] == 0.0


def test_half_plane_cut_cell():
    cfg = Config(dim=2, n=(10, 10, 1), lo=(0, 0, 0), hi=(1, 1, 1), nv=8, kn=0.0,
                 inflow=(1.0, 0.0, 0.0, 0.0, 1.0), body=Body("halfplane", (0.56, 0.5, 0.0), (0, 0, 0), theta=math.pi))
    n, _ = number(cfg)
    assert n[0] == pytest.approx(0.5 * (1.0 / 0.6 + 1.0) / 2.0, rel=1e-12)


def test_strict_mode():
    from paper_1503_04544_amd._capi import CCError
    cfg = workload("cyl32").with_(cfl=0.9)
    n, _ = number(cfg)                      # warns, binds
    assert n[2] > 1.0
    with pytest.raises(CCError) as e:
        number(cfg.with_(cfl_strict=1))
    assert e.value.status == -4
    n, _ = number(workload("cyl32").with_(cfl_strict=1))   # 0.5: below 1
    assert 0.5 <= n[0] < 1.0
