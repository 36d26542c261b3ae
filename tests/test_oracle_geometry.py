"""Pins of the oracle's geometry (Appendix A) against exact geometry.

* A half-plane level set is linear, so linear interpolation of the crossing
  points is exact: every length, normal, wall centre and area must equal the
  analytic clipping of the square cell by the half-plane (Sutherland-Hodgman
  here, written independently of the oracle).
* Gas and solid cells carry the special values listed in Section 3.2.2.
* Circle: total gas area and wall length converge to the exact ones at
  second order in dx.
* Master search: the control-volume example of Section 3.2.3 (a small cut
  cell whose largest gas edge is its upper edge merges with (i, j+1)); the
  area of every control volume is at least half a Cartesian cell.
* A cell crossed twice by the boundary (saddle) is rejected.
"""
import math

import numpy as np
import pytest

from ccdvm_inputs import Body, small_2d, workload
from oracle import Oracle2D, OracleError


def clip_polygon(poly, nrm, c):
    """Sutherland-Hodgman clip of poly to {x : (x - c).nrm >= 0}."""
    out = []
    d = [(p[0] - c[0]) * nrm[0] + (p[1] - c[1]) * nrm[1] for p in poly]
    for k in range(len(poly)):
        a, b = poly[k], poly[(k + 1) % len(poly)]
        da, db = d[k], d[(k + 1) % len(poly)]
        if da >= 0:
            out.append(a)
        if (da >= 0) != (db >= 0):
            t = da / (da - db)
            out.append((a[0] + t * (b[0] - a[0]), a[1] + t * (b[1] - a[1])))
    return out


def shoelace(poly):
    s = 0.0
    for k in range(len(poly)):
        a, b = poly[k], poly[(k + 1) % len(poly)]
        s += a[0] * b[1] - a[1] * b[0]
    return 0.5 * s


def seg_gas_length(a, b, nrm, c):
    da = (a[0] - c[0]) * nrm[0] + (a[1] - c[1]) * nrm[1]
    db = (b[0] - c[0]) * nrm[0] + (b[1] - c[1]) * nrm[1]
    L = math.hypot(b[0] - a[0], b[1] - a[1])
    if da >= 0 and db >= 0:
        return L
    if da < 0 and db < 0:
        return 0.0
    t = da / (da - db)
    return t * L if da >= 0 else (1 - t) * L


@pytest.mark.parametrize("seed", range(6))
def test_halfplane_exact(seed):
    rng = np.random.default_rng(seed)
    th = rng.uniform(0, 2 * math.pi)
    c = (0.5 + rng.uniform(-0.05, 0.05), 0.5 + rng.uniform(-0.05, 0.05))
    nx, ny = 9, 7
    cfg = small_2d(nx, ny, 4, body=Body("halfplane", (c[0], c[1], 0.0), theta=th))
    o = Oracle2D(cfg)
    geo = o.geometry()
    dx, dy = 1.0 / nx, 1.0 / ny
    nrm = (math.cos(th), math.sin(th))
    for j in range(ny):
        for i in range(nx):
            k = j * nx + i
            x0, y0 = i * dx, j * dy
            sq = [(x0, y0), (x0 + dx, y0), (x0 + dx, y0 + dy), (x0, y0 + dy)]
            poly = clip_polygon(sq, nrm, c)
            area = shoelace(poly) if len(poly) >= 3 else 0.0
            assert geo["sbar"][k] == pytest.approx(area, abs=1e-15)
            assert geo["lxm"][k] == pytest.approx(seg_gas_length(sq[0], sq[3], nrm, c), abs=1e-15)
            assert geo["lxp"][k] == pytest.approx(seg_gas_length(sq[1], sq[2], nrm, c), abs=1e-15)
            assert geo["lym"][k] == pytest.approx(seg_gas_length(sq[0], sq[1], nrm, c), abs=1e-15)
            assert geo["lyp"][k] == pytest.approx(seg_gas_length(sq[3], sq[2], nrm, c), abs=1e-15)
            ds = [(p[0] - c[0]) * nrm[0] + (p[1] - c[1]) * nrm[1] for p in sq]
            if min(ds) > 0 or max(ds) < 0:
                assert geo["lw"][k] == 0.0
                assert geo["type"][k] == (0 if min(ds) > 0 else 2)
            else:
                assert geo["type"][k] == 1
                # wall edge = the chord of the line inside the cell
                on_line = [p for p in poly if abs((p[0] - c[0]) * nrm[0] + (p[1] - c[1]) * nrm[1]) < 1e-13]
                assert len(on_line) == 2
                chord = math.hypot(on_line[0][0] - on_line[1][0], on_line[0][1] - on_line[1][1])
                assert geo["lw"][k] == pytest.approx(chord, abs=1e-15)
                # normal points into the solid
                assert geo["nwx"][k] == pytest.approx(-nrm[0], abs=1e-12)
                assert geo["nwy"][k] == pytest.approx(-nrm[1], abs=1e-12)
                mid = (0.5 * (on_line[0][0] + on_line[1][0]), 0.5 * (on_line[0][1] + on_line[1][1]))
                assert geo["rwx"][k] == pytest.approx(mid[0], abs=1e-15)
                assert geo["rwy"][k] == pytest.approx(mid[1], abs=1e-15)


def test_gas_and_solid_special_values():
    cfg = workload("cyl32")
    geo = Oracle2D(cfg).geometry()
    dx = dy = 1.0 / 32
    gas = geo["type"] == 0
    solid = geo["type"] == 2
    for k in ("lxm", "lxp"):
        assert np.all(geo[k][gas] == dy) and np.all(geo[k][solid] == 0.0)
    for k in ("lym", "lyp"):
        assert np.all(geo[k][gas] == dx) and np.all(geo[k][solid] == 0.0)
    assert np.all(geo["lw"][gas] == 0.0) and np.all(geo["lw"][solid] == 0.0)
    assert np.allclose(geo["sbar"][gas], dx * dy, rtol=0, atol=1e-18)
    assert np.all(geo["sbar"][solid] == 0.0)
    assert np.all(geo["master"][solid] == -1)
    cut = geo["type"] == 1
    assert np.all(geo["lw"][cut] > 0) and np.all(geo["lw"][cut] <= math.hypot(dx, dy) * (1 + 1e-14))
    # per-cell closure: sum over the five edges of |L| n = 0
    cx = geo["lxp"] - geo["lxm"] + geo["lw"] * geo["nwx"]
    cy = geo["lyp"] - geo["lym"] + geo["lw"] * geo["nwy"]
    assert np.max(np.abs(cx)) < 1e-17 and np.max(np.abs(cy)) < 1e-17


def test_circle_convergence():
    errs_a, errs_l = [], []
    for n in (16, 32, 64, 128):
        cfg = small_2d(n, n, 2, body=Body("circle", (0.5, 0.5, 0.0), (0.2, 0.2, 0.0)))
        geo = Oracle2D(cfg).geometry()
        errs_a.append(abs(geo["sbar"].sum() - (1 - math.pi * 0.04)))
        errs_l.append(abs(geo["lw"].sum() - 2 * math.pi * 0.2))
    # second order: the error drops by ~4 per refinement
    for e0, e1 in zip(errs_a[:-1], errs_a[1:]):
        assert e1 < e0 / 2.5
    for e0, e1 in zip(errs_l[:-1], errs_l[1:]):
        assert e1 < e0 / 2.5
    assert errs_a[-1] < 1e-4 and errs_l[-1] < 1e-3


def test_merge_example_upper_edge():
    # Half-plane y > y0 with y0 above the centre of row j = 3: the cut cells
    # of that row have their centre in the solid and a full upper edge, so
    # they merge upward into row 4 (the control-volume example of 3.2.3).
    n = 8
    y0 = 3.7 / n
    cfg = small_2d(n, n, 2, body=Body("halfplane", (0.5, y0, 0.0), theta=math.pi / 2 + 1e-3))
    geo = Oracle2D(cfg).geometry()
    for i in range(1, n - 1):
        k = 3 * n + i
        assert geo["type"][k] == 1
        assert geo["lyp"][k] == pytest.approx(1.0 / n)
        assert geo["master"][k] == 4 * n + i
        assert geo["scv"][4 * n + i] == pytest.approx(geo["sbar"][k] + 1.0 / n ** 2)


@pytest.mark.parametrize("name", ["cyl32", "cyl512"])
def test_control_volume_at_least_half_cell(name):
    cfg = workload(name)
    geo = Oracle2D(cfg).geometry()
    dx = (cfg.hi[0] - cfg.lo[0]) / cfg.n[0]
    dy = (cfg.hi[1] - cfg.lo[1]) / cfg.n[1]
    masters = np.nonzero(geo["master"] == np.arange(cfg.ncell))[0]
    assert np.min(geo["scv"][masters]) >= 0.5 * dx * dy
    # every non-solid cell points to a master that is its own master
    m = geo["master"][geo["master"] >= 0]
    assert np.all(geo["master"][m] == m)
    # total gas area is the sum of the control volumes
    assert geo["scv"][masters].sum() == pytest.approx(geo["sbar"].sum(), rel=1e-13)


def test_ellipse_workload_geometry():
    cfg = workload("ellipse256")
    geo = Oracle2D(cfg).geometry()
    a, b = 0.1, 0.02
    assert geo["sbar"].sum() == pytest.approx(1 - math.pi * a * b, abs=2e-5)
    masters = np.nonzero(geo["master"] == np.arange(cfg.ncell))[0]
    assert np.min(geo["scv"][masters]) >= 0.5 / 256 ** 2


def test_saddle_rejected():
    # a thin ellipse along the diagonal through a vertex: diagonal vertices in
    # the solid, off-diagonal ones in the gas -> two boundary pieces per cell
    cfg = small_2d(32, 32, 2, body=Body("ellipse", (0.5, 0.5, 0.0), (0.1, 0.004, 0.0),
                                        theta=math.pi / 4))
    with pytest.raises(OracleError):
        Oracle2D(cfg)
