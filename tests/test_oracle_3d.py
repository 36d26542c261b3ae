"""Pins of the 3D oracle (Section 5) against what geometry and mathematics fix.

* A body whose surface is planar over every cell (a sphere of radius 1e6)
  gives exact cut cells: the gas polygon of each face, the planar wall
  polygon and the gas polyhedron (convex hull of gas corners and edge
  crossings) are computed here independently and must match.
* On a sphere the gas volume and the wall area converge to the exact ones
  at second order.
* A gas at rest with a wall at the same temperature stays at rest to
  round-off without collisions; the force at rest vanishes.
* Without collisions the change of mass equals the net flux through the
  domain boundary exactly (the wall carries no net mass, interior faces
  cancel).
* Pure transport without a body is the 3D first-order upwind formula per
  velocity (catches a velocity component taken from the wrong index).
* One step equals a face-loop formulation on tiny grids with cut and merged
  cells, with and without collisions.
* The first-step force on a sphere in a uniform stream tends to the
  free-molecular force integrated over the exact sphere.
"""
import math

import numpy as np
import pytest
from scipy.spatial import ConvexHull
from scipy.special import ndtr

from ccdvm_inputs import Body, Config, random_state, small_3d, workload
from oracle.oracle import Oracle3D
from tests.brute import brute_step_3d


def _plane_cfg(seed, n=(6, 5, 5)):
    rng = np.random.default_rng(seed)
    nrm = rng.normal(size=3)
    nrm /= np.linalg.norm(nrm)
    x0 = np.array([0.5, 0.25, 0.25]) + rng.uniform(-0.03, 0.03, 3)
    R = 1.0e7
    c = x0 - R * nrm
    cfg = small_3d(*n, nv=2, body=Body("sphere", tuple(c), (R, R, R)))
    return cfg, nrm, x0


def _clip(poly, nrm, x0):
    out = []
    d = [float(np.dot(p - x0, nrm)) for p in poly]
    for k in range(len(poly)):
        a, b = poly[k], poly[(k + 1) % len(poly)]
        da, db = d[k], d[(k + 1) % len(poly)]
        if da >= 0:
            out.append(a)
        if (da >= 0) != (db >= 0):
            out.append(a + da / (da - db) * (b - a))
    return out


def _area3(poly):
    if len(poly) < 3:
        return 0.0
    s = np.zeros(3)
    for k in range(len(poly)):
        s += np.cross(poly[k], poly[(k + 1) % len(poly)])
    return 0.5 * np.linalg.norm(s)


@pytest.mark.parametrize("seed", range(5))
def test_planar_cut_cells_exact(seed):
    cfg, nrm, x0 = _plane_cfg(seed)
    o = Oracle3D(cfg)
    g = o.geometry()
    nx, ny, nz = cfg.n
    h = np.array([(cfg.hi[d] - cfg.lo[d]) / cfg.n[d] for d in range(3)])
    ncut = 0
    for k in range(nz):
        for j in range(ny):
            for i in range(nx):
                c = (k * ny + j) * nx + i
                lo = np.array(cfg.lo) + h * (i, j, k)
                corners = [lo + h * ((t & 1), (t >> 1) & 1, (t >> 2) & 1) for t in range(8)]
                # faces: polygons in the corner order used for (d1, d2)
                for d in range(3):
                    d1, d2 = (d + 1) % 3, (d + 2) % 3
                    for sd in range(2):
                        quad = []
                        for a, b in ((0, 0), (1, 0), (1, 1), (0, 1)):
                            off = np.zeros(3)
                            off[d], off[d1], off[d2] = sd, a, b
                            quad.append(lo + h * off)
                        area = _area3(_clip(quad, nrm, x0))
                        assert g["S"][c, 2 * d + sd] == pytest.approx(area, abs=2e-6 * h[d1] * h[d2])
                t = g["type"][c]
                gas = [p for p in corners if np.dot(p - x0, nrm) >= 0]
                if t != 1:
                    continue
                ncut += 1
                cross = []
                for e0 in range(8):
                    for d in range(3):
                        if e0 >> d & 1:
                            continue
                        e1 = e0 | (1 << d)
                        da, db = np.dot(corners[e0] - x0, nrm), np.dot(corners[e1] - x0, nrm)
                        if (da >= 0) != (db >= 0):
                            cross.append(corners[e0] + da / (da - db) * (corners[e1] - corners[e0]))
                vol = ConvexHull(np.array(gas + cross)).volume
                assert g["vbar"][c] == pytest.approx(vol, abs=5e-6 * np.prod(h))
                # planar wall polygon: crossings ordered around their centre
                ctr = np.mean(cross, axis=0)
                e1 = cross[0] - ctr
                e1 /= np.linalg.norm(e1)
                e2 = np.cross(nrm, e1)
                ang = [math.atan2(np.dot(p - ctr, e2), np.dot(p - ctr, e1)) for p in cross]
                poly = [cross[q] for q in np.argsort(ang)]
                assert g["sw"][c] == pytest.approx(_area3(poly), abs=2e-6 * h[0] * h[1])
                assert np.allclose(g["nw"][c], -nrm, atol=1e-6)
                assert np.allclose(g["rw"][c], ctr, atol=1e-7)
    assert ncut > 10


def test_special_values_and_closure():
    cfg = small_3d(16, 8, 8, nv=2)
    o = Oracle3D(cfg)
    g = o.geometry()
    h = np.array([(cfg.hi[d] - cfg.lo[d]) / cfg.n[d] for d in range(3)])
    full = np.array([h[1] * h[2], h[1] * h[2], h[2] * h[0], h[2] * h[0], h[0] * h[1], h[0] * h[1]])
    gas, cut, solid = g["type"] == 0, g["type"] == 1, g["type"] == 2
    assert gas.sum() > 0 and cut.sum() > 0 and solid.sum() > 0
    assert np.all(g["S"][gas] == full)
    assert np.all(g["vbar"][gas] == h[0] * h[1] * h[2])
    assert np.all(g["S"][solid] == 0) and np.all(g["vbar"][solid] == 0)
    assert np.all(g["master"][solid] == -1)
    # closure of every cut cell: sum of outward face vectors + wall vector = 0
    sgn = np.array([-1, 1, -1, 1, -1, 1])
    for c in np.nonzero(cut)[0]:
        vec = np.array([sgn[2 * d] * g["S"][c, 2 * d] + sgn[2 * d + 1] * g["S"][c, 2 * d + 1]
                        for d in range(3)])
        assert np.linalg.norm(vec + g["sw"][c] * g["nw"][c]) < 1e-15
        assert 0 < g["vbar"][c] < np.prod(h)
    # masters own themselves; a control volume is the sum of its members
    m = g["master"]
    live = m >= 0
    assert np.all(m[m[live]] == m[live])
    vcv = np.zeros(cfg.ncell)
    np.add.at(vcv, m[live], g["vbar"][live])
    assert np.allclose(vcv[m[live]], g["vcv"][m[live]], rtol=1e-14)


def test_sphere_convergence():
    r = 0.3
    errs_v, errs_a = [], []
    for n in (16, 32, 64):
        cfg = Config(dim=3, n=(n, n, n), lo=(0, 0, 0), hi=(1, 1, 1), nv=2,
                     body=Body("sphere", (0.503, 0.498, 0.501), (r, r, r)))
        g = Oracle3D(cfg).geometry()
        errs_v.append(abs(g["vbar"].sum() - (1 - 4 / 3 * math.pi * r ** 3)))
        errs_a.append(abs(g["sw"].sum() - 4 * math.pi * r ** 2) / (4 * math.pi * r ** 2))
    assert errs_a[0] < 2e-2
    for e in (errs_v, errs_a):
        assert e[0] / e[1] > 3.0 and e[1] / e[2] > 3.0


def test_workload_geometry_accepted():
    cfg = workload("sphere128").with_(nv=2)
    g = Oracle3D(cfg).geometry()
    assert np.sum(g["type"] == 1) > 1000
    assert g["vbar"].sum() == pytest.approx(0.25 - 4 / 3 * math.pi * 0.1 ** 3, rel=1e-4)


def test_rest_state_is_stationary_without_collisions():
    cfg = small_3d(12, 8, 8, nv=8, kn=0.0, mach=0.0)
    o = Oracle3D(cfg)
    F = o.init()
    F1, d = o.step(F)
    assert np.max(np.abs(F1 - F)) / np.max(F) < 1e-14
    assert np.max(np.abs(d[:3])) < 1e-15


def test_mass_balance_without_collisions():
    cfg = small_3d(10, 6, 6, nv=6, kn=0.0, mach=0.6, body=Body("sphere", (0.5, 0.24, 0.27), (0.13,) * 3, t_wall=1.4))
    o = Oracle3D(cfg)
    g = o.geometry()
    F, _ = random_state(cfg.ncell, cfg.nv, 3, seed=7, with_g=False)
    F = o.merge(F)
    F1, d0 = o.step(F)
    _, d1 = o.step(F1)
    nx, ny, nz = cfg.n
    N = cfg.nv
    v = o.velocity()
    w = ((cfg.vmax - cfg.vmin) / N) ** 3
    vd = [np.tile(v, N * N), np.tile(np.repeat(v, N), N), np.repeat(v, N * N)]
    rho, ux, uy, uz, T = cfg.inflow
    ghost = rho / (2 * math.pi * T) ** 1.5 * np.exp(
        -((vd[0] - ux) ** 2 + (vd[1] - uy) ** 2 + (vd[2] - uz) ** 2) / (2 * T))
    out = 0.0  # net mass leaving through the domain boundary
    idx = np.arange(cfg.ncell)
    ii, jj, kk = idx % nx, (idx // nx) % ny, idx // (nx * ny)
    for d, pos in ((0, ii), (1, jj), (2, kk)):
        for side, at in ((0, 0), (1, cfg.n[d] - 1)):
            for c in idx[pos == at]:
                A = g["S"][c, 2 * d + side]
                cn = vd[d] if side else -vd[d]
                out += A * np.sum(np.maximum(cn, 0) * F[c] + np.minimum(cn, 0) * ghost) * w
    dm = d1[3] - d0[3]
    assert dm == pytest.approx(-o.dt * out, rel=1e-11, abs=1e-15)


def test_pure_upwind_transport_closed_form():
    n = (5, 4, 6)
    cfg = Config(dim=3, n=n, lo=(0, 0, 0), hi=(1, 1, 1), nv=2, vmin=-2.0, vmax=2.0,
                 kn=0.0, dt=0.03, body=Body("none"))
    o = Oracle3D(cfg)
    v = o.velocity()
    F, _ = random_state(cfg.ncell, 2, 3, seed=5, with_g=False)
    F1, _ = o.step(F)
    a = [0.03 * n[d] for d in range(3)]
    nx, ny = n[0], n[1]
    for k in range(1, n[2] - 1):
        for j in range(1, ny - 1):
            for i in range(1, nx - 1):
                c = (k * ny + j) * nx + i
                for p in range(8):
                    vv = (v[p % 2], v[(p // 2) % 2], v[p // 4])
                    up = [c - 1 if vv[0] > 0 else c + 1, c - nx if vv[1] > 0 else c + nx,
                          c - nx * ny if vv[2] > 0 else c + nx * ny]
                    expect = (1 - sum(a)) * F[c, p] + sum(a[d] * F[up[d], p] for d in range(3))
                    assert F1[c, p] == pytest.approx(expect, rel=1e-14, abs=1e-17)


TINY = [
    small_3d(6, 5, 5, nv=3, kn=0.07, mach=0.4, body=Body("sphere", (0.5, 0.26, 0.24), (0.17,) * 3)),
    small_3d(5, 5, 6, nv=4, kn=0.0, mach=0.7, body=Body("sphere", (0.48, 0.24, 0.27), (0.16,) * 3, t_wall=1.6)),
]


@pytest.mark.parametrize("k", range(len(TINY)))
def test_step_equals_brute_force(k):
    cfg = TINY[k]
    o = Oracle3D(cfg)
    g = o.geometry()
    merged = np.sum((g["master"] >= 0) & (g["master"] != np.arange(cfg.ncell)))
    assert merged > 0 and np.sum(g["type"] == 1) > 0
    F, _ = random_state(cfg.ncell, cfg.nv, 3, seed=200 + k, with_g=False)
    F1, _ = o.step(F)
    B = brute_step_3d(cfg, g, o.velocity(), o.dt, F, collide=cfg.kn > 0)
    assert np.max(np.abs(F1 - B)) / np.max(np.abs(F1)) < 1e-13


def free_molecular_force_sphere(r, U, T=1.0, Tw=1.0, n=400):
    """Force on a sphere of radius r in a free stream (rho = 1, u = (U,0,0),
    T) with diffuse re-emission at Tw: continuous half-range fluxes
    integrated over the exact sphere (Gauss-Legendre in cos(polar angle))."""
    s = math.sqrt(T)
    xs, ws = np.polynomial.legendre.leggauss(n)
    F = 0.0
    for mu, wt in zip(xs, ws):
        # axisymmetric about x: n_w = -(mu, sin, 0) averaged over the azimuth
        nwx = -mu
        Un = U * nwx
        z = Un / s
        pdf = math.exp(-0.5 * z * z) / math.sqrt(2 * math.pi)
        cdf = float(ndtr(z))
        n_in = Un * cdf + s * pdf
        p_n = (Un * Un + T) * cdf + Un * s * pdf
        pn_tot = p_n + n_in / math.sqrt(Tw / (2 * math.pi)) * Tw / 2.0
        # x-component: normal pressure along n_w plus tangential momentum
        fx = pn_tot * nwx + n_in * (U - Un * nwx)
        F += fx * wt * 2 * math.pi * r * r
    return F


def test_first_step_force_tends_to_free_molecular():
    U = 0.8 * math.sqrt(5.0 / 3.0)
    r = 0.2
    exact = free_molecular_force_sphere(r, U, Tw=1.5)
    # textbook closed form of the free-molecular sphere drag coefficient
    sr = U / math.sqrt(2.0)
    cd = (math.exp(-sr * sr) * (2 * sr * sr + 1) / (math.sqrt(math.pi) * sr ** 3)
          + math.erf(sr) * (4 * sr ** 4 + 4 * sr * sr - 1) / (2 * sr ** 4)
          + 2 * math.sqrt(math.pi) / (3 * sr) * math.sqrt(1.5))
    assert exact == pytest.approx(cd * 0.5 * U * U * math.pi * r * r, rel=1e-10)
    errs = []
    for n, nv in ((16, 12), (32, 12)):
        cfg = Config(dim=3, n=(n, n, n), lo=(0, 0, 0), hi=(1, 1, 1), nv=nv,
                     inflow=(1.0, U, 0.0, 0.0, 1.0),
                     body=Body("sphere", (0.5, 0.5, 0.5), (r, r, r), t_wall=1.5))
        o = Oracle3D(cfg)
        d = o.force(o.init())
        errs.append(abs(d[0] - exact) / exact)
        assert abs(d[1]) < 1e-12 * exact and abs(d[2]) < 1e-12 * exact
    # second order in the cell size (surface error dominates)
    assert errs[0] < 4e-2 and errs[1] < 1e-2 and errs[0] / errs[1] > 3.0
