"""Pins of the oracle's Shakhov model (Section 2.1; reduced form eq.
ShakhovDD), none of which retypes the formula:

* Pr = 1 reduces it to BGK, for the explicit and the semi-implicit step, 2D
  and 3D.
* On a fine velocity grid the equilibria (f_eq, g_eq) of a smooth state keep
  its mass, momentum and energy, and their heat flux is (1 - Pr) q -- the
  property that gives the model its Prandtl number; a wrong constant in
  either polynomial factor breaks the momentum or the heat flux.
* The reduced equilibria equal the 3D Shakhov equilibrium integrated over
  v_z against (1, v_z^2/2), for a 3D state with u_z = q_z = 0.
* On interior cells of a uniform state only the relaxation acts: the heat
  flux after one step is (1 - nu Pr) q (explicit) or
  (1 + nu (1 - Pr))/(1 + nu) q (semi-implicit), nu = dt/tau.
* One step equals the face-loop formulation of tests/brute.py, with merged
  cells, 2D and 3D, explicit and semi-implicit.
"""
import numpy as np
import pytest

from ccdvm_inputs import Body, Config, random_state, small_2d, small_3d
from oracle.oracle import Oracle2D, Oracle3D
from tests.brute import brute_step, brute_step_3d

PR = 2.0 / 3.0


def maxw(rho, u, T, vs):
    c2 = sum((vd - ud) ** 2 for vd, ud in zip(vs, u))
    return rho / (2 * np.pi * T) ** (len(vs) / 2) * np.exp(-c2 / (2 * T))


def one_cell_2d(nv, vmax, **kw):
    return Config(dim=2, n=(2, 2, 1), lo=(0, 0, 0), hi=(1, 1, 1), nv=nv, vmin=-vmax, vmax=vmax,
                  kn=0.1, body=Body("none"), model="shakhov", **kw)


def mixture_2d(vx, vy):
    """A smooth, far-from-equilibrium (f, g): two reduced Maxwellians."""
    f = 0.7 * maxw(1.0, (0.9, -0.2), 0.6, (vx, vy)) + 0.5 * maxw(1.0, (-0.5, 0.4), 1.1, (vx, vy))
    g = 0.5 * 0.6 * 0.7 * maxw(1.0, (0.9, -0.2), 0.6, (vx, vy)) + \
        0.5 * 1.3 * 0.5 * maxw(1.0, (-0.5, 0.4), 1.1, (vx, vy))
    return f, g


def moments_2d(f, g, vx, vy, w):
    rho = f.sum() * w
    ux, uy = (vx * f).sum() * w / rho, (vy * f).sum() * w / rho
    E = (0.5 * (vx ** 2 + vy ** 2) * f + g).sum() * w
    cx, cy = vx - ux, vy - uy
    h = 0.5 * (cx ** 2 + cy ** 2) * f + g
    return np.array([rho, rho * ux, rho * uy, E]), np.array([(cx * h).sum() * w, (cy * h).sum() * w])


@pytest.mark.parametrize("scheme", ["explicit", "imex"])
def test_prandtl_one_is_bgk(scheme):
    cfg = small_2d(10, 10, 8, kn=0.05, mach=0.7, scheme=scheme)
    f, g = random_state(cfg.ncell, cfg.nv, 2, seed=21)
    a = Oracle2D(cfg).step(f, g)
    b = Oracle2D(cfg.with_(model="shakhov", prandtl=1.0)).step(f, g)
    assert np.max(np.abs(a[0] - b[0])) <= 1e-15 * np.max(np.abs(a[0]))
    assert np.max(np.abs(a[1] - b[1])) <= 1e-15 * np.max(np.abs(a[1]))
    c = Oracle2D(cfg.with_(model="shakhov")).step(f, g)
    assert np.max(np.abs(a[0] - c[0])) > 1e-6 * np.max(np.abs(a[0]))   # Pr = 2/3 differs
    cfg3 = small_3d(6, 5, 5, nv=6, kn=0.05, mach=0.5, body=Body("sphere", (0.5, 0.26, 0.24), (0.17,) * 3),
                    scheme=scheme)
    F, _ = random_state(cfg3.ncell, cfg3.nv, 3, seed=22, with_g=False)
    a3 = Oracle3D(cfg3).step(F)[0]
    b3 = Oracle3D(cfg3.with_(model="shakhov", prandtl=1.0)).step(F)[0]
    assert np.max(np.abs(a3 - b3)) <= 1e-15 * np.max(np.abs(a3))


@pytest.mark.parametrize("pr", [0.0, 2.0 / 3.0, 0.9])
def test_equilibria_keep_invariants_and_scale_heat_flux(pr):
    o = Oracle2D(one_cell_2d(48, 9.0, prandtl=pr))
    v = o.velocity()
    w = (v[1] - v[0]) ** 2
    vx, vy = np.tile(v, 48), np.repeat(v, 48)
    f, g = mixture_2d(vx, vy)
    fe, ge = o.equilibrium_values(f, g)
    m0, q0 = moments_2d(f, g, vx, vy, w)
    m1, q1 = moments_2d(fe, ge, vx, vy, w)
    assert np.linalg.norm(q0) > 0.05
    assert np.allclose(m1, m0, rtol=0, atol=1e-11)
    assert np.allclose(q1, (1 - pr) * q0, rtol=0, atol=1e-11)


def test_reduced_equilibria_are_the_integrated_3d_equilibrium():
    N, vmax = 24, 8.0
    cfg3 = Config(dim=3, n=(2, 2, 2), lo=(0, 0, 0), hi=(1, 1, 1), nv=N, vmin=-vmax, vmax=vmax,
                  kn=0.1, body=Body("none"), model="shakhov")
    o3 = Oracle3D(cfg3)
    v = o3.velocity()
    dv = v[1] - v[0]
    vx = np.tile(v, N * N)
    vy = np.tile(np.repeat(v, N), N)
    vz = np.repeat(v, N * N)
    F = 0.7 * maxw(1.0, (0.9, -0.2, 0.0), 0.6, (vx, vy, vz)) + 0.5 * maxw(1.0, (-0.5, 0.4, 0.0), 1.1, (vx, vy, vz))
    Fe = o3.equilibrium_values(F)
    # reduce over v_z (p3 is the slowest index)
    def reduce(A):
        A3 = A.reshape(N, N * N)
        return A3.sum(axis=0) * dv, (0.5 * vz.reshape(N, N * N) ** 2 * A3).sum(axis=0) * dv
    f, g = reduce(F)
    fe_ref, ge_ref = reduce(Fe)
    o2 = Oracle2D(one_cell_2d(N, vmax))
    fe, ge = o2.equilibrium_values(f, g)
    assert np.max(np.abs(fe - fe_ref)) < 1e-12 * np.max(fe_ref)
    assert np.max(np.abs(ge - ge_ref)) < 1e-12 * np.max(ge_ref)
    # and the correction is not negligible here
    Fm = o3.__class__(cfg3.with_(model="bgk")).equilibrium_values(F)
    assert np.max(np.abs(Fe - Fm)) > 1e-3 * np.max(Fm)


@pytest.mark.parametrize("scheme", ["explicit", "imex"])
def test_heat_flux_relaxes_with_prandtl_number(scheme):
    nx = ny = 5
    nv, vmax, kn = 40, 9.0, 0.5
    cfg = Config(dim=2, n=(nx, ny, 1), lo=(0, 0, 0), hi=(1, 1, 1), nv=nv, vmin=-vmax, vmax=vmax, kn=kn,
                 body=Body("none"), inflow=(1.0, 0.3, -0.2, 0.0, 1.1), model="shakhov", scheme=scheme)
    o = Oracle2D(cfg)
    v = o.velocity()
    w = (v[1] - v[0]) ** 2
    vx, vy = np.tile(v, nv), np.repeat(v, nv)
    f0, g0 = mixture_2d(vx, vy)
    f = np.repeat(f0[None], nx * ny, axis=0)
    g = np.repeat(g0[None], nx * ny, axis=0)
    f1, g1, _ = o.step(f, g)
    c = 2 * nx + 2
    m0, q0 = moments_2d(f[c], g[c], vx, vy, w)
    m1, q1 = moments_2d(f1[c], g1[c], vx, vy, w)
    nu = o.dt / (np.sqrt(np.pi) / 2 * kn / np.sqrt(2.0) / m0[0])
    assert 0.005 < nu < 0.5
    rate = (1 - nu * PR) if scheme == "explicit" else (1 + nu * (1 - PR)) / (1 + nu)
    assert np.allclose(m1, m0, rtol=0, atol=1e-11)
    assert np.allclose(q1, rate * q0, rtol=0, atol=1e-11)
    assert np.max(np.abs(q1 - q0)) > 1e-4    # it did relax


TINY2 = [
    small_2d(6, 6, 4, kn=0.07, mach=0.4, body=Body("circle", (0.5, 0.52, 0), (0.19, 0.19, 0)), model="shakhov"),
    small_2d(8, 6, 6, kn=0.01, mach=0.8, body=Body("circle", (0.47, 0.52, 0), (0.18, 0.18, 0), t_wall=1.7),
             model="shakhov", prandtl=0.3, scheme="imex"),
]


@pytest.mark.parametrize("k", range(len(TINY2)))
def test_step_equals_brute_force_2d(k):
    cfg = TINY2[k]
    o = Oracle2D(cfg)
    geo = o.geometry()
    f, g = random_state(cfg.ncell, cfg.nv, 2, seed=400 + k)
    f1, g1, _ = o.step(f, g)
    bf, bg = brute_step(cfg, geo, o.velocity(), o.dt, f, g, collide=True, imex=cfg.scheme == "imex")
    assert np.max(np.abs(f1 - bf)) / np.max(np.abs(f1)) < 1e-13
    assert np.max(np.abs(g1 - bg)) / np.max(np.abs(g1)) < 1e-13
    # the Shakhov term is visible at this Kn
    b0 = brute_step(cfg.with_(model="bgk"), geo, o.velocity(), o.dt, f, g, collide=True,
                    imex=cfg.scheme == "imex")[0]
    assert np.max(np.abs(f1 - b0)) > 1e-8 * np.max(np.abs(f1))


@pytest.mark.parametrize("scheme", ["explicit", "imex"])
def test_step_equals_brute_force_3d(scheme):
    cfg = small_3d(6, 5, 5, nv=4, kn=0.02, mach=0.4, body=Body("sphere", (0.5, 0.26, 0.24), (0.17,) * 3),
                   model="shakhov", scheme=scheme)
    o = Oracle3D(cfg)
    F, _ = random_state(cfg.ncell, cfg.nv, 3, seed=410, with_g=False)
    F1, _ = o.step(F)
    B = brute_step_3d(cfg, o.geometry(), o.velocity(), o.dt, F, collide=True, imex=scheme == "imex")
    assert np.max(np.abs(F1 - B)) / np.max(np.abs(F1)) < 1e-13
