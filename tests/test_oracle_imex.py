"""Pins of the oracle's semi-implicit scheme (eq. ImpSchemeDD): explicit
transport, implicit relaxation toward the equilibrium of t^{n+1}, whose
moments are those of the transported value.

* It equals a face-loop formulation of the same scheme on tiny grids with
  cut and merged cells (2D and 3D).
* Without collisions (very large Kn) it coincides with the explicit scheme.
* Asymptotic preservation: for Kn -> 0 one step returns, in every control
  volume, the Maxwellian of its own new moments.
* With the conservative equilibrium the relaxation conserves mass,
  momentum and energy exactly, and a gas at rest with an isothermal wall
  stays at rest with collisions.
* Stability: at dt/tau ~ 1e4 it stays positive and bounded where the
  explicit scheme diverges.
* One step differs from the explicit one by O(dt^2) (both first order).
"""
import numpy as np
import pytest

from ccdvm_inputs import Body, Config, random_state, small_2d, small_3d
from oracle import Oracle2D
from oracle.oracle import Oracle3D
from tests.brute import brute_step, brute_step_3d

TINY2 = [
    small_2d(6, 6, 4, kn=0.07, mach=0.4, body=Body("circle", (0.5, 0.52, 0), (0.19, 0.19, 0)), scheme="imex"),
    small_2d(8, 6, 6, kn=0.01, mach=0.8, body=Body("circle", (0.47, 0.52, 0), (0.18, 0.18, 0), t_wall=1.7), scheme="imex"),
]


@pytest.mark.parametrize("k", range(len(TINY2)))
def test_step_equals_brute_force_2d(k):
    cfg = TINY2[k]
    o = Oracle2D(cfg)
    geo = o.geometry()
    f, g = random_state(cfg.ncell, cfg.nv, 2, seed=300 + k)
    f1, g1, _ = o.step(f, g)
    bf, bg = brute_step(cfg, geo, o.velocity(), o.dt, f, g, collide=True, imex=True)
    assert np.max(np.abs(f1 - bf)) / np.max(np.abs(f1)) < 1e-13
    assert np.max(np.abs(g1 - bg)) / np.max(np.abs(g1)) < 1e-13


def test_step_equals_brute_force_3d():
    cfg = small_3d(6, 5, 5, nv=3, kn=0.02, mach=0.4, body=Body("sphere", (0.5, 0.26, 0.24), (0.17,) * 3), scheme="imex")
    o = Oracle3D(cfg)
    F, _ = random_state(cfg.ncell, cfg.nv, 3, seed=310, with_g=False)
    F1, _ = o.step(F)
    B = brute_step_3d(cfg, o.geometry(), o.velocity(), o.dt, F, collide=True, imex=True)
    assert np.max(np.abs(F1 - B)) / np.max(np.abs(F1)) < 1e-13


def test_collisionless_limit_equals_explicit():
    cfg = small_2d(12, 12, 8, kn=1e15, mach=0.6)
    f, g = random_state(cfg.ncell, cfg.nv, 2, seed=5)
    a = Oracle2D(cfg).step(f, g)
    b = Oracle2D(cfg.with_(scheme="imex")).step(f, g)
    assert np.max(np.abs(a[0] - b[0])) / np.max(np.abs(a[0])) < 1e-14


@pytest.mark.parametrize("mode", ["direct", "conservative"])
def test_asymptotic_preservation(mode):
    """Kn -> 0: every new control-volume value is a sampled Maxwellian, i.e.
    ln f is exactly of the form a + b.v + c|v|^2 over the velocity grid, and
    g/f is the constant T/2."""
    cfg = small_2d(10, 10, 12, kn=1e-13, mach=0.5, scheme="imex", maxwellian=mode)
    o = Oracle2D(cfg)
    f, g = random_state(cfg.ncell, cfg.nv, 2, seed=9)
    f1, g1, _ = o.step(f, g)
    v = o.velocity()
    vx, vy = np.tile(v, 12), np.repeat(v, 12)
    A = np.stack([np.ones_like(vx), vx, vy, vx ** 2 + vy ** 2], axis=1)
    geo = o.geometry()
    worst_log, worst_ratio = 0.0, 0.0
    for c in np.nonzero(geo["master"] == np.arange(cfg.ncell))[0]:
        lf = np.log(f1[c])
        coef, *_ = np.linalg.lstsq(A, lf, rcond=None)
        worst_log = max(worst_log, np.max(np.abs(A @ coef - lf)))
        r = g1[c] / f1[c]
        worst_ratio = max(worst_ratio, (r.max() - r.min()) / r.mean())
    assert worst_log < 1e-8 and worst_ratio < 1e-8


def test_conservation_and_rest_with_conservative_equilibrium():
    n = 5
    cfg = Config(dim=2, n=(n, n, 1), lo=(0, 0, 0), hi=(1, 1, 1), nv=10, kn=0.002,
                 body=Body("none"), inflow=(1.0, 0.3, -0.2, 0.0, 1.1), maxwellian="conservative",
                 scheme="imex")
    o = Oracle2D(cfg)
    v = o.velocity()
    vx, vy, w = np.tile(v, 10), np.repeat(v, 10), 1.2 ** 2
    gauss = lambda ax, ay, T: np.exp(-((vx - ax) ** 2 + (vy - ay) ** 2) / (2 * T)) / (2 * np.pi * T)
    f0 = 0.6 * gauss(1.4, 0.2, 0.4) + 0.5 * gauss(-0.9, -0.4, 0.5)
    g0 = 0.4 * f0 + 0.2 * gauss(0.0, 0.3, 0.9)
    f = np.repeat(f0[None], n * n, axis=0)
    g = np.repeat(g0[None], n * n, axis=0)
    f1, g1, _ = o.step(f, g)
    c = 2 * n + 2
    mom = lambda a, b: np.array([a.sum(), (vx * a).sum(), (vy * a).sum(),
                                 (0.5 * (vx ** 2 + vy ** 2) * a + b).sum()]) * w
    assert np.max(np.abs(f1[c] - f[c])) > 1e-2 * np.max(f[c])
    assert np.max(np.abs(mom(f1[c], g1[c]) - mom(f[c], g[c]))) / np.abs(mom(f[c], g[c])).max() < 2e-15
    cfg = small_2d(32, 32, 16, kn=0.01, mach=0.0, maxwellian="conservative", scheme="imex")
    o = Oracle2D(cfg)
    f, g = o.init()
    f1, g1, _ = o.step(f, g)
    assert np.max(np.abs(f1 - f)) / np.max(f) < 1e-14
    cfg = small_3d(10, 6, 6, nv=8, kn=0.01, mach=0.0, maxwellian="conservative", scheme="imex")
    o = Oracle3D(cfg)
    F = o.init()
    F1, _ = o.step(F)
    assert np.max(np.abs(F1 - F)) / np.max(F) < 1e-14


def test_stiff_relaxation_stays_bounded():
    base = small_2d(16, 16, 8, kn=1e-5, mach=0.7, body=Body("circle", (0.5, 0.5, 0), (0.2, 0.2, 0), t_wall=1.3))
    f0, g0 = random_state(base.ncell, base.nv, 2, seed=21)
    for scheme, ok in (("imex", True), ("explicit", False)):
        o = Oracle2D(base.with_(scheme=scheme))
        f, g = o.merge(f0, g0)
        for _ in range(10):
            f, g, _ = o.step(f, g)
        bounded = np.all(np.isfinite(f)) and f.min() >= 0.0 and np.max(np.abs(f)) < 10 * np.max(f0)
        assert bounded == ok


def test_first_order_agreement_with_explicit():
    diffs = []
    for cfl in (0.2, 0.1, 0.05):
        cfg = small_2d(16, 16, 8, kn=0.5, mach=0.5, cfl=cfl)
        o = Oracle2D(cfg)
        f, g = o.merge(*o.init())
        # a smooth perturbation of the inflow state
        f = f * (1.0 + 0.2 * np.sin(np.arange(cfg.ncell) / 7.0))[:, None]
        a = Oracle2D(cfg).step(f, g)[0]
        b = Oracle2D(cfg.with_(scheme="imex")).step(f, g)[0]
        diffs.append(np.max(np.abs(a - b)))
    assert diffs[0] / diffs[1] > 3.5 and diffs[1] / diffs[2] > 3.5
