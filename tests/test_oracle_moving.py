"""Pins of the oracle's moving-body step (seven-step summary, Section 3.3.4).

* Mass is conserved to round-off by the cut-cell scheme with a moving body
  (the proof of Section 3.4.2 covers the area ratio S^n/S^{n+1,*} and the
  appearing/disappearing cells): rotating ellipse, pure transport, gas at
  rest, before any disturbance reaches the outer faces.
* An ellipse aligned with a uniform flow feels no torque (symmetry), so a
  body free to rotate stays at rest to round-off.
* An imposed rotation advances the angle by dt*omega per step exactly
  (eq. motionDD_posit), and a body with zero velocity takes the same step
  as a fixed body (the moving machinery reduces to the fixed one).
* Free rotation integrates the torque with explicit Euler (eq.
  motionDD_vit): omega^{n+1} - omega^n = dt T^n / J for every step.
"""
import math

import numpy as np
import pytest

from ccdvm_inputs import Body, small_2d
from oracle import Oracle2D


def _ellipse(motion, omega=0.0, theta=math.pi / 8, kn=0.0, mach=0.0, n=48, nv=12, inertia=0.01):
    return small_2d(n, n, nv, kn=kn, mach=mach,
                    body=Body("ellipse", (0.5, 0.5, 0), (0.15, 0.06, 0), theta=theta,
                              motion=motion, omega=omega, inertia=inertia))


def test_mass_conserved_with_rotating_body():
    cfg = _ellipse("imposed", omega=20.0)
    o = Oracle2D(cfg)
    f, g = o.init()
    f, g, d = o.run(f, g, 12)
    assert np.max(np.abs(d[:, 3] - d[0, 3])) / d[0, 3] < 1e-13
    assert np.all(f >= 0.0)
    # the body did move: the angle advanced by 12 dt omega exactly
    s = o.body_state()
    assert s[2] == pytest.approx(math.pi / 8 + 12 * o.dt * 20.0, rel=1e-14)


def test_zero_velocity_moving_step_equals_fixed_step():
    fixed = Oracle2D(_ellipse("fixed", kn=0.1, mach=0.5))
    moving = Oracle2D(_ellipse("imposed", omega=0.0, kn=0.1, mach=0.5))
    f, g = fixed.init()
    f1, g1, d1 = fixed.run(f, g, 3)
    f2, g2, d2 = moving.run(f, g, 3)
    assert np.max(np.abs(f1 - f2)) <= 1e-15 * np.max(f1)
    assert np.allclose(d1, d2, rtol=1e-14, atol=1e-16)


def test_symmetric_ellipse_feels_no_torque():
    cfg = _ellipse("free_rotation", theta=0.0, kn=0.1, mach=0.5)
    o = Oracle2D(cfg)
    f, g = o.init()
    f, g, d = o.run(f, g, 6)
    assert np.max(np.abs(d[:, 2])) < 1e-14
    assert abs(o.body_state()[5]) < 1e-12


def test_free_rotation_is_explicit_euler_on_the_torque():
    cfg = _ellipse("free_rotation", theta=math.pi / 8, kn=0.1, mach=0.6, inertia=0.05)
    o = Oracle2D(cfg)
    f, g = o.init()
    omegas, thetas, torques = [], [], []
    for _ in range(5):
        s = o.body_state()
        omegas.append(s[5]); thetas.append(s[2])
        f, g, d = o.step(f, g)
        torques.append(d[2])
    s = o.body_state()
    omegas.append(s[5]); thetas.append(s[2])
    assert abs(torques[0]) > 1e-6
    for n in range(5):
        assert omegas[n + 1] - omegas[n] == pytest.approx(o.dt * torques[n] / 0.05, rel=1e-12)
        # the difference of two angles ~0.4 carries their rounding (~1e-16)
        assert thetas[n + 1] - thetas[n] == pytest.approx(o.dt * omegas[n], rel=1e-12, abs=2e-16)


def test_spinning_circle_torque_is_the_free_molecular_torque():
    """A circle of radius R spinning at imposed angular velocity omega in a
    gas at rest (rho = 1, T = 1) with an isothermal diffuse wall
    (eqs. uwDD, BoundaryDDv, StressTensorDD, eq-torque).  In the first step
    the incident molecules carry no tangential momentum, and the re-emitted
    ones leave at the incident mass flux m = int_{c_n > 0} c_n M dc_n with
    the wall's tangential velocity omega R, so the gas pulls the wall back
    with the shear m omega R per unit length: torque -2 pi R^2 m omega R per
    unit length of cylinder (m is integrated numerically here).  The
    oracle's first-step torque must have that sign and scale, converge to it
    in the grid spacing, and be odd in omega with no net force.  A reversed
    wall velocity (r - c)^perp or a wrong torque orientation flips the sign;
    a wall velocity left out of the re-emitted Maxwellian gives zero."""
    from scipy.integrate import quad
    R = 0.25
    m, _ = quad(lambda c: c * math.exp(-0.5 * c * c) / math.sqrt(2.0 * math.pi), 0.0, math.inf)
    errs = []
    for n in (32, 64, 128):
        torques = []
        for omega in (1.0, -1.0):
            cfg = small_2d(n, n, 24, kn=0.1, mach=0.0,
                           body=Body("circle", (0.5, 0.5, 0), (R, R, 0), motion="imposed", omega=omega))
            o = Oracle2D(cfg)
            f, g = o.init()
            _, _, d = o.step(f, g)
            exact = -2.0 * math.pi * R * R * m * omega * R
            assert d[2] * exact > 0.0
            assert abs(d[0]) < 1e-14 and abs(d[1]) < 1e-14
            torques.append(d[2])
            if omega > 0:
                errs.append(abs(d[2] - exact) / abs(exact))
        assert torques[0] == pytest.approx(-torques[1], rel=1e-13)
    assert errs[0] < 7e-3 and errs[1] < 1.5e-3 and errs[2] < 6e-4, errs
    assert errs[2] < errs[1] < errs[0]
