"""GPU parity of the moving-body step (geometry rebuilt every step on the
device, area ratio S^n/S^{n+1,*}, appearing/disappearing cells, wall
velocity, rigid-body update) with the oracle."""
import math

import numpy as np
import pytest

from ccdvm_inputs import Body, small_2d, workload
from oracle import Oracle2D

pytestmark = pytest.mark.gpu
torch = pytest.importorskip("torch")


@pytest.fixture(scope="module", autouse=True)
def _gpu():
    if not torch.cuda.is_available():
        pytest.skip("no GPU")


def solver(cfg):
    from paper_1503_04544_amd.solver import Solver
    return Solver(cfg, device="cuda:0")


def relerr(a, b):
    return float(np.max(np.abs(a - b)) / max(np.max(np.abs(b)), 1e-300))


MOVING = {
    "rotating_collisionless": small_2d(48, 48, 12, kn=0.0, mach=0.0, body=Body(
        "ellipse", (0.5, 0.5, 0), (0.15, 0.06, 0), theta=math.pi / 8, motion="imposed", omega=20.0)),
    "free_rotation_bgk": small_2d(48, 40, 12, kn=0.1, mach=0.6, body=Body(
        "ellipse", (0.5, 0.5, 0), (0.15, 0.06, 0), theta=math.pi / 8, motion="free_rotation",
        inertia=0.002)),
    "translating_circle": small_2d(48, 48, 8, kn=0.2, mach=0.3, body=Body(
        "circle", (0.45, 0.5, 0), (0.15, 0.15, 0), motion="imposed", vel=(1.0, 0.3, 0.0), t_wall=1.3)),
    # the free-molecular torque pin's set-up: a circle spinning in a gas at rest
    "spinning_circle": small_2d(48, 48, 16, kn=0.1, mach=0.0, body=Body(
        "circle", (0.5, 0.5, 0), (0.25, 0.25, 0), motion="imposed", omega=3.0)),
}


@pytest.mark.parametrize("name", sorted(MOVING))
def test_moving_steps_match_oracle(name):
    cfg = MOVING[name]
    nsteps = 40
    s = solver(cfg)
    s.init_maxwellian()
    d = s.step(nsteps, diag=True).cpu().numpy()
    f1, g1 = (t.cpu().numpy() for t in s.store_state())
    o = Oracle2D(cfg)
    f, g = o.init()
    fo, go, do = o.run(f, g, nsteps)
    assert relerr(f1, fo) < 1e-10
    assert relerr(g1, go) < 1e-10
    assert np.max(np.abs(d[:, 3] - do[:, 3]) / do[:, 3]) < 1e-12
    fs = max(np.max(np.abs(do[:, :3])), 1e-12)
    assert np.max(np.abs(d[:, :3] - do[:, :3])) < 1e-9 * fs
    assert np.allclose(s.body_state(), o.body_state(), rtol=1e-10, atol=1e-13)
    # the geometry of the current time level is the oracle's
    gg, go_ = s.geometry(), o.geometry()
    assert np.array_equal(gg["type"], go_["type"])
    assert np.array_equal(gg["master"], go_["master"])


def test_rotating_body_conserves_mass_gpu():
    cfg = MOVING["rotating_collisionless"]
    s = solver(cfg)
    s.init_maxwellian()
    d = s.step(12, diag=True).cpu().numpy()
    assert np.max(np.abs(d[:, 3] - d[0, 3])) / d[0, 3] < 1e-13


def test_ellipse256_full_size_two_steps():
    """The moving workload at full size (256^2 cells, 40^2 velocities, free
    rotation), two steps against the oracle."""
    cfg = workload("ellipse256")
    s = solver(cfg)
    s.init_maxwellian()
    d = s.step(2, diag=True).cpu().numpy()
    f1, g1 = (t.cpu().numpy() for t in s.store_state())
    o = Oracle2D(cfg)
    f, g = o.init()
    fo, go, do = o.run(f, g, 2)
    assert relerr(f1, fo) < 1e-12
    assert relerr(g1, go) < 1e-12
    assert np.max(np.abs(d[:, 2] - do[:, 2])) < 1e-10 * np.max(np.abs(do[:, 2]))
    assert np.allclose(s.body_state(), o.body_state(), rtol=1e-12, atol=1e-15)
