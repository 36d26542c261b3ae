"""GPU parity of the conservative equilibrium (Section 3.1, Newton on the
triplet) with the oracle, 2D and 3D, and its exact invariants on the GPU.

Tolerances as for the direct equilibrium: one step <= 1e-12 of max|f|,
tens of steps <= 1e-9, force <= 1e-10 of |F|, mass <= 1e-12.
"""
import numpy as np
import pytest

from ccdvm_inputs import Body, random_state, small_2d, small_3d, workload
from oracle import Oracle2D
from oracle.oracle import Oracle3D

pytestmark = pytest.mark.gpu

torch = pytest.importorskip("torch")


@pytest.fixture(scope="module", autouse=True)
def _gpu():
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    from paper_1503_04544_amd.solver import Solver  # noqa: F401


def solver(cfg):
    from paper_1503_04544_amd.solver import Solver
    return Solver(cfg, device="cuda:0")


def relerr(a, b):
    return float(np.max(np.abs(a - b)) / max(np.max(np.abs(b)), 1e-300))


C = "conservative"
CASES2 = {
    "cyl32_n8": small_2d(32, 32, 8, kn=0.1, mach=0.9, maxwellian=C),
    "tiny6_merge": small_2d(6, 6, 4, kn=0.07, mach=0.4, body=Body("circle", (0.5, 0.52, 0), (0.19, 0.19, 0)), maxwellian=C),
    "ragged_n12": small_2d(20, 14, 12, kn=0.3, mach=0.6, body=Body("circle", (0.45, 0.5, 0), (0.22, 0.22, 0), t_wall=1.4), maxwellian=C),
    # 32^2 velocities, as the 512x256 benchmark: the Newton solve over 32 nodes per axis
    "n32_ragged": small_2d(34, 22, 32, kn=0.05, mach=0.8, body=Body("circle", (0.5, 0.48, 0), (0.2, 0.2, 0)), maxwellian=C),
}
CASES3 = {
    "n16": small_3d(16, 8, 8, nv=16, kn=0.1, mach=0.5, maxwellian=C),
    "ragged_n8": small_3d(13, 7, 9, nv=8, kn=0.2, mach=0.9, body=Body("sphere", (0.45, 0.24, 0.26), (0.15,) * 3, t_wall=1.4), maxwellian=C),
    "tiny_n4_merge": small_3d(6, 5, 5, nv=4, kn=0.07, mach=0.4, body=Body("sphere", (0.5, 0.26, 0.24), (0.17,) * 3), maxwellian=C),
}


@pytest.mark.parametrize("name", sorted(CASES2))
def test_one_step_2d(name):
    cfg = CASES2[name]
    f0, g0 = random_state(cfg.ncell, cfg.nv, 2, seed=77)
    s = solver(cfg)
    s.load_state(torch.from_numpy(f0), torch.from_numpy(g0))
    d = s.step(1, diag=True).cpu().numpy()
    f1, g1 = (t.cpu().numpy() for t in s.store_state())
    fo, go, do = Oracle2D(cfg).step(f0, g0)
    assert relerr(f1, fo) < 1e-12
    assert relerr(g1, go) < 1e-12
    assert abs(d[0, 3] - do[3]) <= 1e-12 * abs(do[3])


def test_thirty_steps_2d():
    cfg = CASES2["cyl32_n8"]
    s = solver(cfg)
    s.init_maxwellian()
    d = s.step(30, diag=True).cpu().numpy()
    f1, g1 = (t.cpu().numpy() for t in s.store_state())
    o = Oracle2D(cfg)
    f, g = o.init()
    fo, go, do = o.run(f, g, 30)
    assert relerr(f1, fo) < 1e-9
    assert relerr(g1, go) < 1e-9
    assert np.max(np.abs(d[:, 0] - do[:, 0]) / np.abs(do[:, 0])) < 1e-9


@pytest.mark.parametrize("name", sorted(CASES3))
def test_one_step_3d(name):
    cfg = CASES3[name]
    f0, _ = random_state(cfg.ncell, cfg.nv, 3, seed=78, with_g=False)
    s = solver(cfg)
    s.load_state(torch.from_numpy(f0))
    d = s.step(1, diag=True).cpu().numpy()
    f1 = s.store_state()[0].cpu().numpy()
    fo, do = Oracle3D(cfg).step(f0)
    assert relerr(f1, fo) < 1e-12
    scale = max(np.max(np.abs(do[:3])), 1e-12)
    assert np.all(np.abs(d[0, :3] - do[:3]) <= 1e-10 * scale + 1e-15)


def test_twenty_steps_3d():
    cfg = CASES3["ragged_n8"]
    s = solver(cfg)
    s.init_maxwellian()
    s.step(20)
    f1 = s.store_state()[0].cpu().numpy()
    o = Oracle3D(cfg)
    fo, _ = o.run(o.init(), 20)
    assert relerr(f1, fo) < 1e-9


def test_rest_state_stationary_with_collisions_gpu():
    cfg = small_2d(32, 32, 16, kn=0.1, mach=0.0, maxwellian=C)
    s = solver(cfg)
    s.init_maxwellian()
    f0, g0 = (t.cpu().numpy() for t in s.store_state())
    s.step(5)
    f1, g1 = (t.cpu().numpy() for t in s.store_state())
    assert relerr(f1, f0) < 5e-14 and relerr(g1, g0) < 5e-14
    cfg = small_3d(12, 8, 8, nv=16, kn=0.1, mach=0.0, maxwellian=C)
    s = solver(cfg)
    s.init_maxwellian()
    F0 = s.store_state()[0].cpu().numpy()
    s.step(5)
    F1 = s.store_state()[0].cpu().numpy()
    assert relerr(F1, F0) < 5e-14


def test_adjoint_rejects_conservative():
    from paper_1503_04544_amd._capi import CCError
    s = solver(CASES2["cyl32_n8"])
    with pytest.raises(CCError):
        s.adjoint(2, 1)
