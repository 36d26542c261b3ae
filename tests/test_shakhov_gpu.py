"""GPU parity of the Shakhov model (eq. ShakhovDD) with the oracle: fixed
and moving bodies, explicit and semi-implicit scheme, direct and
conservative triplet, and the full cyl512 size on sampled cells.

Tolerances as for BGK: one step <= 1e-12 of max|f|, 30 steps <= 1e-9
(moving bodies 1e-10 over 30 steps), force <= 1e-10 of |F|, mass <= 1e-12.
"""
import math

import numpy as np
import pytest

from ccdvm_inputs import Body, random_state, small_2d, workload
from oracle import Oracle2D

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


SK = dict(model="shakhov")
CASES = {
    "cyl32": workload("cyl32").with_(**SK),
    "tiny6_merge_pr03": small_2d(6, 6, 4, kn=0.07, mach=0.4, body=Body("circle", (0.5, 0.52, 0), (0.19, 0.19, 0)),
                                 prandtl=0.3, **SK),
    "ragged_n12_cons": small_2d(20, 14, 12, kn=0.3, mach=0.6, body=Body("circle", (0.45, 0.5, 0), (0.22, 0.22, 0),
                                t_wall=1.4), maxwellian="conservative", **SK),
    "n30_kn001": small_2d(24, 20, 30, kn=0.01, mach=0.5, body=Body("ellipse", (0.5, 0.5, 0), (0.25, 0.08, 0),
                          theta=0.7, t_wall=1.3), **SK),
    "cyl32_imex": workload("cyl32").with_(scheme="imex", kn=0.005, **SK),
    "ragged_n12_imex_cons": small_2d(20, 14, 12, kn=0.003, mach=0.6, body=Body("circle", (0.45, 0.5, 0),
                                     (0.22, 0.22, 0), t_wall=1.4), maxwellian="conservative", scheme="imex", **SK),
}


@pytest.mark.parametrize("name", sorted(CASES))
def test_one_step_from_random_state(name):
    cfg = CASES[name]
    f0, g0 = random_state(cfg.ncell, cfg.nv, 2, seed=77)
    s = solver(cfg)
    s.load_state(torch.from_numpy(f0), torch.from_numpy(g0))
    d = s.step(1, diag=True).cpu().numpy()
    f1, g1 = (t.cpu().numpy() for t in s.store_state())
    fo, go, do = Oracle2D(cfg).step(f0, g0)
    assert relerr(f1, fo) < 1e-12
    assert relerr(g1, go) < 1e-12
    scale = max(abs(do[0]), abs(do[1]), 1e-12)
    assert np.all(np.abs(d[0, :3] - do[:3]) <= 1e-10 * scale + 1e-15)
    assert abs(d[0, 3] - do[3]) <= 1e-12 * abs(do[3])
    # the Shakhov term matters in this case
    fb = Oracle2D(cfg.with_(model="bgk")).step(f0, g0)[0]
    assert relerr(fb, fo) > 1e-9


@pytest.mark.parametrize("name", ["cyl32", "cyl32_imex", "ragged_n12_cons"])
def test_thirty_steps(name):
    cfg = CASES[name]
    s = solver(cfg)
    s.init_maxwellian()
    d = s.step(30, diag=True).cpu().numpy()
    f1, g1 = (t.cpu().numpy() for t in s.store_state())
    o = Oracle2D(cfg)
    fo, go, do = o.run(*o.init(), 30)
    assert relerr(f1, fo) < 1e-9
    assert relerr(g1, go) < 1e-9
    assert np.max(np.abs(d[:, 0] - do[:, 0])) <= 1e-9 * np.max(np.abs(do[:, 0]))
    assert np.max(np.abs(d[:, 3] - do[:, 3]) / do[:, 3]) < 1e-12


MOVING = {
    "free_rotation_shakhov": small_2d(48, 40, 12, kn=0.1, mach=0.6, body=Body(
        "ellipse", (0.5, 0.5, 0), (0.15, 0.06, 0), theta=math.pi / 8, motion="free_rotation", inertia=0.002,
        t_wall=1.3), **SK),
    "translating_circle_shakhov": small_2d(48, 48, 8, kn=0.2, mach=0.3, body=Body(
        "circle", (0.45, 0.5, 0), (0.15, 0.15, 0), motion="imposed", vel=(1.0, 0.3, 0.0), t_wall=1.3), **SK),
}


@pytest.mark.parametrize("name", sorted(MOVING))
def test_moving_steps(name):
    cfg = MOVING[name]
    s = solver(cfg)
    s.init_maxwellian()
    d = s.step(30, diag=True).cpu().numpy()
    f1, g1 = (t.cpu().numpy() for t in s.store_state())
    o = Oracle2D(cfg)
    fo, go, do = o.run(*o.init(), 30)
    assert relerr(f1, fo) < 1e-10
    assert relerr(g1, go) < 1e-10
    assert np.max(np.abs(d[:, 3] - do[:, 3]) / do[:, 3]) < 1e-12
    assert np.allclose(s.body_state(), o.body_state(), rtol=1e-10, atol=1e-13)


def test_cyl512_full_size_sampled_cells():
    cfg = workload("cyl512").with_(**SK)
    f0, g0 = random_state(cfg.ncell, cfg.nv, 2, seed=513)
    s = solver(cfg)
    s.load_state(torch.from_numpy(f0), torch.from_numpy(g0))
    s.step(1)
    f1, g1 = s.store_state()
    o = Oracle2D(cfg)
    geo = o.geometry()
    nx, ny = cfg.n[0], cfg.n[1]
    rng = np.random.default_rng(1)
    cut = np.nonzero((geo["type"] == 1) | ((geo["master"] >= 0) & (geo["master"] != np.arange(cfg.ncell))))[0]
    edges = np.concatenate([np.arange(nx), (ny - 1) * nx + np.arange(nx),
                            np.arange(ny) * nx, np.arange(ny) * nx + nx - 1])
    cells = np.unique(np.concatenate([cut, edges[::7], rng.integers(0, cfg.ncell, 400)])).astype(np.int32)
    fm, gm = o.merge(f0, g0)
    fo, go = o.update_cells(fm, gm, cells)
    idx = torch.from_numpy(cells.astype(np.int64)).to(f1.device)
    assert relerr(f1.index_select(0, idx).cpu().numpy(), fo) < 1e-12
    assert relerr(g1.index_select(0, idx).cpu().numpy(), go) < 1e-12


def test_prandtl_one_equals_bgk_gpu():
    cfg = workload("cyl32")
    f0, g0 = random_state(cfg.ncell, cfg.nv, 2, seed=78)
    out = []
    for c in (cfg, cfg.with_(model="shakhov", prandtl=1.0)):
        s = solver(c)
        s.load_state(torch.from_numpy(f0), torch.from_numpy(g0))
        s.step(3)
        out.append(s.store_state()[0].cpu().numpy())
    assert relerr(out[1], out[0]) < 1e-14


def test_adjoint_rejects_shakhov():
    from paper_1503_04544_amd._capi import CCError
    s = solver(CASES["cyl32"])
    with pytest.raises(CCError):
        s.adjoint(2, 1)


# ---------------------------------------------------------------- 3D
from ccdvm_inputs import small_3d  # noqa: E402
from oracle.oracle import Oracle3D  # noqa: E402

CASES3 = {
    "n16": small_3d(16, 8, 8, nv=16, kn=0.01, mach=0.5, **SK),
    "ragged_n8_cons": small_3d(13, 7, 9, nv=8, kn=0.05, mach=0.9, body=Body("sphere", (0.45, 0.24, 0.26), (0.15,) * 3,
                               t_wall=1.4), maxwellian="conservative", **SK),
    "n6_merge_pr03": small_3d(6, 5, 5, nv=6, kn=0.02, mach=0.4, body=Body("sphere", (0.5, 0.26, 0.24), (0.17,) * 3),
                              prandtl=0.3, **SK),
    "n16_imex": small_3d(16, 8, 8, nv=16, kn=0.002, mach=0.5, scheme="imex", **SK),
    "n12_imex_cons": small_3d(12, 9, 8, nv=12, kn=0.003, mach=0.7, body=Body("sphere", (0.5, 0.3, 0.25), (0.14,) * 3,
                              t_wall=1.2), scheme="imex", maxwellian="conservative", **SK),
}


@pytest.mark.parametrize("name", sorted(CASES3))
def test_one_step_3d(name):
    cfg = CASES3[name]
    F0, _ = random_state(cfg.ncell, cfg.nv, 3, seed=79, with_g=False)
    s = solver(cfg)
    s.load_state(torch.from_numpy(F0))
    d = s.step(1, diag=True).cpu().numpy()
    F1 = s.store_state()[0].cpu().numpy()
    Fo, do = Oracle3D(cfg).step(F0)
    assert relerr(F1, Fo) < 1e-12
    scale = max(np.max(np.abs(do[:3])), 1e-12)
    assert np.all(np.abs(d[0, :3] - do[:3]) <= 1e-10 * scale + 1e-15)
    assert abs(d[0, 3] - do[3]) <= 1e-12 * abs(do[3])
    Fb = Oracle3D(cfg.with_(model="bgk")).step(F0)[0]
    assert relerr(Fb, Fo) > 1e-9


@pytest.mark.parametrize("name", ["n16", "ragged_n8_cons", "n16_imex"])
def test_twenty_steps_3d(name):
    cfg = CASES3[name]
    s = solver(cfg)
    s.init_maxwellian()
    d = s.step(20, diag=True).cpu().numpy()
    F1 = s.store_state()[0].cpu().numpy()
    o = Oracle3D(cfg)
    Fo, do = o.run(o.init(), 20)
    assert relerr(F1, Fo) < 1e-9
    assert np.max(np.abs(d[:, 3] - do[:, 3]) / do[:, 3]) < 1e-12


@pytest.mark.timeout(900)
def test_sphere128_full_size_sampled_cells():
    """Full sphere128 size (128 x 64 x 64 cells, 16^3 velocities) with the
    Shakhov model: one step from a seeded state, sampled cells (cut and
    merged control volumes, domain faces, random interior cells)
    recomputed by the oracle."""
    from ccdvm_inputs import tiled_random_state
    cfg = workload("sphere128").with_(**SK)
    f0 = tiled_random_state(cfg.ncell, cfg.nv, 3, seed=129)
    s = solver(cfg)
    s.load_state(torch.from_numpy(f0))
    s.step(1)
    f1 = s.store_state()[0]
    o = Oracle3D(cfg)
    geo = o.geometry()
    nx, ny, nz = cfg.n
    idx = np.arange(cfg.ncell)
    ii, jj, kk = idx % nx, (idx // nx) % ny, idx // (nx * ny)
    rng = np.random.default_rng(3)
    cut = np.nonzero((geo["type"] == 1) | ((geo["master"] >= 0) & (geo["master"] != idx)))[0]
    faces = idx[(ii == 0) | (ii == nx - 1) | (jj == 0) | (jj == ny - 1) | (kk == 0) | (kk == nz - 1)]
    cells = np.unique(np.concatenate([cut, faces[::97], rng.integers(0, cfg.ncell, 300)])).astype(np.int32)
    fm = o.merge(f0)
    del f0
    fo = o.update_cells(fm, cells)
    del fm
    sel = f1.index_select(0, torch.from_numpy(cells.astype(np.int64)).to(f1.device)).cpu().numpy()
    assert relerr(sel, fo) < 1e-12
