"""A body turning on the octree (Section 5, steps 1-7, with the mesh adapted
to the body every step): the GPU step against the oracle on every mesh the
body passes through.  Each step compares the leaf set, the leaf types, the
state of every leaf, the diag row (Fx, Fy, torque about the axis, mass) and
the body's angle and angular velocity.

Tolerances: one step 1e-12 of the largest value (reduction order of the
wall density and of the moments), 1e-10 after up to 12 steps (the
difference grows with the number of steps through the relaxation and the
torque feedback); mesh, types and leaf order exactly.
"""
import math

import numpy as np
import pytest

from ccdvm_inputs import Body
from ccdvm_inputs.configs import Config, _inflow, workload
from oracle.oracle import Oracle3A

pytestmark = pytest.mark.gpu

VANE = Body("vane", (0.5, 0.5, 0.25), (0.2, 0.06, 0.12), theta=math.pi / 8, inertia=0.01,
            motion="free_rotation", omega=20.0)


def vane_case(nv=4, depth=2, kn=0.1, body=VANE, n=(8, 8, 4), mach=0.5):
    return Config(dim=3, n=n, lo=(0.0, 0.0, 0.0), hi=(1.0, 1.0, 0.5), nv=nv, kn=kn, inflow=_inflow(mach),
                  body=body, amr_depth=depth)


def compare(cfg, nsteps, tol_first=1e-12, tol=1e-10, cells=None):
    from paper_1503_04544_amd.solver import Solver
    print(f"turning body: {cfg.body.kind} n={cfg.n} depth={cfg.amr_depth} N={cfg.nv} steps={nsteps}", flush=True)
    s = Solver(cfg, device="cuda:0")
    s.init_maxwellian()
    o = Oracle3A(cfg)
    F = o.init()
    counts = {s.ncell}
    for n in range(nsteps):
        d = s.step(1, diag=True).cpu().numpy()[0]
        F, do = o.step(F)
        counts.add(o.nleaf)
        assert s.ncell == o.nleaf
        L, Lo = s.amr_leaves(), o.leaves()
        for k in ("lvl", "ijk", "type", "master"):
            assert np.array_equal(L[k], Lo[k]), (n, k)
        Fg = s.store_state()[0].cpu().numpy()
        t = tol_first if n == 0 else tol
        scale = np.max(np.abs(F))
        assert np.max(np.abs(Fg - F)) <= t * scale, (n, np.max(np.abs(Fg - F)) / scale)
        for q in range(4):
            ref = abs(do[q]) if q == 3 else max(abs(do[0]), abs(do[1]), abs(do[2]))
            assert abs(d[q] - do[q]) <= t * max(ref, 1e-300), (n, q, d[q], do[q])
        b, bo = s.body_state(), o.body()
        assert abs(b[2] - bo[0]) <= 1e-14 * max(abs(bo[0]), 1.0) and abs(b[5] - bo[1]) <= t * abs(bo[1]) + 1e-300
    s.close()
    return counts


@pytest.mark.parametrize("nv", [4, 8])
def test_vane_one_step(nv):
    compare(vane_case(nv=nv), 1)


def test_vane_steps_through_changing_meshes():
    counts = compare(vane_case(nv=4), 12)
    assert len(counts) > 3          # leaves were split and merged on the way


def test_vane_collisionless_and_imposed_rotation():
    body = Body("vane", VANE.center, VANE.axes, theta=0.2, motion="imposed", omega=-15.0)
    compare(vane_case(nv=6, kn=0.0, body=body), 6)


def test_spinning_sphere():
    body = Body("sphere", (0.5, 0.5, 0.25), (0.15,) * 3, inertia=0.05, motion="free_rotation", omega=3.0)
    compare(vane_case(nv=8, body=body, mach=0.3), 4)


def test_vane_at_depth_zero_is_the_uniform_grid():
    body = Body("vane", VANE.center, (0.2, 0.05, 0.12), theta=0.4, inertia=0.01, motion="free_rotation",
                omega=10.0)
    compare(vane_case(nv=4, depth=0, n=(32, 32, 16), body=body), 3)


def test_vane_amr_full_size():
    cfg = workload("vane_amr")
    compare(cfg, 2)


def test_steps_without_diag_rows():
    from paper_1503_04544_amd.solver import Solver
    cfg = vane_case(nv=4)
    s = Solver(cfg, device="cuda:0")
    s.init_maxwellian()
    o = Oracle3A(cfg)
    F = o.init()
    s.step(3)                       # no diag rows: the torque goes through an internal row
    for _ in range(3):
        F, _ = o.step(F)
    assert s.ncell == o.nleaf
    Fg = s.store_state()[0].cpu().numpy()
    assert np.max(np.abs(Fg - F)) <= 1e-10 * np.max(np.abs(F))
    b, bo = s.body_state(), o.body()
    assert abs(b[2] - bo[0]) <= 1e-14 and abs(b[5] - bo[1]) <= 1e-10 * abs(bo[1])
    s.close()


def test_body_leaving_the_refined_band_is_rejected():
    # a turn of about two radians per step: coarse leaves are cut at the
    # next time; the host plan rejects the step before any kernel runs
    from paper_1503_04544_amd.solver import CCError, Solver
    body = Body("vane", VANE.center, VANE.axes, theta=0.3, motion="imposed", omega=2000.0)
    s = Solver(vane_case(nv=4, body=body), device="cuda:0")
    s.init_maxwellian()
    with pytest.raises(CCError) as e:
        s.step(1)
    assert e.value.status == -3
    s.close()
