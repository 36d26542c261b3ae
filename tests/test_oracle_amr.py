"""Pins of the oracle's octree mesh (Section 5.1, octree procedure) around a
fixed sphere:

* with no refinement it is the uniform 3D oracle (bitwise, leaves permuted);
  refined everywhere to depth 1 it is the uniform oracle on the doubled grid;
* the leaves tile the domain, obey the refinement criterion (checked from
  the level set, not from the oracle's decisions) and differ by at most one
  depth across a face;
* every face list equals a brute-force search over all leaf pairs for
  shared faces and their overlap areas;
* cut cells lie at the finest depth and have the uniform grid's geometry
  there; one step from the farfield state gives the same force and the same
  cut-cell values as the uniform grid of the finest spacing;
* a gas at rest with an isothermal wall stays at rest across depth jumps;
  without collisions the change of mass equals the net farfield flux.
"""
import math

import numpy as np
import pytest

from ccdvm_inputs import Body, random_state, small_3d
from oracle.oracle import Oracle3A, Oracle3D

SPH = Body("sphere", (0.5, 0.25, 0.25), (0.1,) * 3)


def case(n=(16, 8, 8), nv=4, depth=1, **kw):
    kw.setdefault("body", SPH)
    return small_3d(*n, nv=nv, kn=kw.pop("kn", 0.1), mach=kw.pop("mach", 0.5), amr_depth=depth,
                    lo=(0.0, 0.0, 0.0), hi=(1.0, 0.5, 0.5), **kw)


def uniform_index(L, n, depth):
    """uniform-grid cell index of every leaf of depth `depth`"""
    i, j, k = L["ijk"][:, 0], L["ijk"][:, 1], L["ijk"][:, 2]
    return (k * n[1] + j) * n[0] + i


@pytest.mark.parametrize("scheme,model", [("explicit", "bgk"), ("imex", "shakhov")])
def test_depth_zero_is_the_uniform_grid(scheme, model):
    cfg = case(depth=0, nv=6, scheme=scheme, model=model)
    a, u = Oracle3A(cfg), Oracle3D(cfg.with_(amr_depth=0))
    L = a.leaves()
    idx = uniform_index(L, cfg.n, 0)
    assert a.nleaf == u.ncell and np.array_equal(np.sort(idx), np.arange(u.ncell))
    F, _ = random_state(u.ncell, cfg.nv, 3, seed=61, with_g=False)
    Fu, du = u.step(F)
    Fa, da = a.step(F[idx])
    assert a.dt == u.dt
    assert np.array_equal(Fa, Fu[idx])
    assert np.allclose(da, du, rtol=1e-13, atol=1e-17)   # force sums run in another order


def test_refined_everywhere_is_the_doubled_uniform_grid():
    cfg = case(n=(8, 4, 4), depth=1, amr_band=1e9)
    a = Oracle3A(cfg)
    L = a.leaves()
    assert np.all(L["lvl"] == 1)
    n2 = (16, 8, 8)
    u = Oracle3D(cfg.with_(n=n2, amr_depth=0))
    idx = uniform_index(L, n2, 1)
    g = u.geometry()
    assert np.array_equal(L["type"], g["type"][idx])
    inv = np.empty(u.ncell, np.int64); inv[idx] = np.arange(u.ncell)
    m = L["master"]
    assert np.array_equal(np.where(m >= 0, idx[np.maximum(m, 0)], -1), g["master"][idx])
    F, _ = random_state(u.ncell, cfg.nv, 3, seed=62, with_g=False)
    Fu, du = u.step(F)
    Fa, da = a.step(F[idx])
    assert np.array_equal(Fa, Fu[idx])
    assert abs(da[3] - du[3]) <= 1e-14 * du[3]


def boxes(a, cfg):
    L = a.leaves()
    h0 = [(cfg.hi[d] - cfg.lo[d]) / cfg.n[d] for d in range(3)]
    s = 1.0 / (1 << L["lvl"])
    lo = np.stack([cfg.lo[d] + L["ijk"][:, d] * h0[d] * s for d in range(3)], 1)
    hi = np.stack([cfg.lo[d] + (L["ijk"][:, d] + 1) * h0[d] * s for d in range(3)], 1)
    return L, lo, hi, h0


@pytest.mark.parametrize("depth", [1, 2, 3])
def test_leaves_tile_and_obey_the_criterion(depth):
    cfg = case(depth=depth)
    a = Oracle3A(cfg)
    L, lo, hi, h0 = boxes(a, cfg)
    vol = np.prod(hi - lo, axis=1)
    assert abs(vol.sum() - 1.0 * 0.5 * 0.5) < 1e-12
    Dx = max(h0)
    c = 0.5 * (lo + hi)
    dist = np.abs(np.linalg.norm(c - np.array(SPH.center), axis=1) - SPH.axes[0])
    band = 2 * math.sqrt(2)
    lvl = L["lvl"]
    # a leaf above the finest depth is outside the band; its parent was inside
    assert np.all(dist[lvl < depth] >= band * Dx / (1 << lvl[lvl < depth]))
    pc = np.stack([cfg.lo[d] + ((L["ijk"][:, d] >> 1) + 0.5) * h0[d] * 2.0 / (1 << lvl) for d in range(3)], 1)
    pdist = np.abs(np.linalg.norm(pc - np.array(SPH.center), axis=1) - SPH.axes[0])
    sub = lvl > 0
    assert np.all(pdist[sub] < band * Dx * 2.0 / (1 << lvl[sub]))
    # cut cells only at the finest depth
    assert np.all(lvl[L["type"] == 1] == depth) and np.sum(L["type"] == 1) > 0
    # at most one depth across a face
    f = a.faces()
    for q in range(a.nleaf):
        for e in range(f["ptr"][q], f["ptr"][q + 1]):
            nb = f["nb"][e]
            if nb >= 0:
                assert abs(int(lvl[nb]) - int(lvl[q])) <= 1


def test_face_lists_equal_brute_force_overlaps():
    cfg = case(n=(8, 4, 4), depth=2)
    a = Oracle3A(cfg)
    L, lo, hi, h0 = boxes(a, cfg)
    f = a.faces()
    gas = L["type"] == 0
    n = a.nleaf
    tol = 1e-12
    dom_lo, dom_hi = np.array(cfg.lo), np.array(cfg.hi)
    for q in np.nonzero(gas)[0]:
        expect = {}
        for t in range(6):
            d, sd = t >> 1, t & 1
            plane = hi[q, d] if sd else lo[q, d]
            # candidates touching the plane from the other side
            other = lo[:, d] if sd else hi[:, d]
            cand = np.nonzero(np.abs(other - plane) < tol)[0]
            d1, d2 = (d + 1) % 3, (d + 2) % 3
            tot = 0.0
            for y in cand:
                o1 = min(hi[q, d1], hi[y, d1]) - max(lo[q, d1], lo[y, d1])
                o2 = min(hi[q, d2], hi[y, d2]) - max(lo[q, d2], lo[y, d2])
                if o1 > tol and o2 > tol and L["type"][y] != 2:
                    expect[(int(y), t)] = o1 * o2
                    tot += o1 * o2
            full = (hi[q, d1] - lo[q, d1]) * (hi[q, d2] - lo[q, d2])
            on_boundary = abs(plane - (dom_hi[d] if sd else dom_lo[d])) < tol
            if on_boundary:
                expect[(-1, t)] = full
        got = {}
        for e in range(f["ptr"][q], f["ptr"][q + 1]):
            got[(int(f["nb"][e]), int(f["dir"][e]))] = f["area"][e]
        assert set(got) == set(expect), q
        for key in got:
            assert abs(got[key] - expect[key]) <= 1e-12 * expect[key]


def test_cut_cells_match_the_finest_uniform_grid_and_first_step():
    depth = 2
    cfg = case(n=(8, 4, 4), depth=depth, nv=6, kn=0.05)
    a = Oracle3A(cfg)
    nf = tuple(x << depth for x in cfg.n)
    u = Oracle3D(cfg.with_(n=nf, amr_depth=0))
    L, g = a.leaves(), u.geometry()
    fine = L["lvl"] == depth
    idx = uniform_index(L, nf, depth)
    q = np.nonzero(fine)[0]
    ui = idx[q]
    assert np.array_equal(L["type"][q], g["type"][ui])
    assert np.array_equal(L["sw"][q], g["sw"][ui]) and np.array_equal(L["vbar"][q], g["vbar"][ui])
    assert np.array_equal(L["S"][q], g["S"][ui])
    cut = q[L["type"][q] == 1]
    m = L["master"][cut]
    assert np.array_equal(idx[m], g["master"][idx[cut]])
    assert a.dt == u.dt
    # one step from the farfield state: same force, same values in cut cells
    Fa, da = a.step(a.init())
    Fu, du = u.step(u.init())
    assert np.allclose(da[:3], du[:3], rtol=1e-13, atol=1e-16) and np.max(np.abs(du[:3])) > 1e-6
    assert np.max(np.abs(Fa[cut] - Fu[idx[cut]])) <= 1e-14 * np.max(Fu)


def test_rest_state_stays_at_rest_across_depth_jumps():
    for extra in ({"kn": 0.0}, {"kn": 0.1, "maxwellian": "conservative"}):
        cfg = case(depth=2, nv=6, mach=0.0, **extra)
        a = Oracle3A(cfg)
        assert len(np.unique(a.leaves()["lvl"])) == 3
        F0 = a.init()
        F1, d = a.step(F0)
        assert np.max(np.abs(F1 - F0)) <= 1e-14 * np.max(F0)
        assert np.max(np.abs(d[:3])) < 1e-14


def test_mass_change_equals_farfield_flux_collisionless():
    cfg = case(depth=2, nv=4, kn=0.0, mach=0.8)
    a = Oracle3A(cfg)
    F0, _ = random_state(a.nleaf, cfg.nv, 3, seed=63, with_g=False)
    L = a.leaves()
    F0[L["type"] == 2] = 0.0
    F0 = a.merge(F0)
    F1, d0 = a.step(F0)
    _, d1 = a.step(F1)
    v = a.velocity()
    N = cfg.nv
    vd = [np.tile(v, N * N), np.tile(np.repeat(v, N), N), np.repeat(v, N * N)]
    w = (v[1] - v[0]) ** 3
    rho, ux, uy, uz, T = cfg.inflow
    ghost = rho / (2 * np.pi * T) ** 1.5 * np.exp(-((vd[0] - ux) ** 2 + (vd[1] - uy) ** 2 + (vd[2] - uz) ** 2) / (2 * T))
    f = a.faces()
    net = 0.0
    for q in range(a.nleaf):
        for e in range(f["ptr"][q], f["ptr"][q + 1]):
            if f["nb"][e] >= 0:
                continue
            t = f["dir"][e]
            c = vd[t >> 1] if t & 1 else -vd[t >> 1]
            net += f["area"][e] * np.sum(np.maximum(c, 0) * F0[q] + np.minimum(c, 0) * ghost) * w
    assert abs((d1[3] - d0[3]) + a.dt * net) <= 1e-12 * d0[3]
    assert abs(d1[3] - d0[3]) > 1e-8 * d0[3]
