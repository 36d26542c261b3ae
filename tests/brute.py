"""Brute-force face-loop reference of one fixed-geometry step (tiny grids only).

A second, differently organised formulation of the explicit cut-cell step
(eqs. FusionDD, FluxDD, BoundaryDDv, ExSchemeDD, UpdateDD): every Cartesian
face is visited once and its upwind flux is added to the control volume on
its left/bottom and subtracted from the one on its right/top; every wall edge
adds its flux to its own control volume.  It takes the geometry tables as
input (pinned separately against analytic clipping) and uses pure Python
loops, so it is only meant for grids of a few cells and velocities.
"""
from __future__ import annotations

import math

import numpy as np


def maxwellian(rho, ux, uy, T, vx, vy):
    return rho / (2 * math.pi * T) * math.exp(-((vx - ux) ** 2 + (vy - uy) ** 2) / (2 * T))


def shakhov_2d(cfg, vel, w, rho, ux, uy, T, f, g, M):
    """(f_eq, g_eq): eq. BGKDD, or eq. ShakhovDD when cfg.model is "shakhov",
    with the heat flux of (f, g) about their own mean velocity."""
    if getattr(cfg, "model", "bgk") != "shakhov":
        return M, 0.5 * T * M
    vx = np.array([a for a, _ in vel])
    vy = np.array([b for _, b in vel])
    mux, muy = (vx * f).sum() / f.sum(), (vy * f).sum() / f.sum()
    cxd, cyd = vx - mux, vy - muy
    h = 0.5 * (cxd ** 2 + cyd ** 2) * f + g
    qx, qy = (cxd * h).sum() * w, (cyd * h).sum() * w
    cx, cy = vx - ux, vy - uy
    c2 = (cx ** 2 + cy ** 2) / T
    s = (1 - cfg.prandtl) * (cx * qx + cy * qy) / (5 * rho * T * T)
    return M * (1 + s * (c2 - 4)), 0.5 * T * M * (1 + s * (c2 - 2))


def brute_step(cfg, geo, v, dt, f, g, collide=True, imex=False):
    nx, ny = cfg.n[0], cfg.n[1]
    N = cfg.nv
    nvel = N * N
    dv = (cfg.vmax - cfg.vmin) / N
    w = dv * dv
    rho_in, ux_in, uy_in, _, T_in = cfg.inflow
    Tw = cfg.body.t_wall
    vel = [(v[p % N], v[p // N]) for p in range(nvel)]
    ghost_f = [maxwellian(rho_in, ux_in, uy_in, T_in, vx, vy) for vx, vy in vel]
    ghost_g = [0.5 * T_in * x for x in ghost_f]
    master = geo["master"]
    ncell = nx * ny
    f = f.copy()
    g = g.copy()
    # merge: S_CV f_CV = sum Sbar f over the members
    groups = {}
    for c in range(ncell):
        if master[c] >= 0:
            groups.setdefault(int(master[c]), []).append(c)
    for m, mem in groups.items():
        if len(mem) > 1:
            fc = sum(geo["sbar"][c] * f[c] for c in mem) / geo["scv"][m]
            gc = sum(geo["sbar"][c] * g[c] for c in mem) / geo["scv"][m]
            for c in mem:
                f[c] = fc
                g[c] = gc
    Rf = {m: np.zeros(nvel) for m in groups}
    Rg = {m: np.zeros(nvel) for m in groups}

    def val(arr, ghost, i, j, p):
        if 0 <= i < nx and 0 <= j < ny:
            return arr[j * nx + i][p]
        return ghost[p]

    # vertical faces x = x_{a-1/2}: cells (a-1, j) | (a, j)
    for j in range(ny):
        for a in range(nx + 1):
            L = geo["lxm"][j * nx + a] if a < nx else geo["lxp"][j * nx + nx - 1]
            if L == 0.0:
                continue
            for p in range(nvel):
                vx = vel[p][0]
                F = L * (min(vx, 0) * val(f, ghost_f, a, j, p) + max(vx, 0) * val(f, ghost_f, a - 1, j, p))
                G = L * (min(vx, 0) * val(g, ghost_g, a, j, p) + max(vx, 0) * val(g, ghost_g, a - 1, j, p))
                if a - 1 >= 0:
                    m = int(master[j * nx + a - 1]); Rf[m][p] += F; Rg[m][p] += G
                if a < nx:
                    m = int(master[j * nx + a]); Rf[m][p] -= F; Rg[m][p] -= G
    # horizontal faces y = y_{b-1/2}: cells (i, b-1) | (i, b)
    for b in range(ny + 1):
        for i in range(nx):
            L = geo["lym"][b * nx + i] if b < ny else geo["lyp"][(ny - 1) * nx + i]
            if L == 0.0:
                continue
            for p in range(nvel):
                vy = vel[p][1]
                F = L * (min(vy, 0) * val(f, ghost_f, i, b, p) + max(vy, 0) * val(f, ghost_f, i, b - 1, p))
                G = L * (min(vy, 0) * val(g, ghost_g, i, b, p) + max(vy, 0) * val(g, ghost_g, i, b - 1, p))
                if b - 1 >= 0:
                    m = int(master[(b - 1) * nx + i]); Rf[m][p] += F; Rg[m][p] += G
                if b < ny:
                    m = int(master[b * nx + i]); Rf[m][p] -= F; Rg[m][p] -= G
    # wall edges (fixed body: wall velocity zero)
    for k in range(ncell):
        L = geo["lw"][k]
        if L <= 0.0:
            continue
        n = (geo["nwx"][k], geo["nwy"][k])
        cn = [vx * n[0] + vy * n[1] for vx, vy in vel]
        Mw = [maxwellian(1.0, 0.0, 0.0, Tw, vx, vy) for vx, vy in vel]
        num = sum(cn[p] * f[k][p] * w for p in range(nvel) if cn[p] > 0)
        den = sum(cn[p] * Mw[p] * w for p in range(nvel) if cn[p] < 0)
        phi = -num / den
        m = int(master[k])
        for p in range(nvel):
            if cn[p] < 0:
                Rf[m][p] += L * cn[p] * phi * Mw[p]
                Rg[m][p] += L * cn[p] * phi * 0.5 * Tw * Mw[p]
            else:
                Rf[m][p] += L * cn[p] * f[k][p]
                Rg[m][p] += L * cn[p] * g[k][p]
    out_f = np.zeros_like(f)
    out_g = np.zeros_like(g)
    tau_c = math.sqrt(math.pi) / 2 * cfg.kn * cfg.lref / math.sqrt(2.0)
    for m, mem in groups.items():
        S = geo["scv"][m]
        fm, gm = f[m], g[m]
        newf = fm - dt / S * Rf[m]
        newg = gm - dt / S * Rg[m]
        if collide and imex:
            # implicit relaxation toward the equilibrium of the transported value
            rho0 = sum(fm) * w
            nu = dt / (tau_c / rho0)
            rho = sum(newf) * w
            ux = sum(vel[p][0] * newf[p] for p in range(nvel)) * w / rho
            uy = sum(vel[p][1] * newf[p] for p in range(nvel)) * w / rho
            E = sum((0.5 * (vel[p][0] ** 2 + vel[p][1] ** 2) * newf[p] + newg[p]) for p in range(nvel)) * w
            T = (2 * E / rho - ux * ux - uy * uy) / 3
            Eq = np.array([maxwellian(rho, ux, uy, T, vx, vy) for vx, vy in vel])
            Ef, Eg = shakhov_2d(cfg, vel, w, rho, ux, uy, T, newf, newg, Eq)
            newf = (newf + nu * Ef) / (1 + nu)
            newg = (newg + nu * Eg) / (1 + nu)
        elif collide:
            rho = sum(fm) * w
            ux = sum(vel[p][0] * fm[p] for p in range(nvel)) * w / rho
            uy = sum(vel[p][1] * fm[p] for p in range(nvel)) * w / rho
            E = sum((0.5 * (vel[p][0] ** 2 + vel[p][1] ** 2) * fm[p] + gm[p]) for p in range(nvel)) * w
            T = (2 * E / rho - ux * ux - uy * uy) / 3
            tau = tau_c / rho
            Eq = np.array([maxwellian(rho, ux, uy, T, vx, vy) for vx, vy in vel])
            Ef, Eg = shakhov_2d(cfg, vel, w, rho, ux, uy, T, fm, gm, Eq)
            newf = newf + dt / tau * (Ef - fm)
            newg = newg + dt / tau * (Eg - gm)
        for c in mem:
            out_f[c] = newf
            out_g[c] = newg
    return out_f, out_g


def maxwellian3(rho, u, T, v):
    c2 = (v[0] - u[0]) ** 2 + (v[1] - u[1]) ** 2 + (v[2] - u[2]) ** 2
    return rho / (2 * math.pi * T) ** 1.5 * math.exp(-c2 / (2 * T))


def shakhov_3d(cfg, vd, w, rho, u, T, F, M):
    """The Maxwellian M, or the 3D Shakhov equilibrium (Section 2.1) when
    cfg.model is "shakhov", with the heat flux of F about its mean velocity."""
    if getattr(cfg, "model", "bgk") != "shakhov":
        return M
    mu = [(vd[d] * F).sum() / F.sum() for d in range(3)]
    cd = [vd[d] - mu[d] for d in range(3)]
    h = 0.5 * (cd[0] ** 2 + cd[1] ** 2 + cd[2] ** 2) * F
    q = [(cd[d] * h).sum() * w for d in range(3)]
    c = [vd[d] - u[d] for d in range(3)]
    c2 = (c[0] ** 2 + c[1] ** 2 + c[2] ** 2) / T
    s = (1 - cfg.prandtl) * (c[0] * q[0] + c[1] * q[1] + c[2] * q[2]) / (5 * rho * T * T)
    return M * (1 + s * (c2 - 5))


def brute_step_3d(cfg, geo, v, dt, F, collide=True, imex=False):
    """Face-loop formulation of one fixed-geometry 3D step (eq. eq-schema3D):
    every Cartesian face is visited once, its upwind flux added to the control
    volume below it and subtracted from the one above; wall faces add their
    flux to their own control volume."""
    nx, ny, nz = cfg.n
    N = cfg.nv
    nvel = N ** 3
    dv = (cfg.vmax - cfg.vmin) / N
    w = dv ** 3
    rho_in, ux, uy, uz, T_in = cfg.inflow
    Tw = cfg.body.t_wall
    vel = [(v[p % N], v[(p // N) % N], v[p // (N * N)]) for p in range(nvel)]
    ghost = np.array([maxwellian3(rho_in, (ux, uy, uz), T_in, q) for q in vel])
    master = geo["master"]
    S, vbar, vcv = geo["S"], geo["vbar"], geo["vcv"]
    ncell = nx * ny * nz
    F = F.copy()
    groups = {}
    for c in range(ncell):
        if master[c] >= 0:
            groups.setdefault(int(master[c]), []).append(c)
    for m, mem in groups.items():
        if len(mem) > 1:
            fc = sum(vbar[c] * F[c] for c in mem) / vcv[m]
            for c in mem:
                F[c] = fc
    R = {m: np.zeros(nvel) for m in groups}
    n3 = (nx, ny, nz)
    stride = (1, nx, nx * ny)
    vd = [np.array([q[d] for q in vel]) for d in range(3)]

    def cell(idx):
        return idx[0] + nx * (idx[1] + ny * idx[2])

    for d in range(3):
        others = [e for e in range(3) if e != d]
        for a in range(n3[others[0]]):
            for b in range(n3[others[1]]):
                for s in range(n3[d] + 1):
                    lo = [0, 0, 0]
                    lo[others[0]] = a
                    lo[others[1]] = b
                    lo[d] = s - 1
                    hi = list(lo)
                    hi[d] = s
                    has_lo, has_hi = s - 1 >= 0, s < n3[d]
                    A = S[cell(hi), 2 * d] if has_hi else S[cell(lo), 2 * d + 1]
                    if has_lo and has_hi:
                        assert S[cell(lo), 2 * d + 1] == A
                    if A == 0.0:
                        continue
                    f_lo = F[cell(lo)] if has_lo else ghost
                    f_hi = F[cell(hi)] if has_hi else ghost
                    flux = A * (np.minimum(vd[d], 0) * f_hi + np.maximum(vd[d], 0) * f_lo)
                    if has_lo:
                        R[int(master[cell(lo)])] += flux
                    if has_hi:
                        R[int(master[cell(hi)])] -= flux
    for k in range(ncell):
        A = geo["sw"][k]
        if A <= 0.0:
            continue
        n = geo["nw"][k]
        cn = vd[0] * n[0] + vd[1] * n[1] + vd[2] * n[2]
        Mw = np.array([maxwellian3(1.0, (0, 0, 0), Tw, q) for q in vel])
        num = np.sum(np.where(cn > 0, cn * F[k], 0.0)) * w
        den = np.sum(np.where(cn < 0, cn * Mw, 0.0)) * w
        phi = -num / den
        R[int(master[k])] += A * np.where(cn < 0, cn * phi * Mw, cn * F[k])
    out = np.zeros_like(F)
    tau_c = math.sqrt(math.pi) / 2 * cfg.kn * cfg.lref / math.sqrt(2.0)
    for m, mem in groups.items():
        fm = F[m]
        new = fm - dt / vcv[m] * R[m]
        if collide and imex:
            nu = dt / (tau_c / (fm.sum() * w))
            rho = new.sum() * w
            u = [float((vd[d] * new).sum() * w / rho) for d in range(3)]
            E = float((0.5 * (vd[0] ** 2 + vd[1] ** 2 + vd[2] ** 2) * new).sum() * w)
            T = (2 * E / rho - u[0] ** 2 - u[1] ** 2 - u[2] ** 2) / 3
            Eq = shakhov_3d(cfg, vd, w, rho, u, T, new, np.array([maxwellian3(rho, u, T, q) for q in vel]))
            new = (new + nu * Eq) / (1 + nu)
        elif collide:
            rho = fm.sum() * w
            u = [float((vd[d] * fm).sum() * w / rho) for d in range(3)]
            E = float((0.5 * (vd[0] ** 2 + vd[1] ** 2 + vd[2] ** 2) * fm).sum() * w)
            T = (2 * E / rho - u[0] ** 2 - u[1] ** 2 - u[2] ** 2) / 3
            Eq = shakhov_3d(cfg, vd, w, rho, u, T, fm, np.array([maxwellian3(rho, u, T, q) for q in vel]))
            new = new + dt / (tau_c / rho) * (Eq - fm)
        for c in mem:
            out[c] = new
    return out
