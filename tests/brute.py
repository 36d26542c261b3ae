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


def brute_step(cfg, geo, v, dt, f, g, collide=True):
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
        if collide:
            rho = sum(fm) * w
            ux = sum(vel[p][0] * fm[p] for p in range(nvel)) * w / rho
            uy = sum(vel[p][1] * fm[p] for p in range(nvel)) * w / rho
            E = sum((0.5 * (vel[p][0] ** 2 + vel[p][1] ** 2) * fm[p] + gm[p]) for p in range(nvel)) * w
            T = (2 * E / rho - ux * ux - uy * uy) / 3
            tau = tau_c / rho
            Eq = np.array([maxwellian(rho, ux, uy, T, vx, vy) for vx, vy in vel])
            newf = newf + dt / tau * (Eq - fm)
            newg = newg + dt / tau * (0.5 * T * Eq - gm)
        for c in mem:
            out_f[c] = newf
            out_g[c] = newg
    return out_f, out_g
