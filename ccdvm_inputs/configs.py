"""Workload descriptions (nondimensional units: R = T0 = rho0 = 1, L_ref = 1).

Every workload here is synthetic and deterministic: the paper's
experiments are simulations whose comparison data is not available, so
the inputs are the flow set-ups themselves (domain, grid, velocity box,
obstacle, Knudsen number, inflow Mach number, wall temperature).

Readings of the paper that fix these recipes:
  * inflow speed from the Mach number with gamma = 5/3 (monatomic gas,
    three translational degrees of freedom kept by the reduced model);
  * farfield outer boundary carrying the inflow Maxwellian;
  * initial state = the inflow Maxwellian in every gas cell.
"""
from __future__ import annotations

import math
from dataclasses import dataclass, field, replace
from typing import Tuple

import numpy as np

GAMMA = 5.0 / 3.0

BODY_KINDS = ("none", "circle", "ellipse", "cavity", "halfplane", "sphere", "vane")
MOTIONS = ("fixed", "free_rotation", "imposed")


def mach_to_speed(mach: float, temperature: float = 1.0) -> float:
    """Inflow speed u = Ma * sqrt(gamma R T) with gamma = 5/3 and R = 1."""
    return mach * math.sqrt(GAMMA * temperature)


@dataclass(frozen=True)
class Body:
    """Obstacle described by an analytic signed distance (gas side positive).

    kind      'none' | 'circle' (axes[0] = radius) | 'ellipse' (semi-axes
              axes[0], axes[1], rotated by theta) | 'cavity' (gas inside a
              circle of radius axes[0]) | 'halfplane' (gas on the side of the
              unit normal (cos theta, sin theta) through center) | 'sphere'
              (3D, axes[0] = radius) | 'vane' (3D plate with rounded edges:
              the points within min(axes) of the box of half-sizes
              axes - min(axes), turned by theta about the z axis)
    motion    'fixed' | 'free_rotation' (rotation about center driven by the
              gas torque, translation off; in 3D about the z axis) |
              'imposed' (constant vel/omega)
    """
    kind: str = "none"
    center: Tuple[float, float, float] = (0.5, 0.5, 0.5)
    axes: Tuple[float, float, float] = (0.2, 0.2, 0.2)
    theta: float = 0.0
    t_wall: float = 1.0
    mass: float = 1.0
    inertia: float = 1.0
    motion: str = "fixed"
    vel: Tuple[float, float, float] = (0.0, 0.0, 0.0)
    omega: float = 0.0


@dataclass(frozen=True)
class Config:
    dim: int
    n: Tuple[int, int, int]
    lo: Tuple[float, float, float]
    hi: Tuple[float, float, float]
    nv: int
    vmin: float = -6.0
    vmax: float = 6.0
    kn: float = 0.1            # <= 0 selects the collisionless (pure transport) limit
    lref: float = 1.0
    cfl: float = 0.5
    dt: float = 0.0            # <= 0 : derived from cfl
    inflow: Tuple[float, float, float, float, float] = (1.0, 0.0, 0.0, 0.0, 1.0)
    body: Body = field(default_factory=Body)
    steps: int = 1
    name: str = ""
    maxwellian: str = "direct"  # "direct" moments or "conservative" (Newton) equilibrium
    scheme: str = "explicit"    # "explicit" or "imex" (semi-implicit relaxation)
    model: str = "bgk"          # relaxation model: "bgk" or "shakhov"
    prandtl: float = 2.0 / 3.0  # Prandtl number of the Shakhov model
    amr_depth: int = 0          # 3D octree: finest depth below the coarse grid n (0: uniform)
    amr_band: float = 0.0       # octree refinement band in coarse spacings (<= 0: 2 sqrt 2)
    cfl_strict: int = 0         # 1: binding fails when the positivity number exceeds 1

    @property
    def ncell(self) -> int:
        return self.n[0] * self.n[1] * self.n[2]

    @property
    def nvel(self) -> int:
        return self.nv ** self.dim

    def with_(self, **kw) -> "Config":
        return replace(self, **kw)


def _inflow(mach: float, t: float = 1.0):
    return (1.0, mach_to_speed(mach, t), 0.0, 0.0, t)


def small_2d(nx=32, ny=32, nv=16, kn=0.1, mach=0.5, body=None, steps=50,
             lo=(0.0, 0.0, 0.0), hi=(1.0, 1.0, 1.0), **kw) -> Config:
    if body is None:
        body = Body("circle", (0.5, 0.5, 0.0), (0.2, 0.2, 0.0))
    return Config(dim=2, n=(nx, ny, 1), lo=lo, hi=hi, nv=nv, kn=kn,
                  inflow=_inflow(mach), body=body, steps=steps, **kw)


def small_3d(nx=16, ny=8, nz=8, nv=8, kn=0.1, mach=0.5, body=None, steps=5,
             lo=(0.0, 0.0, 0.0), hi=(1.0, 0.5, 0.5), **kw) -> Config:
    if body is None:
        body = Body("sphere", (0.5, 0.25, 0.25), (0.15, 0.15, 0.15))
    return Config(dim=3, n=(nx, ny, nz), lo=lo, hi=hi, nv=nv, kn=kn,
                  inflow=_inflow(mach), body=body, steps=steps, **kw)


def workload(name: str, kn: float | None = None) -> Config:
    """The five headline workloads, by name ('cyl32', 'cyl512', 'ellipse256',
    'sphere128', and the batch through :func:`batch_instances`)."""
    if name == "cyl32":        # 2D 32x32, circle r=0.2, 16^2 velocities
        return small_2d(32, 32, 16, kn=0.1 if kn is None else kn, mach=0.5,
                        steps=50, name=name)
    if name == "cyl512":       # 2D 512x256 on [0,1]x[0,0.5], circle r=0.05
        return Config(dim=2, n=(512, 256, 1), lo=(0.0, 0.0, 0.0),
                      hi=(1.0, 0.5, 1.0), nv=32, kn=0.1 if kn is None else kn,
                      inflow=_inflow(0.8),
                      body=Body("circle", (0.5, 0.25, 0.0), (0.05, 0.05, 0.0)),
                      steps=2000, name=name)
    if name == "ellipse256":   # 2D moving ellipse, free rotation
        return Config(dim=2, n=(256, 256, 1), lo=(0.0, 0.0, 0.0),
                      hi=(1.0, 1.0, 1.0), nv=40, kn=0.05 if kn is None else kn,
                      inflow=_inflow(0.5),
                      body=Body("ellipse", (0.5, 0.5, 0.0), (0.1, 0.02, 0.0),
                                theta=math.pi / 8, mass=1.0, inertia=0.01,
                                motion="free_rotation"),
                      steps=5000, name=name)
    if name == "sphere128":    # 3D 128x64x64, sphere r=0.1, 16^3 velocities
        return Config(dim=3, n=(128, 64, 64), lo=(0.0, 0.0, 0.0),
                      hi=(1.0, 0.5, 0.5), nv=16, kn=0.1 if kn is None else kn,
                      inflow=_inflow(0.5),
                      body=Body("sphere", (0.5, 0.25, 0.25), (0.1, 0.1, 0.1)),
                      steps=500, name=name)
    if name == "sphere_amr":   # 3D octree: 32x16x16 coarse, depth 2 (1/128 near the sphere), 16^3 velocities
        return Config(dim=3, n=(32, 16, 16), lo=(0.0, 0.0, 0.0),
                      hi=(1.0, 0.5, 0.5), nv=16, kn=0.1 if kn is None else kn,
                      inflow=_inflow(0.5),
                      body=Body("sphere", (0.5, 0.25, 0.25), (0.1, 0.1, 0.1)),
                      steps=500, name=name, amr_depth=2)
    if name == "vane_amr":     # 3D octree, turning vane: 32x32x16 coarse, depth 2, 16^3 velocities
        return Config(dim=3, n=(32, 32, 16), lo=(0.0, 0.0, 0.0),
                      hi=(1.0, 1.0, 0.5), nv=16, kn=0.1 if kn is None else kn,
                      inflow=_inflow(0.5),
                      body=Body("vane", (0.5, 0.5, 0.25), (0.2, 0.03, 0.12),
                                theta=math.pi / 8, inertia=0.002, motion="free_rotation",
                                omega=2.0),
                      steps=500, name=name, amr_depth=2)
    raise KeyError(name)


WORKLOADS = ("cyl32", "cyl512", "ellipse256", "sphere128", "sphere_amr", "vane_amr")

BATCH_SEED = 20150316


def batch_instances(count: int = 64, seed: int = BATCH_SEED, steps: int = 200):
    """Heterogeneous 2D fixed-cylinder instances drawn with numpy PCG64.

    Per instance, in this order: grid n in {64,128,256}, velocity grid N in
    {16,24,32}, Kn = 10**U(-2,0), T_w ~ U(0.5,2), Ma ~ U(0.3,1).
    """
    rng = np.random.Generator(np.random.PCG64(seed))
    out = []
    for k in range(count):
        n = int(rng.choice([64, 128, 256]))
        nv = int(rng.choice([16, 24, 32]))
        kn = float(10.0 ** rng.uniform(-2.0, 0.0))
        tw = float(rng.uniform(0.5, 2.0))
        ma = float(rng.uniform(0.3, 1.0))
        out.append(Config(dim=2, n=(n, n, 1), lo=(0.0, 0.0, 0.0),
                          hi=(1.0, 1.0, 1.0), nv=nv, kn=kn,
                          inflow=_inflow(ma),
                          body=Body("circle", (0.5, 0.5, 0.0), (0.2, 0.2, 0.0),
                                    t_wall=tw),
                          steps=steps, name=f"batch{k}"))
    return out
