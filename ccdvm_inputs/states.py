"""Seeded random distribution states for one-step parity checks.

A state is two float64 arrays f, g of shape (ncell, nvel), cell index
fastest in x, velocity index fastest in the first velocity component.
Values are strictly positive and bounded, shaped by a smooth bump over the
velocity *indices* (not velocities) so that the state looks like a
distribution peaked in the middle of the velocity box with small tails.
Solid cells are not special here: the solver defines what a solid cell
holds.
"""
from __future__ import annotations

import numpy as np


def random_state(ncell: int, nv: int, dim: int, seed: int, with_g: bool = True):
    rng = np.random.Generator(np.random.PCG64(seed))
    idx = (np.arange(nv) - (nv - 1) / 2.0) / max(nv / 4.0, 1.0)
    bump1 = np.exp(-0.5 * idx * idx)
    if dim == 2:
        bump = np.outer(bump1, bump1).reshape(-1)
    else:
        bump = np.einsum("i,j,k->ijk", bump1, bump1, bump1).reshape(-1)
    nvel = bump.size
    f = (0.5 + rng.random((ncell, nvel))) * (0.15 * bump + 1e-6)
    g = None
    if with_g:
        g = (0.5 + rng.random((ncell, nvel))) * (0.08 * bump + 1e-6)
    return f, g


def tiled_random_state(ncell: int, nv: int, dim: int, seed: int, period: int = 64):
    """Large-state variant of random_state: the random factor of cell c and
    velocity p is U[c, p % period], so a state of billions of values is built
    from ncell*period draws.  Returns one float64 array (ncell, nv**dim)."""
    rng = np.random.Generator(np.random.PCG64(seed))
    idx = (np.arange(nv) - (nv - 1) / 2.0) / max(nv / 4.0, 1.0)
    bump1 = np.exp(-0.5 * idx * idx)
    if dim == 2:
        bump = np.outer(bump1, bump1).reshape(-1)
    else:
        bump = np.einsum("i,j,k->ijk", bump1, bump1, bump1).reshape(-1)
    nvel = bump.size
    reps = -(-nvel // period)
    u = 0.5 + rng.random((ncell, period))
    out = np.empty((ncell, nvel))
    for r in range(reps):
        sl = slice(r * period, min((r + 1) * period, nvel))
        np.multiply(u[:, : sl.stop - sl.start], 0.15 * bump[sl] + 1e-6, out=out[:, sl])
    return out
