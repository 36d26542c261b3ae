"""Seeded synthetic inputs shared by the oracle side and the HIP side.

This module only describes workloads (grid, velocity box, body, gas
parameters) and draws seeded random numbers.  It holds none of the
method's arithmetic: no velocity grid, no Maxwellian, no geometry, no
flux.  Both implementations turn a :class:`Config` into their own
structures.
"""
from .configs import (Body, Config, mach_to_speed, workload, WORKLOADS,
                      small_2d, small_3d, batch_instances)
from .states import random_state, tiled_random_state

__all__ = ["Body", "Config", "mach_to_speed", "workload", "WORKLOADS",
           "small_2d", "small_3d", "batch_instances", "random_state",
           "tiled_random_state"]
