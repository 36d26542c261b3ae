"""CPU FP64 oracle of the cut-cell DVM method -- test infrastructure only.

Only ``tests/``, ``__graft_entry__.smoke()`` and the CPU-baseline leg of
``bench.py`` may import this package.  The solver library never does.
"""
from .oracle import Oracle2D, OracleError, cfg_struct, set_threads, threads  # noqa: F401
