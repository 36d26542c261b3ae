"""ccdvm: Cartesian cut-cell discrete-velocity solver (MI355X, HIP).

The solver library is ``libccdvm.so`` (C-ABI in ``include/ccdvm.h``);
:class:`Solver` wraps it.  Importing this package does not load the library;
creating a Solver does, and fails loudly when it has not been built.
"""
from ._capi import CCError, LIB_PATH, lib  # noqa: F401


def __getattr__(name):
    if name == "Solver":
        from .solver import Solver
        return Solver
    raise AttributeError(name)
