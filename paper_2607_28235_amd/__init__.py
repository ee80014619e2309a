"""R3MG-C on MI355X: PCG preconditioned by one V-cycle of an R-tree agglomeration hierarchy (gfx950 HIP).

The solver lives in libr3mg.so (C ABI in include/r3mg.h); this package only marshals arguments to it and
adds the differentiable solve (autograd.py).  Nothing here falls back to a CPU implementation.
"""
from ._lib import (Assembler, Hierarchy, Options, R3mgError, lib, rtree, solve_group, EXPORTED, LIB_PATH,
                   NOALLOC_SCRATCH_BYTES)


def __getattr__(name):
    # the autograd wrapper imports torch; load it on first use only
    if name in ("AdjointPoisson", "PoissonSolve"):
        from . import autograd
        return getattr(autograd, name)
    raise AttributeError(name)


__all__ = ["Assembler", "Hierarchy", "Options", "R3mgError", "lib", "rtree", "solve_group", "EXPORTED",
           "LIB_PATH", "NOALLOC_SCRATCH_BYTES", "AdjointPoisson", "PoissonSolve"]
