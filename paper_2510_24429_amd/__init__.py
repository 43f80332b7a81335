"""MI355X-native restarted, diagonally preconditioned PDHG for standard-form LP.

The compute path lives in the HIP shared library ``libpdhg.so`` (C ABI declared
in ``include/pdhg.h``); ``_lib`` marshals arguments to it and ``solver`` /
``autograd`` wrap it.  Importing the package does not load the library, so the
input generators in ``lpgen`` stay usable on machines without a GPU.
"""
__all__ = ["lpgen"]


def __getattr__(name):
    if name in ("Solver", "SolveResult"):
        from . import solver
        return getattr(solver, name)
    if name in ("PDHGUnroll",):
        from . import autograd
        return getattr(autograd, name)
    raise AttributeError(name)
