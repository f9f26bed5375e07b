"""MI355X-native deflated block-Jacobi conjugate gradient for XFEM/GFEM crack systems.

CG preconditioned by the adapted-deflation operator A-DEF2 with a block-Jacobi
smoother over nodal blocks (Agathos, Dodwell, Chatzi, Bordas), implemented as HIP
kernels for gfx950 behind the C ABI of ``include/dpcg.h``.  This package is the
binding: ``Solver`` marshals device tensors to the library, which does all of the
arithmetic.
"""
from ._binding import (DpcgError, Elements, Info, Options, Solver, Stats, lib,  # noqa: F401
                       solve_many, status_string)
from . import _binding as abi  # noqa: F401

__all__ = ["Solver", "Elements", "DpcgError", "lib", "status_string", "abi", "solve", "solve_many"]


def solve(f, solver, scale=None, elements=None, tol=1e-8, **opts):
    """Differentiable u = K^{-1} f (see paper_2111_09294_amd.autograd.solve)."""
    from .autograd import solve as _solve
    return _solve(f, solver, scale=scale, elements=elements, tol=tol, **opts)
