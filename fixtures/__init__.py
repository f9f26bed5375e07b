"""Seeded synthetic XFEM inputs (mesh, K, f, Z, nodal blocks) shared by tests and bench.

Holds none of the solver's arithmetic; see ``fixtures.xfem``.
"""
from .configs import CONFIGS, load  # noqa: F401
from .xfem import Problem, build_problem  # noqa: F401
