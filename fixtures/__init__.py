"""Seeded synthetic XFEM inputs (mesh, K, f, Z, nodal blocks, element matrices) shared by
tests and bench.

Holds none of the solver's arithmetic; see ``fixtures.xfem``.
"""
from .configs import (CONFIGS, box, load, load_elements, log_normal_moduli, problem_with_moduli,  # noqa: F401
                      uneven_systems)
from .xfem import Problem, build_problem  # noqa: F401
