"""Seeded synthetic XFEM inputs (mesh, K, f, Z, nodal blocks, element matrices) shared by
tests and bench.

Holds none of the solver's arithmetic; see ``fixtures.xfem``.
"""
from .configs import (CONFIGS, box, load, load_elements, log_normal_moduli, permuted,  # noqa: F401
                      problem_with_moduli, subdomain_order, uneven_systems, with_subdomain_blocks)
from .xfem import Problem, build_problem  # noqa: F401
