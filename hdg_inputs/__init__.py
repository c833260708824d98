"""Seeded synthetic inputs for the HDG hot path: meshes, coefficient fields, workloads.

This package only *generates inputs*: Kuhn-split cube meshes (optionally with
interior vertex jitter), the boundary-triangle lists, manufactured solutions and
random coefficient fields as plain functions of (x, y, z), and the named
workload configurations.  It holds none of the HDG method's arithmetic (no
quadrature, no basis, no local matrices).  Both the CPU oracle and the HIP
library's tests draw their inputs from here.
"""
from .mesh import kuhn_mesh, KuhnMesh, permute_element_vertices
from .fields import (Problem, manufactured_sin_xyz, manufactured_sin_pi, polynomial_problem, rff_field, constant_rhs_problem,
                     convection_sin_problem, convection_polynomial_problem)
from .configs import config, CONFIGS

__all__ = [
    "kuhn_mesh", "KuhnMesh", "permute_element_vertices", "Problem", "manufactured_sin_xyz", "manufactured_sin_pi",
    "polynomial_problem", "rff_field", "constant_rhs_problem", "convection_sin_problem",
    "convection_polynomial_problem", "config", "CONFIGS",
]
