"""Named synthetic workloads.

The paper's own experiments run on a polyhedron whose geometry is only given in
a figure; these unit-cube workloads stand in for it.  Each entry is a plain
dict: mesh size n, jitter, degree k, boundary sides, and a problem factory.

  small      Kuhn n=2 (48 tets), k=1, kappa=1, c=0, tau=1, all Dirichlet,
             u = sin(pi x) sin(pi y) sin(pi z)
  smooth     Kuhn n=16 (24,576 tets), k=2, kappa = 1 + 0.5 sin(2 pi x) cos(2 pi y),
             c = 1 + |x|^2, tau=1, Dirichlet on x=0,1, Neumann elsewhere, u = sin(xyz)
  jitter_k3  Kuhn n=24 (82,944 tets), k=3, the 'smooth' data, interior vertex jitter
             up to 0.15 h (seed 0)  -- the throughput workload
  batch      256 cubes, n ~ U{4..12}, k ~ U{1..4} (PCG64(3)), kappa = exp(g) with a
             unit-variance Gaussian field of correlation length 0.2 (seed 1000+i),
             c=1, f=1, homogeneous Dirichlet, tau=1
  lognormal  Kuhn n=32 (196,608 tets), k=2, kappa = exp(1.5 g) (corr. length 0.1,
             seed 4), c=0.1, f=1, homogeneous Dirichlet, tau=1
"""
from __future__ import annotations

import numpy as np

from .fields import constant_rhs_problem, manufactured_sin_pi, manufactured_sin_xyz
from .mesh import SIDES

CONFIGS = {
    "small": dict(n=2, k=1, jitter=0.0, seed=0, dirichlet=SIDES, neumann=(),
                  problem=lambda: manufactured_sin_pi()),
    "smooth": dict(n=16, k=2, jitter=0.0, seed=0, dirichlet=("x0", "x1"),
                   neumann=("y0", "y1", "z0", "z1"), problem=lambda: manufactured_sin_xyz("c1", "c1")),
    "jitter_k3": dict(n=24, k=3, jitter=0.15, seed=0, dirichlet=("x0", "x1"),
                      neumann=("y0", "y1", "z0", "z1"), problem=lambda: manufactured_sin_xyz("c1", "c1")),
    "lognormal": dict(n=32, k=2, jitter=0.0, seed=0, dirichlet=SIDES, neumann=(),
                      problem=lambda: constant_rhs_problem(1.5, 0.1, 4, 0.1)),
}

CONFIG_ORDER = ("small", "smooth", "jitter_k3", "batch", "lognormal")


def batch_members(count: int = 256, seed: int = 3):
    """(n, k, field_seed) for each mesh of the batch workload."""
    rng = np.random.Generator(np.random.PCG64(seed))
    ns = rng.integers(4, 13, size=count)
    ks = rng.integers(1, 5, size=count)
    return [dict(n=int(ns[i]), k=int(ks[i]), jitter=0.0, seed=0, dirichlet=SIDES, neumann=(),
                 problem=(lambda i=i: constant_rhs_problem(1.0, 0.2, 1000 + i, 1.0)))
            for i in range(count)]


def config(name_or_index):
    if isinstance(name_or_index, int):
        name_or_index = CONFIG_ORDER[name_or_index]
    if name_or_index == "batch":
        return dict(name="batch", members=batch_members())
    d = dict(CONFIGS[name_or_index])
    d["name"] = name_or_index
    return d
