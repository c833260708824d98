"""Pins of the oracle's convection-diffusion HDG (Section 9, "Matrices for convection-diffusion
problems", eq 9.1; the conservative method stated in oracle/convection.py):

* with beta = 0 the element matrices are the diffusion HDG ones (Section 5);
* consistency: a polynomial u of degree <= k with constant kappa and c and an affine beta is
  reproduced exactly (u_h = u, q_h = q, uhat = u on the faces), with mixed boundary
  conditions on a mesh with every face orientation;
* static condensation reproduces the uncondensed system exactly;
* observed rates k+1 for q, u and uhat on n = 2, 4, 8.
"""
import math

import numpy as np
import pytest

from hdg_inputs import kuhn_mesh, permute_element_vertices
from hdg_inputs.fields import convection_polynomial_problem, convection_sin_problem
from hdg_inputs.mesh import single_tet_mesh
from oracle import convection as CV, globalsys as G, local as L, mesh as OM

MIXED = dict(dirichlet_sides=("x0", "x1", "z0"), neumann_sides=("y0", "y1", "z1"))


def _ex(m):
    return OM.expand(m.coordinates, m.elements, m.dirichlet, m.neumann)


@pytest.mark.parametrize("k", [1, 2])
def test_zero_convection_is_diffusion_hdg(k):
    ex = _ex(kuhn_mesh(2, jitter=0.1, seed=1, **MIXED))
    pb = convection_sin_problem(beta_scale=0.0, tau=1.3)
    C, Cf = CV.condense(ex, pb, k)
    C0, Cf0 = L.condense(L.local_blocks(ex, pb, L.rules(k)))
    assert np.abs(C - C0).max() <= 1e-13 * np.abs(C0).max()
    assert np.abs(Cf - Cf0).max() <= 1e-13 * np.abs(Cf0).max()


@pytest.mark.parametrize("k", [0, 1, 2, 3])
def test_polynomial_reproduction(k):
    ex = _ex(permute_element_vertices(kuhn_mesh(2, jitter=0.15, seed=4, **MIXED), seed=4))
    pb = convection_polynomial_problem(k, seed=10 + k)
    out = CV.solve_problem(ex, pb, k)
    err = G.errors(ex, pb, k, out["q"], out["u"], out["uhat"])
    assert err["e_u"] < 1e-10 and err["e_uhat"] < 1e-10, err
    if k:
        assert err["e_q"] < 1e-10, err


@pytest.mark.parametrize("k", [1, 2])
def test_condensed_equals_uncondensed(k):
    for m in (kuhn_mesh(2, jitter=0.1, seed=2, **MIXED), single_tet_mesh()):
        ex = _ex(m)
        pb = convection_sin_problem(beta_scale=2.0)
        out = CV.solve_problem(ex, pb, k)
        q, u, uh = CV.brute_solve(ex, pb, k)
        for a, b_ in ((out["q"], q), (out["u"], u), (out["uhat"], uh)):
            assert np.abs(a - b_).max() <= 1e-11 * np.abs(b_).max()


@pytest.mark.parametrize("k", [1, 2])
def test_rates(k):
    pb = convection_sin_problem(beta_scale=1.0)
    errs = []
    for n in (2, 4, 8):
        ex = _ex(kuhn_mesh(n, dirichlet_sides=("x0", "x1"), neumann_sides=("y0", "y1", "z0", "z1")))
        out = CV.solve_problem(ex, pb, k)
        errs.append(G.errors(ex, pb, k, out["q"], out["u"], out["uhat"]))
    rate = {a: math.log2(errs[1][a] / errs[2][a]) for a in errs[0]}
    for a in ("e_q", "e_u", "e_uhat"):
        assert rate[a] >= k + 1 - 0.3, rate
