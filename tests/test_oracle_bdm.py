"""Pins of the oracle's hybridized BDM (Section 9, "BDM") against what the mixed method fixes:

* static condensation reproduces the uncondensed system (eq 1.2 with tau = 0 and eq 1.2b
  tested in P_{k-1}) exactly;
* exactness: for u in P_k(Omega) with constant kappa and c, the mixed method gives
  q_h = q, u_h = the L2 projection of u onto P_{k-1}(K) and uhat = u on every face (the
  errors are orthogonal to div V_h = P_{k-1} and to the normal traces P_k(e));
* the reduced trace system is symmetric positive definite;
* observed rates k+1 for q and k for u on n = 2, 4, 8.
"""
import math

import numpy as np
import pytest

from hdg_inputs import kuhn_mesh, manufactured_sin_xyz, permute_element_vertices, polynomial_problem
from hdg_inputs.mesh import single_tet_mesh
from oracle import basis, bdm, globalsys as G, local as L, mesh as OM

MIXED = dict(dirichlet_sides=("x0", "x1", "z0"), neumann_sides=("y0", "y1", "z1"))


def _ex(m):
    return OM.expand(m.coordinates, m.elements, m.dirichlet, m.neumann)


@pytest.mark.parametrize("k", [1, 2])
def test_bdm_condensed_equals_uncondensed(k):
    for m in (kuhn_mesh(2, jitter=0.1, seed=3, **MIXED), single_tet_mesh()):
        ex = _ex(m)
        pb = manufactured_sin_xyz("c1", "c1")
        out = bdm.solve_problem(ex, pb, k)
        q, u, uh = bdm.brute_solve(ex, pb, k)
        for a, b_ in ((out["q"], q), (out["u"], u), (out["uhat"], uh)):
            assert np.abs(a - b_).max() <= 1e-11 * np.abs(b_).max()


@pytest.mark.parametrize("k", [1, 2, 3])
def test_bdm_polynomial_exactness(k):
    ex = _ex(permute_element_vertices(kuhn_mesh(2, jitter=0.15, seed=7, **MIXED), seed=7))
    pb = polynomial_problem(k, seed=k, kappa=1.7, c=0.6)
    out = bdm.solve_problem(ex, pb, k)
    err = G.errors(ex, pb, k, out["q"], out["u"], out["uhat"])
    assert err["e_q"] < 1e-11 and err["e_uhat"] < 1e-11, err
    # u_h is the L2 projection of u onto P_{k-1}(K): (u - u_h, P_i)_K = 0 for i < d3 - d2
    R = L.rules(k)
    low = basis.dim3(k) - basis.dim2(k)
    v, B, vol, _ = L.geometry(ex, np.arange(ex.nelt))
    xq = v[:, None, 0, :] + np.einsum("eij,qj->eqi", B, R.vol_pts)
    ue = pb.u(xq[..., 0], xq[..., 1], xq[..., 2]) * np.ones(xq.shape[:2])
    mom = np.einsum("q,eq,qi->ei", R.vol_w, ue - out["u"] @ R.P.T, R.P[:, :low])
    assert np.abs(mom).max() < 1e-11 * np.abs(ue).max()
    assert not out["u"][:, low:].any()


@pytest.mark.parametrize("k", [1, 2])
def test_bdm_trace_system_spd(k):
    ex = _ex(kuhn_mesh(2, **MIXED))
    pb = manufactured_sin_xyz("c1", "c1")
    C, _ = bdm.condense(ex, pb, k)
    assert np.abs(C - C.transpose(0, 2, 1)).max() <= 1e-13 * np.abs(C).max()
    H, _ = G.assemble(ex, k, C, np.zeros(C.shape[:2]))
    d2 = basis.dim2(k)
    free = np.ones(ex.nfc, dtype=bool)
    free[ex.dirfaces] = False
    I = np.nonzero(np.repeat(free, d2))[0]
    HII = H.toarray()[np.ix_(I, I)]
    np.linalg.cholesky(0.5 * (HII + HII.T))


@pytest.mark.parametrize("k", [1, 2])
def test_bdm_rates(k):
    """Mixed-method orders for BDM_k: k+1 for q (and uhat), k for u in P_{k-1}."""
    pb = manufactured_sin_xyz("c1", "c1")
    errs = []
    for n in (2, 4, 8):
        ex = _ex(kuhn_mesh(n, dirichlet_sides=("x0", "x1"), neumann_sides=("y0", "y1", "z0", "z1")))
        out = bdm.solve_problem(ex, pb, k)
        errs.append(G.errors(ex, pb, k, out["q"], out["u"], out["uhat"]))
    rate = {a: math.log2(errs[1][a] / errs[2][a]) for a in errs[0]}
    assert rate["e_q"] >= k + 1 - 0.3, rate
    assert rate["e_u"] >= k - 0.25, rate
    assert rate["e_u"] < k + 0.5, rate  # no better: u_h lives in P_{k-1}
