"""Hybridized BDM (Section 9, "BDM"; oracle).

W_h = P_{k-1}(K) per element, V_h = P_k(K)^3, M_h unchanged, k >= 1.  The method is eq 1.2
with tau = 0 and the scalar equation eq 1.2b tested in P_{k-1}(K) only.  The paper's recipe
(read as this: it drops the degree-k modes of u and of its test space, which is what makes
the local system square) is to delete
  the last d2 rows and columns of A1, the last d2 rows of A2 and Af, the last d2 columns of A3
from the HDG local matrices of Section 5 (hierarchical basis: the last d2 modes of P_k(K) are
the degree-k ones).  Everything downstream (condensation eq 5.5-5.6 without tau DD, assembly
eq 6.5, boundary data, reconstruction) is the HDG code.  The uncondensed system is assembled
as in ``brute`` with the same deletions, to pin the condensation.
"""
from __future__ import annotations

from types import SimpleNamespace

import numpy as np
import scipy.sparse as sp
import scipy.sparse.linalg as spla

from . import basis
from .globalsys import assemble, dirichlet_data, neumann_load, rhs_with_neumann, solve_trace
from .local import local_blocks, local_solver_matrices, rules


def _zero_tau(problem):
    return SimpleNamespace(kappa=problem.kappa, c=problem.c, f=problem.f, tau=0.0)


def bdm_matrices(ex, problem, R, elems=None):
    """A1, A2, Af, A3 of the hybridized BDM element (the HDG ones with tau = 0 and the last
    d2 rows / columns deleted as listed above)."""
    k = R.k
    d3, d2 = basis.dim3(k), basis.dim2(k)
    b = local_blocks(ex, _zero_tau(problem), R, elems)
    A1, A2, Af, A3 = local_solver_matrices(b)
    n = 4 * d3 - d2
    return A1[:, :n, :n], A2[:, :n, :], Af[:, :n], A3[:, :, :n]


def condense(ex, problem, k, nq=None):
    """C^K = A3 A1^{-1} A2 and Cf^K = A3 A1^{-1} Af (eq 5.5-5.6; tau DD = 0)."""
    R = rules(k, nq)
    A1, A2, Af, A3 = bdm_matrices(ex, problem, R)
    X = np.linalg.solve(A1, np.concatenate([A2, Af[:, :, None]], axis=2))
    return np.einsum("eij,ejk->eik", A3, X[:, :, :-1]), np.einsum("eij,ej->ei", A3, X[:, :, -1])


def solve_problem(ex, problem, k, nq=None):
    """The hybridized BDM pipeline; u is returned in P_k(K) coefficients with the degree-k
    modes zero, so that it can be compared with the HDG layout."""
    R = rules(k, nq)
    d3, d2 = basis.dim3(k), basis.dim2(k)
    A1, A2, Af, A3 = bdm_matrices(ex, problem, R)
    X = np.linalg.solve(A1, np.concatenate([A2, Af[:, :, None]], axis=2))
    C = np.einsum("eij,ejk->eik", A3, X[:, :, :-1])
    Cf = np.einsum("eij,ej->ei", A3, X[:, :, -1])
    H, F = assemble(ex, k, C, Cf)
    uD = dirichlet_data(ex, problem, R)
    GN = neumann_load(ex, problem, R)
    b = rhs_with_neumann(ex, k, F, GN)
    uhat = solve_trace(ex, k, H, b, uD)
    uK = uhat[ex.facebyele].reshape(ex.nelt, -1)
    x = np.linalg.solve(A1, (Af - np.einsum("eij,ej->ei", A2, uK))[:, :, None])[:, :, 0]
    q = x[:, :3 * d3].reshape(-1, 3, d3)
    u = np.zeros((ex.nelt, d3))
    u[:, :d3 - d2] = x[:, 3 * d3:]
    return dict(C=C, Cf=Cf, H=H, F=F, b=b, uD=uD, uhat=uhat, q=q, u=u)


def brute_solve(ex, problem, k, nq=None):
    """eq 1.2 for hybridized BDM without condensation: the element equations with the
    deleted rows / columns, flux continuity on interior faces, Neumann and Dirichlet rows."""
    R = rules(k, nq)
    d3, d2 = basis.dim3(k), basis.dim2(k)
    A1, A2, Af, A3 = bdm_matrices(ex, problem, R)
    nv = 4 * d3 - d2
    Nelt, Nfc = ex.nelt, ex.nfc
    off = nv * Nelt
    N = off + d2 * Nfc
    rows, cols, vals = [], [], []
    rhs = np.zeros(N)

    def add(r, c, M):
        rr, cc = np.meshgrid(r, c, indexing="ij")
        rows.append(rr.ravel())
        cols.append(cc.ravel())
        vals.append(np.asarray(M).ravel())

    isD = np.zeros(Nfc, dtype=bool)
    isD[ex.dirfaces] = True
    for K in range(Nelt):
        vK = np.arange(nv) + nv * K
        tK = (off + ex.facebyele[K][:, None] * d2 + np.arange(d2)[None, :]).ravel()
        add(vK, vK, A1[K])
        add(vK, tK, A2[K])
        rhs[vK] = Af[K]
        keep = ~np.repeat(isD[ex.facebyele[K]], d2)
        add(tK[keep], vK, A3[K][keep])
    GN = neumann_load(ex, problem, R)
    for r, f in enumerate(ex.neufaces):
        rhs[off + f * d2: off + (f + 1) * d2] = -GN[r]
    uD = dirichlet_data(ex, problem, R)
    for r, f in enumerate(ex.dirfaces):
        idx = off + f * d2 + np.arange(d2)
        add(idx, idx, np.eye(d2))
        rhs[idx] = uD[r]
    A = sp.coo_matrix((np.concatenate(vals), (np.concatenate(rows), np.concatenate(cols))), shape=(N, N)).tocsc()
    x = spla.splu(A).solve(rhs)
    qu = x[:off].reshape(Nelt, nv)
    q = qu[:, :3 * d3].reshape(Nelt, 3, d3)
    u = np.zeros((Nelt, d3))
    u[:, :d3 - d2] = qu[:, 3 * d3:]
    return q, u, x[off:].reshape(Nfc, d2)
