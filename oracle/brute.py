"""The uncondensed HDG system, eq 1.2a-e, solved directly (oracle, tiny meshes).

Unknowns: (q_K, u_K) for every element (4 d3 each) and uhat_e for every face
(d2 each).  Equations:
  eq 1.2a-b on each K:       A1 [q; u]_K + A2 u_dK = Af                      (eq 5.1-5.3)
  eq 1.2c on interior faces: sum over the two elements of the face rows of
                              A3 [q; u]_K - tauDD u_dK  =  0
  eq 1.2e on Neumann faces:  -(A3 [q; u]_K - tauDD u_dK)_face = Phi_N      (eq 6.4)
  eq 1.2d on Dirichlet faces: <uhat, v> = <u_D, v> on the face            (eq 6.1)
Static condensation must reproduce this solution exactly (up to rounding).
"""
from __future__ import annotations

import numpy as np
import scipy.sparse as sp
import scipy.sparse.linalg as spla

from . import basis
from .globalsys import dirichlet_data, neumann_load
from .local import local_blocks, local_solver_matrices, rules


def brute_solve(ex, problem, k, nq=None):
    R = rules(k, nq)
    d3, d2 = basis.dim3(k), basis.dim2(k)
    nv = 4 * d3
    b = local_blocks(ex, problem, R)
    A1, A2, Af, A3 = local_solver_matrices(b)
    tauDD = b["tauDD"]
    Nelt, Nfc = ex.nelt, ex.nfc
    N = nv * Nelt + d2 * Nfc
    off = nv * Nelt
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
        # flux rows on the element's faces (Dirichlet faces get their own equation)
        keep = ~np.repeat(isD[ex.facebyele[K]], d2)
        add(tK[keep], vK, A3[K][keep])
        add(tK[keep], tK, -tauDD[K][keep])
    # Neumann: -(flux) = Phi_N  <=>  flux = -Phi_N
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
    u = qu[:, 3 * d3:]
    uhat = x[off:].reshape(Nfc, d2)
    return q, u, uhat
