"""Local projections and the superconvergence diagnostics (oracle).

  trace projection   P u in M_h: <P u, v>_e = <u, v>_e for v in P_k(e), each face
                     (eq 9.12), solved with the face quadrature mass as in eq 6.3
  HDG projection     (Pi q, Pi u) in P_k(K)^3 x P_k(K), element by element (eq 9.13):
                       (Pi q, r)_K = (q, r)_K            r in P_{k-1}(K)^3
                       (Pi u, w)_K = (u, w)_K            w in P_{k-1}(K)
                       <Pi q.nu + tau Pi u, v>_{e_l} = <q.nu + tau u, v>_{e_l}
                                                         v in P_k(e_l), l = 1..4
                     assembled as the square system of Section 9 ("HDG projection"):
                     the unit mass matrix of K with its last d2 rows dropped (the
                     hierarchical basis), in each of the four unknown blocks, over the
                     face rows [n_x DP, n_y DP, n_z DP, tau DP]; dense LU per element
  diagnostics        eps_u = ||Pi u - u_h||_Omega / ||u||_Omega and
                     eps_uhat = ||P u - uhat_h||_h / ||u||_h with
                     ||v||_h^2 = sum_e |e| ||v||_e^2 (eq 10.2)

All integrals are quadrature sums in physical space; faces are integrated in their own
parametrisation (y_r = phi_e(qhat_r)), as in the rest of the oracle.
"""
from __future__ import annotations

from types import SimpleNamespace

import numpy as np

from . import basis, quadrature
from .local import Rules, face_points, geometry, local_blocks


def trace_projection(ex, fn, R: Rules, faces=None):
    """P fn on the listed faces (default all), (Nf, d2): eq 9.12 with the face rule of R."""
    if faces is None:
        faces = np.arange(ex.nfc)
    y = face_points(ex, np.asarray(faces), R)
    g = np.asarray(fn(y[..., 0], y[..., 1], y[..., 2]), dtype=np.float64) * np.ones(y.shape[:2])
    WD = R.tri_w[:, None] * R.D
    mass = WD.T @ R.D
    return np.linalg.solve(mass, WD.T @ g.T).T


def hdg_projection(ex, q_fn, u_fn, tau, R: Rules, elems=None):
    """(Pi q, Pi u) of eq 9.13 for the elements ``elems`` (default all).

    q_fn(x, y, z) -> (qx, qy, qz), u_fn(x, y, z) -> u; tau: scalar or (Nelt, 4).
    Returns Pq (Ne, 3, d3) and Pu (Ne, d3)."""
    if elems is None:
        elems = np.arange(ex.nelt)
    elems = np.asarray(elems)
    k = R.k
    d3, d2 = basis.dim3(k), basis.dim2(k)
    low = d3 - d2                                           # dim P_{k-1}(K)
    Ne = elems.size
    v, B, vol, _ = geometry(ex, elems)
    xq = v[:, None, 0, :] + np.einsum("eij,qj->eqi", B, R.vol_pts)
    W = vol[:, None] * R.vol_w[None, :]                     # |K| w_q
    P = R.P
    Mu = np.einsum("eq,qi,qj->eij", W, P, P)                # unit mass matrix of K
    qv = np.stack([np.asarray(c, dtype=np.float64) * np.ones(xq.shape[:2])
                   for c in q_fn(xq[..., 0], xq[..., 1], xq[..., 2])], axis=1)   # (Ne, 3, Nq)
    uv = np.asarray(u_fn(xq[..., 0], xq[..., 1], xq[..., 2]), dtype=np.float64) * np.ones(xq.shape[:2])
    # face blocks (the same n DP and tau DP as the local solver) and face right-hand sides;
    # local_blocks needs coefficient fields, which do not enter these blocks
    one = lambda x, y, z: 0.0 * x + 1.0
    data = SimpleNamespace(kappa=one, c=one, f=one, tau=tau)
    b = local_blocks(ex, data, R, elems)
    nDP, tauDP = b["nDP"], b["tauDP"]                       # (3, Ne, 4, d2, d3), (Ne, 4, d2, d3)
    taus = np.full((ex.nelt, 4), float(tau)) if np.isscalar(tau) else np.asarray(tau, dtype=np.float64).reshape(ex.nelt, 4)
    n = 4 * d3
    A = np.zeros((Ne, n, n))
    rhs = np.zeros((Ne, n))
    row = 0
    for blk in range(4):                                    # q_x, q_y, q_z, u: (Pi ., P_i)_K = (., P_i)_K, i < low
        A[:, row:row + low, blk * d3:(blk + 1) * d3] = Mu[:, :low, :]
        src = qv[:, blk] if blk < 3 else uv
        rhs[:, row:row + low] = np.einsum("eq,eq,qi->ei", W, src, P)[:, :low]
        row += low
    for l in range(4):
        fcs = ex.facebyele[elems, l]
        y = face_points(ex, fcs, R)
        qy = np.stack([np.asarray(c, dtype=np.float64) * np.ones(y.shape[:2])
                       for c in q_fn(y[..., 0], y[..., 1], y[..., 2])], axis=2)       # (Ne, Nq2, 3)
        uy = np.asarray(u_fn(y[..., 0], y[..., 1], y[..., 2]), dtype=np.float64) * np.ones(y.shape[:2])
        nl = ex.normals[elems, l]                           # |n_l| = |e_l|
        T = taus[elems, l] * ex.area[fcs]
        g = np.einsum("erd,ed->er", qy, nl) + T[:, None] * uy
        rows = slice(row, row + d2)
        for s in range(3):
            A[:, rows, s * d3:(s + 1) * d3] = nDP[s, :, l]
        A[:, rows, 3 * d3:] = tauDP[:, l]
        rhs[:, rows] = np.einsum("r,ri,er->ei", R.tri_w, R.D, g)
        row += d2
    assert row == n
    x = np.linalg.solve(A, rhs[:, :, None])[:, :, 0]
    return x[:, :3 * d3].reshape(Ne, 3, d3), x[:, 3 * d3:]


def superconvergence_errors(ex, u_fn, k, Pu, uh, Puhat, uhat, nq=None):
    """eps_u and eps_uhat of eq 10.2 (relative), with a rule of n = k + 4 by default."""
    nq = nq if nq is not None else k + 4
    vp, vw = quadrature.tet_rule(nq)
    tp, tw = quadrature.tri_rule(nq)
    v, B, vol, _ = geometry(ex, np.arange(ex.nelt))
    xq = v[:, None, 0, :] + np.einsum("eij,qj->eqi", B, vp)
    W = vol[:, None] * vw[None, :]
    P = basis.eval3(k, vp)
    ue = np.asarray(u_fn(xq[..., 0], xq[..., 1], xq[..., 2]), dtype=np.float64) * np.ones(xq.shape[:2])
    diff = (Pu - uh) @ P.T
    eps_u = np.sqrt((W * diff ** 2).sum() / (W * ue ** 2).sum())
    w = ex.coordinates[ex.faces]
    y = (w[:, None, 0] + tp[None, :, 0, None] * (w[:, None, 1] - w[:, None, 0])
         + tp[None, :, 1, None] * (w[:, None, 2] - w[:, None, 0]))
    uy = np.asarray(u_fn(y[..., 0], y[..., 1], y[..., 2]), dtype=np.float64) * np.ones(y.shape[:2])
    Dv = basis.eval2(k, tp)
    dy = (Puhat - uhat) @ Dv.T
    a2 = ex.area[:, None] ** 2                              # |e| * (|e| sum_r w_r ...)
    eps_uhat = np.sqrt((a2 * tw[None] * dy ** 2).sum() / (a2 * tw[None] * uy ** 2).sum())
    return {"eps_u": float(eps_u), "eps_uhat": float(eps_uhat)}
