"""Global hybrid system, boundary data, solve, reconstruction, postprocess, errors (oracle).

  assembly       H[dof(K)_i, dof(K)_j] += C^K_ij,  F[dof(K)_i] += Cf^K_i with
                 list(e) = e d2 + [0, d2) (Section 6, "Assembly process", eq 6.5),
                 by scipy's COO->CSR duplicate summation
  Dirichlet      uD_e = ((v.D)^T D)^{-1} (v.D)^T u_D(phi_e(qhat))  (eq 6.1-6.3; eq 6.1's
                 D_j(q_j) read as D_j(q_r))
  Neumann        Phi_N,e = sum_s n_{e,s} (v.D)^T g_s(phi_e(qhat))  (eq 6.4), with n_e the
                 listed (outward) triangle's normal, |n_e| = |e|
  elimination    H_II u_I = F_I + G_I - H_ID uD  (Section 6, last paragraph)
  solve          the paper does not name a solver: sparse LU (small) or CG with a
                 block-Jacobi preconditioner to a tight tolerance (large)
  reconstruction A1 [q; u] = Af - A2 u_dK   (Section 6 "Reconstruction")
  postprocess    (grad u*, grad w)_K = -(kappa^{-1} q_h, grad w)_K for w in P_{k+1},
                 (u*, 1)_K = (u_h, 1)_K  (eq 9.11).  With the orthonormal hierarchical
                 basis (Phat_1 = 1, the rest of zero mean) the mean condition fixes the
                 first coefficient: u*_1 = u_1, and the stiffness system is solved on
                 the remaining modes.
  errors         relative L2 errors of eq 10.1-10.2 with ||v||_h^2 = sum_e |e| ||v||_e^2
"""
from __future__ import annotations

import numpy as np
import scipy.sparse as sp
import scipy.sparse.linalg as spla

from . import basis, quadrature
from .local import Rules, face_points, geometry, local_blocks, recover


def assemble(ex, k, C, Cf):
    """H (CSR, d2 Nfc square) and F (d2 Nfc) from the element blocks (eq 6.5)."""
    d2 = basis.dim2(k)
    dof = (ex.facebyele[:, :, None] * d2 + np.arange(d2)[None, None, :]).reshape(ex.nelt, -1)
    rows = np.repeat(dof[:, :, None], dof.shape[1], axis=2)
    cols = np.repeat(dof[:, None, :], dof.shape[1], axis=1)
    N = d2 * ex.nfc
    H = sp.coo_matrix((C.ravel(), (rows.ravel(), cols.ravel())), shape=(N, N)).tocsr()
    F = np.zeros(N)
    np.add.at(F, dof.ravel(), Cf.ravel())
    return H, F


def dirichlet_data(ex, problem, R: Rules):
    """uD on Dirichlet faces, (Ndir, d2), rows in Dirichlet-list order (eq 6.3)."""
    fcs = ex.dirfaces
    if fcs.size == 0:
        return np.zeros((0, R.D.shape[1]))
    y = face_points(ex, fcs, R)
    g = np.asarray(problem.uD(y[..., 0], y[..., 1], y[..., 2]), dtype=np.float64) * np.ones(y.shape[:2])
    WD = R.tri_w[:, None] * R.D
    mass = WD.T @ R.D
    return np.linalg.solve(mass, (WD.T @ g.T)).T


def neumann_load(ex, problem, R: Rules):
    """Phi_N on Neumann faces, (Nneu, d2), rows in Neumann-list order (eq 6.4)."""
    fcs = ex.neufaces
    if fcs.size == 0:
        return np.zeros((0, R.D.shape[1]))
    y = face_points(ex, fcs, R)
    gx, gy, gz = problem.gN(y[..., 0], y[..., 1], y[..., 2])
    w = ex.coordinates[ex.faces[fcs]]
    n = 0.5 * np.cross(w[:, 1] - w[:, 0], w[:, 2] - w[:, 0])   # (Nneu, 3), |n| = |e|
    gn = n[:, 0:1] * gx + n[:, 1:2] * gy + n[:, 2:3] * gz      # g_N(y_r) . n_e
    return (R.tri_w[None, :, None] * R.D[None] * gn[:, :, None]).sum(axis=1)


def rhs_with_neumann(ex, k, F, GN):
    d2 = basis.dim2(k)
    b = F.copy().reshape(ex.nfc, d2)
    b[ex.neufaces] += GN
    return b.ravel()


def solve_trace(ex, k, H, b, uD, direct_limit=60000, rtol=1e-13):
    """Eliminate Dirichlet faces and solve H_II u_I = b_I - H_ID uD.  Returns (Nfc, d2)."""
    d2 = basis.dim2(k)
    u = np.zeros((ex.nfc, d2))
    u[ex.dirfaces] = uD
    isD = np.zeros(ex.nfc, dtype=bool)
    isD[ex.dirfaces] = True
    Dd = np.repeat(isD, d2)
    I = np.nonzero(~Dd)[0]
    Didx = np.nonzero(Dd)[0]
    HII = H[I][:, I].tocsc()
    rhs = b[I] - H[I][:, Didx] @ u.ravel()[Didx]
    if I.size <= direct_limit:
        xI = spla.splu(HII).solve(rhs)
    else:
        xI = _bj_cg(HII.tocsr(), rhs, d2, rtol)
    u.ravel()[I] = xI
    return u


def _bj_cg(A, b, bs, rtol):
    n = A.shape[0]
    nb = n // bs
    Ad = A.toarray() if n < 2000 else None
    blocks = np.zeros((nb, bs, bs))
    Acoo = A.tocoo()
    same = (Acoo.row // bs) == (Acoo.col // bs)
    r, c, v = Acoo.row[same], Acoo.col[same], Acoo.data[same]
    np.add.at(blocks, (r // bs, r % bs, c % bs), v)
    inv = np.linalg.inv(blocks)
    M = spla.LinearOperator((n, n), matvec=lambda x: np.einsum("bij,bj->bi", inv, x.reshape(nb, bs)).ravel())
    del Ad
    x, info = spla.cg(A, b, rtol=rtol, atol=0.0, M=M, maxiter=20000)
    if info != 0:
        raise RuntimeError(f"oracle CG did not converge (info={info})")
    return x


def trace_by_element(ex, uhat):
    """u_dK (Nelt, 4 d2): the trace coefficients in facebyele order (Section 5)."""
    return uhat[ex.facebyele].reshape(ex.nelt, -1)


def recover_all(ex, problem, R: Rules, uhat, chunk=4096):
    qs, us = [], []
    uK = trace_by_element(ex, uhat)
    for s in range(0, ex.nelt, chunk):
        el = np.arange(s, min(s + chunk, ex.nelt))
        b = local_blocks(ex, problem, R, el)
        q, u = recover(b, uK[el])
        qs.append(q)
        us.append(u)
    return np.concatenate(qs), np.concatenate(us)


def postprocess(ex, problem, R: Rules, q, u, elems=None):
    """u* in P_{k+1} (eq 9.11) with the volume rule of R: (Ne, d3(k+1))."""
    if elems is None:
        elems = np.arange(ex.nelt)
    k = R.k
    v, B, vol, BinvT = geometry(ex, elems)
    xq = v[:, None, 0, :] + np.einsum("eij,qj->eqi", B, R.vol_pts)
    kinv = 1.0 / np.asarray(problem.kappa(xq[..., 0], xq[..., 1], xq[..., 2]), dtype=np.float64)
    W = vol[:, None] * R.vol_w[None, :]
    G1 = basis.grad3(k + 1, R.vol_pts)                          # (3, Nq, d3')
    gradP = np.einsum("eab,bqj->eaqj", BinvT, G1)               # physical
    S = np.einsum("eq,eaqi,eaqj->eij", W, gradP, gradP)
    qh = np.einsum("esj,qj->esq", q, R.P)                       # q_h at qp (Ne, 3, Nq)
    rhs = -np.einsum("eq,esq,esqi->ei", W * kinv, qh, gradP)
    us = np.zeros((elems.size, G1.shape[2]))
    us[:, 0] = u[:, 0]
    us[:, 1:] = np.linalg.solve(S[:, 1:, 1:], rhs[:, 1:, None])[..., 0]
    return us


def errors(ex, problem, k, q, u, uhat, ustar=None, nq=None):
    """Relative errors e_q, e_u, e_uhat (eq 10.1) and e* (eq 10.2) with a rule of n = k+4."""
    nq = nq if nq is not None else k + 4
    vp, vw = quadrature.tet_rule(nq)
    tp, tw = quadrature.tri_rule(nq)
    v, B, vol, _ = geometry(ex, np.arange(ex.nelt))
    xq = v[:, None, 0, :] + np.einsum("eij,qj->eqi", B, vp)
    X, Y, Z = xq[..., 0], xq[..., 1], xq[..., 2]
    W = vol[:, None] * vw[None, :]
    P = basis.eval3(k, vp)
    ue = problem.u(X, Y, Z)
    qe = np.stack(problem.q(X, Y, Z), axis=1)
    uh = u @ P.T
    qh = np.einsum("esj,qj->esq", q, P)
    out = {}
    qn = (W[:, None] * qe ** 2).sum()
    out["e_q"] = np.sqrt((W[:, None] * (qe - qh) ** 2).sum() / (qn if qn > 0 else 1.0))
    out["e_u"] = np.sqrt((W * (ue - uh) ** 2).sum() / (W * ue ** 2).sum())
    # ||v||_h^2 = sum_e |e| ||v||_e^2, ||v||_e^2 = |e| sum_r v_r v(y_r)^2
    w = ex.coordinates[ex.faces]
    y = (w[:, None, 0] + tp[None, :, 0, None] * (w[:, None, 1] - w[:, None, 0])
         + tp[None, :, 1, None] * (w[:, None, 2] - w[:, None, 0]))
    uy = problem.u(y[..., 0], y[..., 1], y[..., 2])
    Dv = basis.eval2(k, tp)
    uhy = uhat @ Dv.T
    a2 = ex.area ** 2
    out["e_uhat"] = np.sqrt((a2[:, None] * tw[None] * (uy - uhy) ** 2).sum() / (a2[:, None] * tw[None] * uy ** 2).sum())
    if ustar is not None:
        P1 = basis.eval3(k + 1, vp)
        ush = ustar @ P1.T
        out["e_star"] = np.sqrt((W * (ue - ush) ** 2).sum() / (W * ue ** 2).sum())
    return out


def solve_problem(ex, problem, k, nq=None, with_post=True):
    """The whole pipeline (Sections 3-6 and eq 9.11); returns a dict of every intermediate."""
    from .local import condense_all, rules
    R = rules(k, nq)
    C, Cf = condense_all(ex, problem, R)
    H, F = assemble(ex, k, C, Cf)
    uD = dirichlet_data(ex, problem, R)
    GN = neumann_load(ex, problem, R)
    b = rhs_with_neumann(ex, k, F, GN)
    uhat = solve_trace(ex, k, H, b, uD)
    q, u = recover_all(ex, problem, R, uhat)
    out = dict(R=R, C=C, Cf=Cf, H=H, F=F, uD=uD, GN=GN, b=b, uhat=uhat, q=q, u=u)
    if with_post:
        out["ustar"] = postprocess(ex, problem, R, q, u)
    return out
