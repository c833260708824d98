"""Per-element HDG blocks and static condensation (oracle).

Everything is computed directly in physical space for a batch of elements, in
float64, following Sections 3-5:

  volume terms (Section 5, "Volume terms"; eq 3.2, 3.55):
      M_m[i,j]  = sum_q |K| w_q m(x_q) P_i(x_q) P_j(x_q),   m in {1/kappa, c}
      C_s[i,j]  = sum_q |K| w_q P_i(x_q) d_s P_j(x_q),      grad = B^{-T} grad_hat
      f[i]      = sum_q |K| w_q f(x_q) P_i(x_q)
  surface terms (Section 4, types (a)-(c); Section 5, "Surface terms"), each face
  integrated in the face's own parametrisation phi_e (Section 2) so that the
  permutation index is *not* used here:
      tauPP[i,j]      = sum_l tau_l |e_l| sum_r v_r P_i(y_r) P_j(y_r)
      tauDP_l[i,j]    = tau_l |e_l| sum_r v_r D_i(qhat_r) P_j(y_r)
      nsDP_l[i,j]     = n_{l,s} sum_r v_r D_i(qhat_r) P_j(y_r)
      tauDD_l[i,j]    = tau_l |e_l| sum_r v_r D_i(qhat_r) D_j(qhat_r)
  with y_r = phi_e(qhat_r) and P_j(y) = Phat_j(F_K^{-1}(y));
  local solver blocks A1, A2, Af, A3 (eq 5.1, 5.2, 5.4; the last block row of A1
  read as [C_x C_y C_z  M_c + tauPP]), and the condensed blocks
      C  = A3 A1^{-1} A2 + tauDD   (eq 5.5),    Cf = A3 A1^{-1} Af   (eq 5.6)
  by dense LU solves.
"""
from __future__ import annotations

from dataclasses import dataclass

import numpy as np

from . import basis, quadrature


@dataclass
class Rules:
    k: int
    nq: int
    vol_pts: np.ndarray
    vol_w: np.ndarray
    P: np.ndarray       # (Nq, d3)
    Pg: np.ndarray      # (3, Nq, d3) reference gradients
    tri_pts: np.ndarray
    tri_w: np.ndarray
    D: np.ndarray       # (Nq2, d2)


def rules(k: int, nq: int | None = None) -> Rules:
    nq = nq if nq is not None else k + 2
    vp, vw = quadrature.tet_rule(nq)
    tp, tw = quadrature.tri_rule(nq)
    return Rules(k=k, nq=nq, vol_pts=vp, vol_w=vw, P=basis.eval3(k, vp), Pg=basis.grad3(k, vp),
                 tri_pts=tp, tri_w=tw, D=basis.eval2(k, tp))


def geometry(ex, elems):
    """B_K (eq 2.0), |K| = det B / 6, B^{-T}, first vertex."""
    v = ex.coordinates[ex.elements[elems]]  # (Ne, 4, 3)
    B = np.stack([v[:, 1] - v[:, 0], v[:, 2] - v[:, 0], v[:, 3] - v[:, 0]], axis=2)  # columns
    vol = np.linalg.det(B) / 6.0
    BinvT = np.linalg.inv(B).transpose(0, 2, 1)
    return v, B, vol, BinvT


def volume_points(ex, elems, R: Rules):
    """Physical quadrature points x_q = F_K(p_q) (eq 3.2, 3.4): (Ne, Nq, 3)."""
    v, B, _, _ = geometry(ex, elems)
    return v[:, None, 0, :] + np.einsum("eij,qj->eqi", B, R.vol_pts)


def face_points(ex, faces, R: Rules):
    """y_r = phi_e(qhat_r) on the given faces (Section 4): (Nf, Nq2, 3)."""
    w = ex.coordinates[ex.faces[faces]]  # (Nf, 3, 3)
    s, t = R.tri_pts[:, 0], R.tri_pts[:, 1]
    return (w[:, None, 0] + s[None, :, None] * (w[:, None, 1] - w[:, None, 0])
            + t[None, :, None] * (w[:, None, 2] - w[:, None, 0]))


def _tau_array(tau, ex):
    if np.isscalar(tau):
        return np.full((ex.nelt, 4), float(tau))
    return np.asarray(tau, dtype=np.float64).reshape(ex.nelt, 4)


def local_blocks(ex, problem, R: Rules, elems=None):
    """All element blocks of Section 5 for the elements ``elems`` (default: all)."""
    if elems is None:
        elems = np.arange(ex.nelt)
    elems = np.asarray(elems)
    k = R.k
    v, B, vol, BinvT = geometry(ex, elems)
    Ne = elems.size
    # ---- volume terms
    xq = volume_points(ex, elems, R)
    X, Y, Z = xq[..., 0], xq[..., 1], xq[..., 2]
    W = vol[:, None] * R.vol_w[None, :]                   # |K| w_q
    kinv = 1.0 / np.asarray(problem.kappa(X, Y, Z), dtype=np.float64)
    cval = np.asarray(problem.c(X, Y, Z), dtype=np.float64) * np.ones_like(X)
    fval = np.asarray(problem.f(X, Y, Z), dtype=np.float64) * np.ones_like(X)
    P = R.P
    M_kinv = np.einsum("eq,qi,qj->eij", W * kinv, P, P)
    M_c = np.einsum("eq,qi,qj->eij", W * cval, P, P)
    fK = np.einsum("eq,qi->ei", W * fval, P)
    gradP = np.einsum("eab,bqj->eaqj", BinvT, R.Pg)        # physical gradients (Ne, 3, Nq, d3)
    C = np.einsum("eq,qi,esqj->seij", W, P, gradP)         # (3, Ne, d3, d3)
    # ---- surface terms, in each face's own parametrisation
    tau = _tau_array(problem.tau, ex)[elems]
    Dh = R.D                                               # (Nq2, d2)
    vw = R.tri_w
    d2 = Dh.shape[1]
    d3 = P.shape[1]
    tauPP = np.zeros((Ne, d3, d3))
    tauDP = np.zeros((Ne, 4, d2, d3))
    nDP = np.zeros((3, Ne, 4, d2, d3))
    tauDD = np.zeros((Ne, 4 * d2, 4 * d2))
    Binv = np.linalg.inv(B)
    for l in range(4):
        fcs = ex.facebyele[elems, l]
        y = face_points(ex, fcs, R)                        # (Ne, Nq2, 3)
        xhat = np.einsum("eij,erj->eri", Binv, y - v[:, None, 0, :])
        Py = basis.eval3(k, xhat)                          # (Ne, Nq2, d3) = P_j(y_r)
        area = ex.area[fcs]
        T = tau[:, l] * area
        tauPP += T[:, None, None] * np.einsum("r,eri,erj->eij", vw, Py, Py)
        DPl = np.einsum("r,ri,erj->eij", vw, Dh, Py)       # sum_r v_r D_i P_j
        tauDP[:, l] = T[:, None, None] * DPl
        for s in range(3):
            nDP[s, :, l] = ex.normals[elems, l, s][:, None, None] * DPl
        DD = np.einsum("r,ri,rj->ij", vw, Dh, Dh)
        tauDD[:, l * d2:(l + 1) * d2, l * d2:(l + 1) * d2] = T[:, None, None] * DD[None]
    return dict(elems=elems, vol=vol, M_kinv=M_kinv, M_c=M_c, C=C, f=fK, tauPP=tauPP,
                tauDP=tauDP, nDP=nDP, tauDD=tauDD, kinv_q=kinv, xq=xq)


def local_solver_matrices(b):
    """A1 (4d3 x 4d3), A2 (4d3 x 4d2), Af (4d3), A3 (4d2 x 4d3): eq 5.1, 5.2, 5.4."""
    Ne, d3, _ = b["M_kinv"].shape
    d2 = b["tauDP"].shape[2]
    m = 4 * d2
    A1 = np.zeros((Ne, 4 * d3, 4 * d3))
    Cx, Cy, Cz = b["C"]
    for s, Cs in enumerate((Cx, Cy, Cz)):
        A1[:, s * d3:(s + 1) * d3, s * d3:(s + 1) * d3] = b["M_kinv"]
        A1[:, s * d3:(s + 1) * d3, 3 * d3:] = -Cs.transpose(0, 2, 1)
        A1[:, 3 * d3:, s * d3:(s + 1) * d3] = Cs
    A1[:, 3 * d3:, 3 * d3:] = b["M_c"] + b["tauPP"]
    # stacked face blocks: rows l*d2 + i
    nDP = b["nDP"].reshape(3, Ne, m, d3)
    tauDP = b["tauDP"].reshape(Ne, m, d3)
    A2 = np.concatenate([nDP[0].transpose(0, 2, 1), nDP[1].transpose(0, 2, 1),
                         nDP[2].transpose(0, 2, 1), -tauDP.transpose(0, 2, 1)], axis=1)
    A3 = np.concatenate([nDP[0], nDP[1], nDP[2], tauDP], axis=2)
    Af = np.zeros((Ne, 4 * d3))
    Af[:, 3 * d3:] = b["f"]
    return A1, A2, Af, A3


def condense(b):
    """C^K and Cf^K (eq 5.5, 5.6)."""
    A1, A2, Af, A3 = local_solver_matrices(b)
    X = np.linalg.solve(A1, np.concatenate([A2, Af[:, :, None]], axis=2))
    C = np.einsum("eij,ejk->eik", A3, X[:, :, :-1]) + b["tauDD"]
    Cf = np.einsum("eij,ej->ei", A3, X[:, :, -1])
    return C, Cf


def condense_all(ex, problem, R: Rules, chunk: int = 4096):
    """C^K, Cf^K for every element, in chunks."""
    Cs, Cfs = [], []
    for s in range(0, ex.nelt, chunk):
        b = local_blocks(ex, problem, R, np.arange(s, min(s + chunk, ex.nelt)))
        C, Cf = condense(b)
        Cs.append(C)
        Cfs.append(Cf)
    return np.concatenate(Cs), np.concatenate(Cfs)


def recover(b, uK):
    """(q_K, u_K) from A1 [q; u] = Af - A2 u_dK (eq 5.3 / Section 6 "Reconstruction").

    uK: (Ne, 4 d2) trace coefficients in facebyele order.  Returns q (Ne, 3, d3), u (Ne, d3)."""
    A1, A2, Af, _ = local_solver_matrices(b)
    x = np.linalg.solve(A1, (Af - np.einsum("eij,ej->ei", A2, uK))[:, :, None])[:, :, 0]
    d3 = b["M_kinv"].shape[1]
    return x[:, :3 * d3].reshape(-1, 3, d3), x[:, 3 * d3:]
