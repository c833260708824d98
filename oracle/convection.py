"""HDG for convection-diffusion (Section 9, "Matrices for convection-diffusion problems";
oracle).

The paper supplies the matrices (eq 9.1: the convection matrices int_K m P_i d_* P_j with a
variable coefficient m; surface matrices int_e alpha D_i P_j and int_e alpha D_i D_j with a
variable alpha) and names the forms that an HDG method for convection-diffusion needs.  The
method is not written out there; the reading taken is the standard conservative HDG
discretisation of

    kappa^{-1} q + grad u = 0,   div(q + beta u) + c u = f,

with the numerical total flux  (q_hat + beta u_hat).nu = q_h.nu + (beta.nu) u_hat_h + tau (u_h - u_hat_h):
  (kappa^{-1} q_h, r)_K - (u_h, div r)_K + <u_hat_h, r.nu>_dK = 0
  (div q_h, w)_K - (beta u_h, grad w)_K + <(beta.nu) u_hat_h + tau (u_h - u_hat_h), w>_dK + (c u_h, w)_K = (f, w)_K
  sum over the elements of a face of <q_h.nu + (beta.nu) u_hat_h + tau (u_h - u_hat_h), v>_e = 0,
with u_hat = u_D on Dirichlet faces and, on Neumann faces, the total normal flux given:
-(q_hat + beta u_hat).nu = g_N.nu.  Testing with the solution itself gives
(kappa^{-1} q, q) + ((c + div(beta)/2) u, u) + sum <(tau - beta.nu / 2)(u - u_hat), u - u_hat>,
so the method is stable for tau >= beta.nu / 2 on every face (and c + div(beta)/2 >= 0).

Element matrices in the HDG layout of Section 5:
  A1 = HDG A1 with  - sum_s E_s^T  added to its u block, E_s[i, j] = int_K beta_s P_i d_s P_j (eq 9.1)
  A2 = HDG A2 with  + (beta.n DP)^T  added to its u rows, (beta.n DP)_l[i, j] = int_{e_l} (beta.nu) D_i P_j
  A3 = HDG A3,   C^K = A3 A1^{-1} A2 + tau DD - (beta.n DD),   Cf^K = A3 A1^{-1} Af,
(beta.n DD)_l[i, j] = int_{e_l} (beta.nu) D_i D_j.  The beta surface integrals are quadrature sums
at the element's own face points phi_l^K(qhat_r) (eq 2.5), where D_i is evaluated through the
face's own parametrisation (D_i(phi_e^{-1}(x))); the rest of the oracle is unchanged.
"""
from __future__ import annotations

from types import SimpleNamespace

import numpy as np
import scipy.sparse as sp
import scipy.sparse.linalg as spla

from . import basis
from .globalsys import assemble, dirichlet_data, neumann_load, rhs_with_neumann
from .local import Rules, geometry, local_blocks, local_solver_matrices, rules

# eq 2.5: the reference faces as maps of (s, t)
_REF_FACE = (lambda s, t: np.stack([s, t, 0 * s], -1), lambda s, t: np.stack([s, 0 * s, t], -1),
             lambda s, t: np.stack([0 * s, s, t], -1), lambda s, t: np.stack([s, t, 1 - s - t], -1))


def element_face_points(ex, elems, R: Rules):
    """Physical points phi_l^K(qhat_r) of the element-local face parametrisation: (Ne, 4, Nq2, 3)."""
    v, B, _, _ = geometry(ex, elems)
    s, t = R.tri_pts[:, 0], R.tri_pts[:, 1]
    out = [v[:, None, 0, :] + np.einsum("eij,rj->eri", B, _REF_FACE[l](s, t)) for l in range(4)]
    return np.stack(out, axis=1)


def face_basis_at(ex, faces, x, k):
    """D_i of each face at physical points on it: x (Nf, Nr, 3) -> (Nf, Nr, d2), through the
    face's own parametrisation (normal equations of the 2 x 2 map)."""
    w = ex.coordinates[ex.faces[faces]]
    e1, e2 = w[:, 1] - w[:, 0], w[:, 2] - w[:, 0]
    G = np.stack([np.stack([(e1 * e1).sum(-1), (e1 * e2).sum(-1)], -1),
                  np.stack([(e2 * e1).sum(-1), (e2 * e2).sum(-1)], -1)], -2)
    rhs = np.stack([np.einsum("frd,fd->fr", x - w[:, None, 0], e1), np.einsum("frd,fd->fr", x - w[:, None, 0], e2)], -1)
    st = np.linalg.solve(G[:, None], rhs[..., None])[..., 0]
    return np.stack([basis.eval2(k, p) for p in st])


def convection_blocks(ex, beta, R: Rules, elems=None):
    """E_s (3, Ne, d3, d3), beta.n DP (Ne, 4, d2, d3), beta.n DD (Ne, 4, d2, d2)."""
    if elems is None:
        elems = np.arange(ex.nelt)
    elems = np.asarray(elems)
    k = R.k
    v, B, vol, BinvT = geometry(ex, elems)
    xq = v[:, None, 0, :] + np.einsum("eij,qj->eqi", B, R.vol_pts)
    bq = np.stack([np.asarray(c, dtype=np.float64) * np.ones(xq.shape[:2]) for c in beta(xq[..., 0], xq[..., 1], xq[..., 2])],
                  axis=0)                                        # (3, Ne, Nq)
    W = vol[:, None] * R.vol_w[None, :]
    gradP = np.einsum("eab,bqj->eaqj", BinvT, R.Pg)              # (Ne, 3, Nq, d3)
    E = np.einsum("eq,seq,qi,esqj->seij", W, bq, R.P, gradP)
    xf = element_face_points(ex, elems, R)                       # (Ne, 4, Nq2, 3)
    d2, d3 = basis.dim2(k), basis.dim3(k)
    bnDP = np.zeros((elems.size, 4, d2, d3))
    bnDD = np.zeros((elems.size, 4, d2, d2))
    Binv = np.linalg.inv(B)
    s, t = R.tri_pts[:, 0], R.tri_pts[:, 1]
    for l in range(4):
        x = xf[:, l]
        bx = np.stack([np.asarray(c, dtype=np.float64) * np.ones(x.shape[:2]) for c in beta(x[..., 0], x[..., 1], x[..., 2])],
                      axis=-1)                                   # (Ne, Nq2, 3)
        alpha = np.einsum("erd,ed->er", bx, ex.normals[elems, l])   # (beta.nu) |e|
        Pl = basis.eval3(k, _REF_FACE[l](s, t))                  # (Nq2, d3)
        Dl = face_basis_at(ex, ex.facebyele[elems, l], x, k)     # (Ne, Nq2, d2)
        bnDP[:, l] = np.einsum("r,er,eri,rj->eij", R.tri_w, alpha, Dl, Pl)
        bnDD[:, l] = np.einsum("r,er,eri,erj->eij", R.tri_w, alpha, Dl, Dl)
    return E, bnDP, bnDD


def cd_matrices(ex, problem, R: Rules, elems=None):
    """A1, A2, Af, A3 and the face blocks tau DD - beta.n DD of the convection-diffusion element."""
    b = local_blocks(ex, problem, R, elems)
    A1, A2, Af, A3 = local_solver_matrices(b)
    E, bnDP, bnDD = convection_blocks(ex, problem.beta, R, b["elems"])
    Ne, d3 = b["M_kinv"].shape[0], b["M_kinv"].shape[1]
    d2 = bnDP.shape[2]
    A1 = A1.copy()
    A1[:, 3 * d3:, 3 * d3:] -= E.sum(axis=0).transpose(0, 2, 1)
    A2 = A2.copy()
    A2[:, 3 * d3:, :] += bnDP.reshape(Ne, 4 * d2, d3).transpose(0, 2, 1)
    face = b["tauDD"].copy()
    for l in range(4):
        face[:, l * d2:(l + 1) * d2, l * d2:(l + 1) * d2] -= bnDD[:, l]
    return A1, A2, Af, A3, face


def condense(ex, problem, k, nq=None, elems=None):
    R = rules(k, nq)
    A1, A2, Af, A3, face = cd_matrices(ex, problem, R, elems)
    X = np.linalg.solve(A1, np.concatenate([A2, Af[:, :, None]], axis=2))
    return np.einsum("eij,ejk->eik", A3, X[:, :, :-1]) + face, np.einsum("eij,ej->ei", A3, X[:, :, -1])


def solve_problem(ex, problem, k, nq=None):
    """Condensation, assembly (eq 6.5), boundary data (eq 6.3, 6.4 with the total flux on
    Neumann faces), a sparse LU solve of the non-symmetric trace system, reconstruction."""
    R = rules(k, nq)
    d3, d2 = basis.dim3(k), basis.dim2(k)
    A1, A2, Af, A3, face = cd_matrices(ex, problem, R)
    X = np.linalg.solve(A1, np.concatenate([A2, Af[:, :, None]], axis=2))
    C = np.einsum("eij,ejk->eik", A3, X[:, :, :-1]) + face
    Cf = np.einsum("eij,ej->ei", A3, X[:, :, -1])
    H, F = assemble(ex, k, C, Cf)
    uD = dirichlet_data(ex, problem, R)
    GN = neumann_load(ex, problem, R)
    b = rhs_with_neumann(ex, k, F, GN)
    uhat = np.zeros((ex.nfc, d2))
    uhat[ex.dirfaces] = uD
    isD = np.zeros(ex.nfc, dtype=bool)
    isD[ex.dirfaces] = True
    Dd = np.repeat(isD, d2)
    I, Di = np.nonzero(~Dd)[0], np.nonzero(Dd)[0]
    rhs = b[I] - H[I][:, Di] @ uhat.ravel()[Di]
    uhat.ravel()[I] = spla.splu(H[I][:, I].tocsc()).solve(rhs)
    uK = uhat[ex.facebyele].reshape(ex.nelt, -1)
    x = np.linalg.solve(A1, (Af - np.einsum("eij,ej->ei", A2, uK))[:, :, None])[:, :, 0]
    return dict(C=C, Cf=Cf, H=H, F=F, b=b, uD=uD, uhat=uhat, X=X,
                q=x[:, :3 * d3].reshape(-1, 3, d3), u=x[:, 3 * d3:])


def brute_solve(ex, problem, k, nq=None):
    """The uncondensed convection-diffusion system: element equations, total-flux continuity
    on interior faces, Neumann and Dirichlet rows."""
    R = rules(k, nq)
    d3, d2 = basis.dim3(k), basis.dim2(k)
    A1, A2, Af, A3, face = cd_matrices(ex, problem, R)
    nv = 4 * d3
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
        add(tK[keep], tK, -face[K][keep])
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
    return qu[:, :3 * d3].reshape(Nelt, 3, d3), qu[:, 3 * d3:], x[off:].reshape(Nfc, d2)
