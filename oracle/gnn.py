"""Learned face-graph preconditioner for the trace system (eq 6.5): reference definitions.

TEST INFRASTRUCTURE (oracle).  Plain NumPy, FP64.  It is imported only by tests and by
the bench's CPU baseline.

The paper fixes no solver for eq 6.5.  This module defines the preconditioner family, the
network that picks a member of it, and the training objective.  Every function states
the definition it implements; the HIP kernels are checked against these.

System and scaling
------------------
H is the block-sparse trace matrix after the Dirichlet elimination.  It has d2 x d2
blocks, and block (i, j) is nonzero when faces i and j share an element.  Dirichlet rows
and columns are the identity.  With H_ii = L_i L_i^T (Cholesky),
    Hs_ij = L_i^{-1} H_ij L_j^{-T}        (so Hs_ii = I),
which is the block-Jacobi-scaled matrix.

Preconditioner
--------------
    G = B (I + N),  N strictly block-lower on the pattern of H,
    B = diag(B_i) block diagonal, each B_i a d2 x d2 lower-triangular matrix with a positive
    diagonal, B_i[a][a] = exp(s_ia),
    M^{-1} = L^{-T} G^T G L^{-1},
which is symmetric positive definite for every N and B (G is triangular with a positive
diagonal).

Network
-------
One node per face, edges = off-diagonal blocks.  The features are:
  * node a_i (5 values): one-hot face type (interior, Dirichlet, Neumann),
    log(|e_i| nfc^{2/3}), and sum_j ||Hs_ij||_F^2 over the off-diagonal blocks of row i;
  * edge b_ij: the d2*d2 entries of Hs_ij, row-major.

The layers (h channels, relu), for l = 1..L:
    X   = relu(W0 a + c0)
    E   = relu(We b + ce)
    M_ij = relu(Wm_l [X_i; X_j; E_ij] + cm_l)
    X_i += relu(Wu_l [X_i; sum_j M_ij] + cu_l)

The head acts on the lower edges (j < i):
    N_ij = mask_ij (-Hs_ij + reshape(Wo [X_i; X_j; E_ij] + co)),
where mask_ij = 0 if face i or face j is a Dirichlet face, and a node head gives each face's
block scaling,
    beta_i = free_i (Wb X_i + cb),  fb = d2 (d2 + 1) / 2 values:
    s_ia = beta_i[a] (a < d2), and the strictly lower entries of B_i row by row
    (B_i[a][b] = beta_i[d2 + a (a - 1) / 2 + b], b < a),
with free_i = 0 on Dirichlet faces (B_i = I there).  With Wo, co, Wb, cb all zero the
preconditioner is the first-order factor G = I - tril(Hs).

Objective
---------
The objective is the logarithm of the Kaporin number (tr/n) / det^{1/n} of the
preconditioned matrix G Hs G^T, which bounds the PCG iteration count.  det(G Hs G^T) =
det(B)^2 det(Hs), and det(Hs) does not depend on the network, so up to a constant
    loss = log T - (2 / n) sum_i sum_a s_ia,
    T = 1 / (p n) sum_z (G^T z)^T Hs (G^T z)   (the probe estimate of tr(G Hs G^T) / n),
with p probe vectors z and n = nfc d2 unknowns.  The loss does not change when G is
multiplied by a constant.

Parameter vector
----------------
One flat array in the order W0, c0, We, ce, then (Wm_l, cm_l, Wu_l, cu_l) for each l,
then Wo, co, then Wb, cb.  Matrices are stored row-major (output, input).
"""
from __future__ import annotations

from dataclasses import dataclass

import numpy as np

F0 = 5  # node features


@dataclass(frozen=True)
class Shape:
    d2: int
    hidden: int = 32
    layers: int = 3

    @property
    def fe(self):
        return self.d2 * self.d2

    @property
    def fb(self):
        return self.d2 * (self.d2 + 1) // 2


def param_layout(s: Shape):
    h, fe = s.hidden, s.fe
    lay = [("W0", (h, F0)), ("c0", (h,)), ("We", (h, fe)), ("ce", (h,))]
    for l in range(s.layers):
        lay += [(f"Wm{l}", (h, 3 * h)), (f"cm{l}", (h,)), (f"Wu{l}", (h, 2 * h)), (f"cu{l}", (h,))]
    lay += [("Wo", (fe, 3 * h)), ("co", (fe,)), ("Wb", (s.fb, h)), ("cb", (s.fb,))]
    return lay


def param_count(s: Shape) -> int:
    return sum(int(np.prod(sh)) for _, sh in param_layout(s))


def unpack(theta, s: Shape):
    out, o = {}, 0
    for name, sh in param_layout(s):
        n = int(np.prod(sh))
        out[name] = np.asarray(theta[o:o + n], dtype=np.float64).reshape(sh)
        o += n
    return out


def pack(p, s: Shape):
    return np.concatenate([np.asarray(p[name], dtype=np.float64).ravel() for name, _ in param_layout(s)])


# ----------------------------------------------------------------------------- graph of one system
def block_pattern(facebyele, nfc):
    """Block pattern of H: (i, j) for every pair of faces of one element (including i = j),
    as CSR with columns ascending in each row; erow[e] = block row of entry e."""
    fbe = np.asarray(facebyele)
    rows = np.repeat(fbe, 4, axis=1).ravel()
    cols = np.tile(fbe, (1, 4)).ravel()
    key = np.unique(rows.astype(np.int64) * nfc + cols)
    r, c = key // nfc, key % nfc
    row_ptr = np.zeros(nfc + 1, dtype=np.int64)
    np.add.at(row_ptr, r + 1, 1)
    return np.cumsum(row_ptr), c.astype(np.int64), r.astype(np.int64)


def bsr_blocks(Hcsr, row_ptr, col_idx, erow, d2):
    """blocks[e] = H[i d2:(i+1) d2, j d2:(j+1) d2] for e = (i, j) of the pattern."""
    Hd = Hcsr.tocsr()
    out = np.zeros((col_idx.size, d2, d2))
    for a in range(d2):
        for b in range(d2):
            out[:, a, b] = np.asarray(Hd[erow * d2 + a, col_idx * d2 + b]).ravel()
    return out


def dirichlet_eliminate(blocks, col_idx, erow, ftype, d2):
    """H_II kept, Dirichlet rows and columns replaced by the identity (eq 6.5 after the
    elimination of the Dirichlet traces)."""
    out = blocks.copy()
    dr = ftype[erow] == 1
    dc = ftype[col_idx] == 1
    out[dr | dc] = 0.0
    out[dr & (erow == col_idx)] = np.eye(d2)
    return out


def mirror_index(row_ptr, col_idx, erow):
    """mirror[e] = position of block (j, i) for e = (i, j)."""
    nfc = row_ptr.size - 1
    key = erow.astype(np.int64) * nfc + col_idx
    tkey = col_idx.astype(np.int64) * nfc + erow
    return np.searchsorted(key, tkey)


def graph(blocks, row_ptr, col_idx, erow, ftype, area):
    """Scaled blocks Hs, the Cholesky inverses Linv, node and edge features."""
    nfc = row_ptr.size - 1
    d2 = blocks.shape[1]
    diag = np.array([row_ptr[i] + np.searchsorted(col_idx[row_ptr[i]:row_ptr[i + 1]], i) for i in range(nfc)])
    Linv = np.linalg.inv(np.linalg.cholesky(blocks[diag]))
    Hs = Linv[erow] @ blocks @ np.transpose(Linv[col_idx], (0, 2, 1))
    off = erow != col_idx
    energy = np.zeros(nfc)
    np.add.at(energy, erow[off], np.sum(Hs[off] ** 2, axis=(1, 2)))
    node = np.zeros((nfc, F0))
    node[np.arange(nfc), np.asarray(ftype)] = 1.0
    node[:, 3] = np.log(np.asarray(area) * nfc ** (2.0 / 3.0))
    node[:, 4] = energy
    return dict(Hs=Hs, Linv=Linv, node=node, edge=Hs.reshape(-1, d2 * d2), diag=diag)


# ----------------------------------------------------------------------------- network
def relu(x):
    return np.maximum(x, 0.0)


def forward(theta, s: Shape, g, row_ptr, col_idx, erow, ftype):
    """N (nnzb, d2, d2), nonzero on the lower off-diagonal blocks, the block-scaling
    parameters beta (nfc, fb), zero on Dirichlet faces, and the cache for backward."""
    p = unpack(theta, s)
    nfc = row_ptr.size - 1
    off = erow != col_idx
    low = col_idx < erow
    mask = (low & (ftype[erow] != 1) & (ftype[col_idx] != 1)).astype(np.float64)
    X = relu(g["node"] @ p["W0"].T + p["c0"])
    B = g["edge"]
    Eh = relu(B @ p["We"].T + p["ce"]) * off[:, None]
    cache = dict(X0=X, Eh=Eh, layers=[])
    for l in range(s.layers):
        Xin = X
        V = np.concatenate([Xin[erow], Xin[col_idx], Eh], axis=1) @ p[f"Wm{l}"].T + p[f"cm{l}"]
        Mm = relu(V) * off[:, None]
        Agg = np.zeros_like(Xin)
        np.add.at(Agg, erow, Mm)
        U = np.concatenate([Xin, Agg], axis=1) @ p[f"Wu{l}"].T + p[f"cu{l}"]
        X = Xin + relu(U)
        cache["layers"].append(dict(Xin=Xin, V=V, Agg=Agg, U=U))
    Z = np.concatenate([X[erow], X[col_idx], Eh], axis=1)
    D = Z @ p["Wo"].T + p["co"]
    N = (mask[:, None] * (-B + D)).reshape(-1, s.d2, s.d2)
    free = (np.asarray(ftype) != 1).astype(np.float64)
    beta = free[:, None] * (X @ p["Wb"].T + p["cb"])
    cache.update(X=X, Zo=Z, mask=mask, off=off, free=free)
    return N, beta, cache


def block_scale(beta, d2):
    """B (nfc, d2, d2): lower triangular, B[a][a] = exp(beta[a]), B[a][b] = beta[d2 + a(a-1)/2 + b]."""
    nfc = beta.shape[0]
    B = np.zeros((nfc, d2, d2))
    for a in range(d2):
        B[:, a, a] = np.exp(beta[:, a])
        for b in range(a):
            B[:, a, b] = beta[:, d2 + a * (a - 1) // 2 + b]
    return B


def apply_GT(N, z, row_ptr, col_idx, erow):
    """u = G^T z = z + N^T z, block vectors (nfc, d2)."""
    u = z.copy()
    low = col_idx < erow
    np.add.at(u, col_idx[low], np.einsum("eab,ea->eb", N[low], z[erow[low]]))
    return u


def apply_H(Hs, u, col_idx, erow):
    out = np.zeros_like(u)
    np.add.at(out, erow, np.einsum("eab,eb->ea", Hs, u[col_idx]))
    return out


def apply_G_lower(N, v, row_ptr, col_idx, erow):
    """(I + N) v for block vectors (nfc, d2): v_i + sum_{j < i} N_ij v_j."""
    out = v.copy()
    low = col_idx < erow
    np.add.at(out, erow[low], np.einsum("eab,eb->ea", N[low], v[col_idx[low]]))
    return out


def kaporin_loss(N, beta, Hs, row_ptr, col_idx, erow, Z):
    """loss = log T - (2/n) sum s (module docstring) and its gradients dloss/dN (on the lower
    blocks; the caller masks) and dloss/dbeta.  Z: (p, nfc, d2) probe vectors.

    With y = B^T z, u = (I + N)^T y, hu = Hs u:
      dT/dN_ij = 2/(p n) sum_z y_i hu_j^T,   dT/dB_i[a][b] = 2/(p n) sum_z z_i[a] w_i[b],
    where w = (I + N) hu."""
    p = Z.shape[0]
    nfc, d2 = Z.shape[1], Z.shape[2]
    n = nfc * d2
    scale = 1.0 / (p * n)
    Bm = block_scale(beta, d2)
    T = 0.0
    dTN = np.zeros_like(N)
    dTB = np.zeros_like(Bm)
    low = col_idx < erow
    for z in Z:
        y = np.einsum("iab,ia->ib", Bm, z)
        u = apply_GT(N, y, row_ptr, col_idx, erow)
        hu = apply_H(Hs, u, col_idx, erow)
        T += scale * float(np.sum(u * hu))
        dTN[low] += 2.0 * scale * np.einsum("ea,eb->eab", y[erow[low]], hu[col_idx[low]])
        w = apply_G_lower(N, hu, row_ptr, col_idx, erow)
        dTB += 2.0 * scale * np.einsum("ia,ib->iab", z, w)
    loss = np.log(T) - 2.0 / n * float(beta[:, :d2].sum())
    dbeta = np.zeros_like(beta)
    for a in range(d2):
        dbeta[:, a] = dTB[:, a, a] * Bm[:, a, a] / T - 2.0 / n
        for b in range(a):
            dbeta[:, d2 + a * (a - 1) // 2 + b] = dTB[:, a, b] / T
    return loss, dTN / T, dbeta


def backward(theta, s: Shape, g, cache, dN, dbeta, row_ptr, col_idx, erow):
    """Gradient of a scalar objective with respect to theta, given its gradients dN and dbeta."""
    p = unpack(theta, s)
    gp = {name: np.zeros(sh) for name, sh in param_layout(s)}
    h = s.hidden
    mask, off = cache["mask"], cache["off"]
    dbeta = cache["free"][:, None] * dbeta
    gp["Wb"] = dbeta.T @ cache["X"]
    gp["cb"] = dbeta.sum(0)
    dD = mask[:, None] * dN.reshape(-1, s.fe)
    gp["Wo"] = dD.T @ cache["Zo"]
    gp["co"] = dD.sum(0)
    dZ = dD @ p["Wo"]
    dX = dbeta @ p["Wb"]
    np.add.at(dX, erow, dZ[:, :h])
    np.add.at(dX, col_idx, dZ[:, h:2 * h])
    dEh = dZ[:, 2 * h:].copy()
    for l in reversed(range(s.layers)):
        c = cache["layers"][l]
        dU = dX * (c["U"] > 0)
        gp[f"Wu{l}"] = dU.T @ np.concatenate([c["Xin"], c["Agg"]], axis=1)
        gp[f"cu{l}"] = dU.sum(0)
        dXin = dX + dU @ p[f"Wu{l}"][:, :h]
        dAgg = dU @ p[f"Wu{l}"][:, h:]
        dV = dAgg[erow] * (c["V"] > 0) * off[:, None]
        gp[f"Wm{l}"] = dV.T @ np.concatenate([c["Xin"][erow], c["Xin"][col_idx], cache["Eh"]], axis=1)
        gp[f"cm{l}"] = dV.sum(0)
        dIn = dV @ p[f"Wm{l}"]
        np.add.at(dXin, erow, dIn[:, :h])
        np.add.at(dXin, col_idx, dIn[:, h:2 * h])
        dEh += dIn[:, 2 * h:]
        dX = dXin
    dEpre = dEh * (cache["Eh"] > 0) * off[:, None]
    gp["We"] = dEpre.T @ g["edge"]
    gp["ce"] = dEpre.sum(0)
    dX0 = dX * (cache["X0"] > 0)
    gp["W0"] = dX0.T @ g["node"]
    gp["c0"] = dX0.sum(0)
    return pack(gp, s)


def loss_and_grad(theta, s: Shape, g, row_ptr, col_idx, erow, ftype, Z):
    N, beta, cache = forward(theta, s, g, row_ptr, col_idx, erow, ftype)
    loss, dN, dbeta = kaporin_loss(N, beta, g["Hs"], row_ptr, col_idx, erow, Z)
    return loss, backward(theta, s, g, cache, dN, dbeta, row_ptr, col_idx, erow), N, beta


def init_params(s: Shape, seed=0):
    """He-style random weights; both heads start at zero (G = I - tril(Hs), B = I)."""
    rng = np.random.default_rng(seed)
    p = {}
    for name, sh in param_layout(s):
        if name.startswith("W") and name not in ("Wo", "Wb"):
            p[name] = rng.standard_normal(sh) * np.sqrt(2.0 / sh[1])
        else:
            p[name] = np.zeros(sh)
    return pack(p, s)


def preconditioner_apply(N, beta, Linv, r, row_ptr, col_idx, erow):
    """z = L^{-T} G^T G L^{-1} r with G = B (I + N), for block vectors (nfc, d2)."""
    d2 = r.shape[1]
    t = np.einsum("iab,ib->ia", Linv, r)
    s_ = apply_G_lower(N, t, row_ptr, col_idx, erow)
    Bm = block_scale(beta, d2)
    v = np.einsum("iab,ib->ia", Bm, s_)
    y = apply_GT(N, np.einsum("iba,ib->ia", Bm, v), row_ptr, col_idx, erow)
    return np.einsum("iba,ib->ia", Linv, y)
