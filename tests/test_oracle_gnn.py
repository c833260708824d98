"""Pins of the learned-preconditioner oracle (oracle/gnn.py).

The preconditioner family and its network are not in the paper, so nothing here is a
printed value.  Parity of the definitions is pinned instead:
  * the hand-written backward against central differences of the forward pass;
  * the log-Kaporin probe loss and its N- and B-gradients against dense linear algebra
    (exact with unit probes: log(tr/n^2) and log det G by slogdet);
  * the Kaporin stationarity of the optimal block scaling B_i = chol(A_ii)^{-1};
  * the structure: unit-diagonal scaling, SPD preconditioner, mirror and pattern integrity.
"""
import numpy as np
import pytest
import scipy.sparse as sp

from hdg_inputs import kuhn_mesh
from hdg_inputs.fields import constant_rhs_problem
from oracle import gnn as OGN, globalsys as OG, local as OL, mesh as OM


def small_system(n=2, k=1, seed=0):
    m = kuhn_mesh(n, jitter=0.1, seed=seed, dirichlet_sides=("x0", "y1"), neumann_sides=("x1", "y0", "z0", "z1"))
    ex = OM.expand(m.coordinates, m.elements, m.dirichlet, m.neumann)
    pb = constant_rhs_problem(1.5, 0.3, 10 + seed, 0.1)
    R = OL.rules(k)
    b = OL.local_blocks(ex, pb, R, np.arange(ex.nelt))
    C, Cf = OL.condense(b)
    H, _ = OG.assemble(ex, k, C, Cf)
    d2 = (k + 1) * (k + 2) // 2
    rp, ci, er = OGN.block_pattern(ex.facebyele, ex.nfc)
    blocks = OGN.dirichlet_eliminate(OGN.bsr_blocks(H, rp, ci, er, d2), ci, er, ex.ftype, d2)
    g = OGN.graph(blocks, rp, ci, er, ex.ftype, ex.area)
    return dict(ex=ex, H=H, d2=d2, rp=rp, ci=ci, er=er, blocks=blocks, g=g)


def dense_blocks(vals, rp, ci, er, nfc, d2):
    A = np.zeros((nfc * d2, nfc * d2))
    for e in range(ci.size):
        A[er[e] * d2:(er[e] + 1) * d2, ci[e] * d2:(ci[e] + 1) * d2] = vals[e]
    return A


@pytest.fixture(scope="module")
def sysk1():
    return small_system()


def test_pattern_holds_every_block_and_mirror(sysk1):
    S = sysk1
    H, d2, nfc = S["H"].tocsr(), S["d2"], S["ex"].nfc
    r, c = H.nonzero()
    pat = set(zip(S["er"].tolist(), S["ci"].tolist()))
    assert set(zip((r // d2).tolist(), (c // d2).tolist())) <= pat
    mir = OGN.mirror_index(S["rp"], S["ci"], S["er"])
    assert np.array_equal(S["er"][mir], S["ci"]) and np.array_equal(S["ci"][mir], S["er"])
    for i in range(nfc):  # columns ascending, each row holds its diagonal
        cols = S["ci"][S["rp"][i]:S["rp"][i + 1]]
        assert np.all(np.diff(cols) > 0) and i in cols
    # every interior face touches 6 others, a boundary face 3 (two / one elements)
    deg = np.diff(S["rp"]) - 1
    nel = np.bincount(S["ex"].facebyele.ravel(), minlength=nfc)
    assert np.array_equal(deg, 3 * nel)


def test_scaled_blocks_and_elimination(sysk1):
    S = sysk1
    g, d2 = S["g"], S["d2"]
    diag = S["er"] == S["ci"]
    assert np.abs(g["Hs"][diag] - np.eye(d2)).max() < 1e-12
    ft = S["ex"].ftype
    dmask = (ft[S["er"]] == 1) | (ft[S["ci"]] == 1)
    assert not g["Hs"][dmask & ~diag].any()
    # Hs = Linv H Linv^T as dense matrices
    nfc = S["ex"].nfc
    A = dense_blocks(S["blocks"], S["rp"], S["ci"], S["er"], nfc, d2)
    Li = np.zeros_like(A)
    for i in range(nfc):
        Li[i * d2:(i + 1) * d2, i * d2:(i + 1) * d2] = g["Linv"][i]
    Hs = dense_blocks(g["Hs"], S["rp"], S["ci"], S["er"], nfc, d2)
    assert np.abs(Hs - Li @ A @ Li.T).max() < 1e-12 * np.abs(Hs).max()
    assert np.abs(A - A.T).max() < 1e-12 * np.abs(A).max()


def test_zero_head_is_first_order_factor(sysk1):
    S = sysk1
    s = OGN.Shape(S["d2"], hidden=8, layers=2)
    th = OGN.init_params(s, seed=1)
    N, beta, _ = OGN.forward(th, s, S["g"], S["rp"], S["ci"], S["er"], S["ex"].ftype)
    ft = S["ex"].ftype
    low = (S["ci"] < S["er"]) & (ft[S["er"]] != 1) & (ft[S["ci"]] != 1)
    assert np.array_equal(N[low], -S["g"]["Hs"][low])
    assert not N[~low].any()
    assert not beta.any()  # B = I
    assert np.array_equal(OGN.block_scale(beta, S["d2"]), np.broadcast_to(np.eye(S["d2"]), (S["ex"].nfc, S["d2"], S["d2"])))


def _dense_G(N, beta, S):
    nfc, d2 = S["ex"].nfc, S["d2"]
    n = nfc * d2
    Bm = OGN.block_scale(beta, d2)
    Bd = np.zeros((n, n))
    for i in range(nfc):
        Bd[i * d2:(i + 1) * d2, i * d2:(i + 1) * d2] = Bm[i]
    return Bd, np.eye(n) + dense_blocks(N, S["rp"], S["ci"], S["er"], nfc, d2)


def _random_heads(S, s, seed):
    rng = np.random.default_rng(seed)
    th = OGN.init_params(s, seed=seed)
    th += 0.05 * rng.standard_normal(th.size)
    N, beta, _ = OGN.forward(th, s, S["g"], S["rp"], S["ci"], S["er"], S["ex"].ftype)
    return N, beta


def test_kaporin_loss_with_unit_probes(sysk1):
    """Unit probes make T the exact trace: T = tr(G Hs G^T) / n^2.  The loss is then
    log T - (1/n) log(det(G Hs G^T) / det(Hs)) = log T - (2/n) log det G, with det G by a
    dense LU (slogdet) of the product G = B (I + N), and the gradients are those of the dense
    formula d tr(G Hs G^T) / dG = 2 G Hs."""
    S = sysk1
    s = OGN.Shape(S["d2"], hidden=8, layers=2)
    N, beta = _random_heads(S, s, 3)
    nfc, d2 = S["ex"].nfc, S["d2"]
    n = nfc * d2
    assert beta[S["ex"].ftype != 1].any() and not beta[S["ex"].ftype == 1].any()
    Z = np.eye(n).reshape(n, nfc, d2)
    loss, dN, dbeta = OGN.kaporin_loss(N, beta, S["g"]["Hs"], S["rp"], S["ci"], S["er"], Z)
    Bd, U = _dense_G(N, beta, S)
    G = Bd @ U
    Hs = dense_blocks(S["g"]["Hs"], S["rp"], S["ci"], S["er"], nfc, d2)
    A = G @ Hs @ G.T
    T = np.trace(A) / (n * n)
    ld = 2.0 * np.linalg.slogdet(G)[1]
    assert abs(loss - (np.log(T) - ld / n)) < 1e-11
    dG = 2.0 * G @ Hs / (n * n)                 # dT/dG
    dU = Bd.T @ dG                              # dT/d(I + N)
    dB = dG @ U.T                               # dT/dB
    low = S["ci"] < S["er"]
    for e in np.where(low)[0][:40]:
        i, j = S["er"][e], S["ci"][e]
        ref = dU[i * d2:(i + 1) * d2, j * d2:(j + 1) * d2] / T
        assert np.abs(dN[e] - ref).max() < 1e-10 * np.abs(dU / T).max()
    assert not dN[~low].any()
    Bm = OGN.block_scale(beta, d2)
    for i in range(nfc):
        blk = dB[i * d2:(i + 1) * d2, i * d2:(i + 1) * d2] / T
        for a in range(d2):
            ref = blk[a, a] * Bm[i, a, a] - 2.0 / n
            assert abs(dbeta[i, a] - ref) < 1e-10 * max(1.0, abs(ref))
            for b in range(a):
                assert abs(dbeta[i, d2 + a * (a - 1) // 2 + b] - blk[a, b]) < 1e-10 * max(1.0, abs(blk[a, b]))


def test_optimal_block_scaling_is_stationary(sysk1):
    """For fixed N the Kaporin measure is minimised over the lower-triangular B_i by
    B_i = chol(A_ii)^{-1}, A = (I + N) Hs (I + N)^T (then B_i A_ii B_i^T = I): the gradient
    in beta vanishes there (unit probes, exact)."""
    S = sysk1
    s = OGN.Shape(S["d2"], hidden=8, layers=2)
    N, _ = _random_heads(S, s, 11)
    nfc, d2 = S["ex"].nfc, S["d2"]
    n = nfc * d2
    _, U = _dense_G(N, np.zeros((nfc, s.fb)), S)
    Hs = dense_blocks(S["g"]["Hs"], S["rp"], S["ci"], S["er"], nfc, d2)
    A = U @ Hs @ U.T
    beta = np.zeros((nfc, s.fb))
    for i in range(nfc):
        Bi = np.linalg.inv(np.linalg.cholesky(A[i * d2:(i + 1) * d2, i * d2:(i + 1) * d2]))
        for a in range(d2):
            beta[i, a] = np.log(Bi[a, a])
            for b in range(a):
                beta[i, d2 + a * (a - 1) // 2 + b] = Bi[a, b]
    beta[S["ex"].ftype == 1] = 0.0  # identity blocks there: chol(I)^{-1} = I
    Z = np.eye(n).reshape(n, nfc, d2)
    _, _, dbeta = OGN.kaporin_loss(N, beta, S["g"]["Hs"], S["rp"], S["ci"], S["er"], Z)
    assert np.abs(dbeta).max() < 1e-9
    # and a perturbation raises the loss
    l0 = OGN.kaporin_loss(N, beta, S["g"]["Hs"], S["rp"], S["ci"], S["er"], Z)[0]
    bp = beta + 0.05 * np.random.default_rng(2).standard_normal(beta.shape) * (S["ex"].ftype != 1)[:, None]
    assert OGN.kaporin_loss(N, bp, S["g"]["Hs"], S["rp"], S["ci"], S["er"], Z)[0] > l0


def test_backward_matches_central_differences(sysk1):
    S = sysk1
    s = OGN.Shape(S["d2"], hidden=6, layers=2)
    rng = np.random.default_rng(5)
    th = OGN.init_params(s, seed=4)
    th += 0.05 * rng.standard_normal(th.size)  # nonzero head and biases: every path active
    nfc, d2 = S["ex"].nfc, S["d2"]
    Z = rng.choice([-1.0, 1.0], size=(3, nfc, d2))
    args = (s, S["g"], S["rp"], S["ci"], S["er"], S["ex"].ftype, Z)
    loss, grad, _, _ = OGN.loss_and_grad(th, *args)
    offs = np.cumsum([0] + [int(np.prod(sh)) for _, sh in OGN.param_layout(s)])
    idx = np.concatenate([rng.choice(np.arange(a, b), size=min(4, b - a), replace=False)
                          for a, b in zip(offs[:-1], offs[1:])])
    eps = 1e-6
    for k in idx:
        tp, tm = th.copy(), th.copy()
        tp[k] += eps
        tm[k] -= eps
        fd = (OGN.loss_and_grad(tp, *args)[0] - OGN.loss_and_grad(tm, *args)[0]) / (2 * eps)
        assert abs(fd - grad[k]) <= 1e-6 * max(1.0, abs(grad).max()), (k, fd, grad[k])


def test_preconditioner_is_spd(sysk1):
    S = sysk1
    s = OGN.Shape(S["d2"], hidden=8, layers=2)
    th = OGN.init_params(s, seed=7)
    th += 0.1 * np.random.default_rng(8).standard_normal(th.size)
    N, beta, _ = OGN.forward(th, s, S["g"], S["rp"], S["ci"], S["er"], S["ex"].ftype)
    assert beta.any()
    nfc, d2 = S["ex"].nfc, S["d2"]
    n = nfc * d2
    Minv = np.stack([OGN.preconditioner_apply(N, beta, S["g"]["Linv"], e.reshape(nfc, d2), S["rp"], S["ci"],
                                              S["er"]).ravel() for e in np.eye(n)], 1)
    # the definition M^{-1} = L^{-T} G^T G L^{-1} written densely
    Bd, U = _dense_G(N, beta, S)
    Li = np.zeros((n, n))
    for i in range(nfc):
        Li[i * d2:(i + 1) * d2, i * d2:(i + 1) * d2] = S["g"]["Linv"][i]
    G = Bd @ U
    assert np.abs(Minv - Li.T @ G.T @ G @ Li).max() < 1e-12 * np.abs(Minv).max()
    assert np.abs(Minv - Minv.T).max() < 1e-12 * np.abs(Minv).max()
    assert np.linalg.eigvalsh(0.5 * (Minv + Minv.T)).min() > 0
