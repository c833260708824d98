"""Pins of the learned-preconditioner oracle (oracle/gnn.py).

The preconditioner family and its network are not in the paper, so nothing here is a
printed value.  Parity of the definitions is pinned instead:
  * the hand-written backward against central differences of the forward pass;
  * the probe loss and its N-gradient against dense linear algebra (exact with unit probes);
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
    N, _ = OGN.forward(th, s, S["g"], S["rp"], S["ci"], S["er"], S["ex"].ftype)
    ft = S["ex"].ftype
    low = (S["ci"] < S["er"]) & (ft[S["er"]] != 1) & (ft[S["ci"]] != 1)
    assert np.array_equal(N[low], -S["g"]["Hs"][low])
    assert not N[~low].any()


def test_trace_loss_with_unit_probes_is_the_trace(sysk1):
    S = sysk1
    s = OGN.Shape(S["d2"], hidden=8, layers=2)
    rng = np.random.default_rng(3)
    th = OGN.init_params(s, seed=2)
    th[-(s.fe * 3 * s.hidden + s.fe):] = 0.05 * rng.standard_normal(s.fe * 3 * s.hidden + s.fe)
    N, _ = OGN.forward(th, s, S["g"], S["rp"], S["ci"], S["er"], S["ex"].ftype)
    nfc, d2 = S["ex"].nfc, S["d2"]
    n = nfc * d2
    Z = np.eye(n).reshape(n, nfc, d2)
    loss, dN = OGN.trace_loss(N, S["g"]["Hs"], S["rp"], S["ci"], S["er"], Z)
    G = np.eye(n) + dense_blocks(N, S["rp"], S["ci"], S["er"], nfc, d2)
    Hs = dense_blocks(S["g"]["Hs"], S["rp"], S["ci"], S["er"], nfc, d2)
    assert abs(loss - np.trace(G @ Hs @ G.T) / (n * n)) < 1e-12 * abs(loss)
    # d tr(G Hs G^T) / dG = 2 G Hs, restricted to the strictly lower blocks
    Dg = 2.0 * G @ Hs / (n * n)
    low = S["ci"] < S["er"]
    for e in np.where(low)[0][:40]:
        i, j = S["er"][e], S["ci"][e]
        assert np.abs(dN[e] - Dg[i * d2:(i + 1) * d2, j * d2:(j + 1) * d2]).max() < 1e-12 * np.abs(Dg).max()
    assert not dN[~low].any()


def test_backward_matches_central_differences(sysk1):
    S = sysk1
    s = OGN.Shape(S["d2"], hidden=6, layers=2)
    rng = np.random.default_rng(5)
    th = OGN.init_params(s, seed=4)
    th += 0.05 * rng.standard_normal(th.size)  # nonzero head and biases: every path active
    nfc, d2 = S["ex"].nfc, S["d2"]
    Z = rng.choice([-1.0, 1.0], size=(3, nfc, d2))
    args = (s, S["g"], S["rp"], S["ci"], S["er"], S["ex"].ftype, Z)
    loss, grad, _ = OGN.loss_and_grad(th, *args)
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
    N, _ = OGN.forward(th, s, S["g"], S["rp"], S["ci"], S["er"], S["ex"].ftype)
    nfc, d2 = S["ex"].nfc, S["d2"]
    n = nfc * d2
    Minv = np.stack([OGN.preconditioner_apply(N, S["g"]["Linv"], e.reshape(nfc, d2), S["rp"], S["ci"],
                                              S["er"]).ravel() for e in np.eye(n)], 1)
    assert np.abs(Minv - Minv.T).max() < 1e-12 * np.abs(Minv).max()
    assert np.linalg.eigvalsh(0.5 * (Minv + Minv.T)).min() > 0
