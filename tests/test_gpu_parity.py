"""GPU parity: the HIP path (through the C ABI) against the CPU oracle on the same seeded
inputs.  Integer index work is compared bit for bit; floating point to 1e-12 relative
(max |x - x_ref| / max |x_ref| per field), the bound the condensation targets in FP64."""
import numpy as np
import pytest
import torch

from hdg_inputs import manufactured_sin_xyz, polynomial_problem, manufactured_sin_pi
from hdg_inputs.fields import Problem
from _gpu_helpers import OG, OL, bsr_to_csr, gpu_system, make_mesh, oracle_expand, rel

pytestmark = pytest.mark.gpu
TOL = 1e-12

MIXED = dict(dirichlet=("x0", "x1"), neumann=("y0", "y1", "z0", "z1"))


def _problem_random_tau(m, seed=0, base=None):
    pb = base or manufactured_sin_xyz("c1", "c1")
    rng = np.random.default_rng(seed)
    pb.tau = rng.uniform(0.3, 2.0, size=(m.elements.shape[0], 4))
    return pb


# ----------------------------------------------------------------------------- mesh expansion
@pytest.mark.parametrize("n,jit,bc", [(1, 0.0, {}), (2, 0.1, MIXED), (5, 0.15, MIXED), (8, 0.0, {})])
def test_mesh_expansion_bit_exact(n, jit, bc):
    from paper_1305_1489_amd import _lib as L
    m = make_mesh(n, jitter=jit, seed=3, **bc)
    print(f"mesh expansion n={n}", flush=True)
    M = L.hdg_mesh_expand(m.coordinates, m.elements, m.dirichlet, m.neumann)
    torch.cuda.synchronize()
    ex = oracle_expand(m)
    assert M.nfc == ex.nfc
    assert np.array_equal(M.faces.cpu().numpy(), ex.faces)
    assert np.array_equal(M.ftype.cpu().numpy(), ex.ftype)
    assert np.array_equal(M.facebyele.cpu().numpy(), ex.facebyele)
    assert np.array_equal(M.perm.cpu().numpy(), ex.perm)
    if M.ndir:
        assert np.array_equal(M.dirfaces[: M.ndir].cpu().numpy(), ex.dirfaces)
    if M.nneu:
        assert np.array_equal(M.neufaces[: M.nneu].cpu().numpy(), ex.neufaces)
    assert rel(M.volume.cpu().numpy(), ex.volume) < 1e-15
    assert rel(M.area.cpu().numpy(), ex.area) < 1e-15
    assert rel(M.normals.cpu().numpy(), ex.normals) < 1e-15
    # block pattern: row f holds f and the faces sharing an element with f, sorted
    rp, ci = M.row_ptr.cpu().numpy(), M.col_idx.cpu().numpy()
    assert rp[-1] == ex.nfc + 12 * ex.nelt
    nb = {f: {f} for f in range(ex.nfc)}
    for K in range(ex.nelt):
        for a in ex.facebyele[K]:
            nb[a] |= set(ex.facebyele[K])
    for f in range(ex.nfc):
        assert list(ci[rp[f]:rp[f + 1]]) == sorted(nb[f])
    slot = M.slot.cpu().numpy().reshape(-1, 4, 4)
    for K in range(ex.nelt):
        for a in range(4):
            for b in range(4):
                assert ci[slot[K, a, b]] == ex.facebyele[K, b]
                assert rp[ex.facebyele[K, a]] <= slot[K, a, b] < rp[ex.facebyele[K, a] + 1]


def test_mesh_errors():
    from paper_1305_1489_amd import _lib as L
    m = make_mesh(2)
    cases = [
        (m.coordinates, m.elements[:, [0, 2, 1, 3]], m.dirichlet, m.neumann, "HDG_ERR_MESH_ORIENTATION"),
        (m.coordinates, m.elements, m.dirichlet[1:], m.neumann, "HDG_ERR_INVALID_ARG"),
        (m.coordinates, m.elements, m.dirichlet[:-2], m.neumann, "HDG_ERR_BOUNDARY_UNLISTED"),
    ]
    bad = m.dirichlet.copy()
    bad[0] = bad[0][[0, 2, 1]]
    cases.append((m.coordinates, m.elements, bad, m.neumann, "HDG_ERR_MESH_ORIENTATION"))
    dup = m.dirichlet.copy()
    dup[1] = dup[0]
    cases.append((m.coordinates, m.elements, dup, m.neumann, "HDG_ERR_BOUNDARY_INVALID"))
    for X, T, D, N, want in cases:
        with pytest.raises(L.HdgError) as e:
            L.hdg_mesh_expand(X, T, D, N)
        assert e.value.name == want, (want, str(e.value))


# ----------------------------------------------------------------------------- local blocks
@pytest.mark.parametrize("k", [0, 1, 2, 3, 4])
def test_local_blocks_parity(k):
    from paper_1305_1489_amd import _lib as L
    m = make_mesh(2, jitter=0.15, seed=k, **MIXED)
    pb = _problem_random_tau(m, seed=k)
    print(f"local blocks k={k}", flush=True)
    S = gpu_system(m, k, pb)
    elems = np.arange(S.mesh.nelt)
    Cg, Cfg = L.hdg_export_local(S.disc, S.mesh, S.kappa, S.c, S.f, S.tau, elems)
    ex = oracle_expand(m)
    b = OL.local_blocks(ex, pb, OL.rules(k))
    C, Cf = OL.condense(b)
    assert rel(Cg.cpu().numpy(), C) < TOL
    assert rel(Cfg.cpu().numpy(), Cf) < TOL
    Cn = Cg.cpu().numpy()
    assert np.array_equal(Cn, Cn.transpose(0, 2, 1))  # exact symmetry


# ----------------------------------------------------------------------------- global system
@pytest.mark.parametrize("k,n,jit", [(1, 2, 0.0), (2, 3, 0.15), (3, 3, 0.1), (4, 2, 0.1)])
def test_global_system_and_boundary_parity(k, n, jit):
    m = make_mesh(n, jitter=jit, seed=7, **MIXED)
    pb = _problem_random_tau(m, seed=n)
    print(f"global system k={k} n={n}", flush=True)
    S = gpu_system(m, k, pb)
    S.assemble()
    torch.cuda.synchronize()
    ex = oracle_expand(m)
    R = OL.rules(k)
    C, Cf = OL.condense_all(ex, pb, R)
    H, F = OG.assemble(ex, k, C, Cf)
    Hg, _ = bsr_to_csr(S)
    assert rel(Hg.toarray(), H.toarray()) < TOL
    assert rel(S.F.cpu().numpy().ravel(), F) < TOL
    assert (Hg - Hg.T).count_nonzero() == 0 or abs(Hg - Hg.T).max() == 0
    # boundary conditions and elimination
    S.boundary()
    torch.cuda.synchronize()
    uD = OG.dirichlet_data(ex, pb, R)
    GN = OG.neumann_load(ex, pb, R)
    b = OG.rhs_with_neumann(ex, k, F, GN)
    d2 = S.disc.d2
    uh = np.zeros((ex.nfc, d2))
    uh[ex.dirfaces] = uD
    isD = np.repeat(np.isin(np.arange(ex.nfc), ex.dirfaces), d2)
    red = b - H[:, isD] @ uh.ravel()[isD]
    red[isD] = uh.ravel()[isD]
    assert rel(S.F.cpu().numpy().ravel(), red) < TOL
    assert rel(S.uhat.cpu().numpy(), uh) < TOL
    Hm, _ = bsr_to_csr(S)
    Href = H.toarray()
    Href[isD, :] = 0
    Href[:, isD] = 0
    Href[isD, isD] = 1
    assert rel(Hm.toarray(), Href) < TOL


def test_determinism_bitwise():
    m = make_mesh(4, jitter=0.15, seed=1, **MIXED)
    pb = manufactured_sin_xyz("c1", "c1")
    S = gpu_system(m, 2, pb)
    S.assemble()
    H1, F1 = S.H.clone(), S.F.clone()
    S.assemble()
    torch.cuda.synchronize()
    assert torch.equal(H1, S.H) and torch.equal(F1, S.F)


# ----------------------------------------------------------------------------- recovery
@pytest.mark.parametrize("k", [0, 1, 2, 3, 4])
def test_recovery_parity_same_uhat(k):
    """q, u, u* from the oracle's own trace solution fed to the library.  162 elements:
    the postprocess works on groups of four, so the last group is ragged (two elements)."""
    m = make_mesh(3, jitter=0.1, seed=k, **MIXED)
    pb = _problem_random_tau(m, seed=10 + k)
    print(f"recovery k={k}", flush=True)
    ex = oracle_expand(m)
    out = OG.solve_problem(ex, pb, k)
    S = gpu_system(m, k, pb)
    S.assemble()
    S.uhat.copy_(torch.as_tensor(out["uhat"]))
    q, u, us = S.recover()
    torch.cuda.synchronize()
    assert rel(q.cpu().numpy(), out["q"]) < TOL
    assert rel(u.cpu().numpy(), out["u"]) < TOL
    assert rel(us.cpu().numpy(), out["ustar"]) < TOL


@pytest.mark.parametrize("k", [0, 2, 4])
def test_postprocess_entry_on_oracle_fields(k):
    """hdg_postprocess alone, fed the oracle's q and u (eq 9.11), on a ragged element count."""
    from paper_1305_1489_amd import _lib as L
    m = make_mesh(3, jitter=0.12, seed=30 + k, **MIXED)
    pb = _problem_random_tau(m, seed=40 + k)
    print(f"postprocess k={k}", flush=True)
    out = OG.solve_problem(oracle_expand(m), pb, k)
    S = gpu_system(m, k, pb)
    q = torch.as_tensor(out["q"], device="cuda").contiguous()
    u = torch.as_tensor(out["u"], device="cuda").contiguous()
    us = L.hdg_postprocess(S.disc, S.mesh, S.kappa, S.tau, q, u)
    torch.cuda.synchronize()
    assert rel(us.cpu().numpy(), out["ustar"]) < TOL
    # with the factor store the geometry is read, not recomputed: the same bits
    S.assemble()
    us2 = L.hdg_postprocess(S.disc, S.mesh, S.kappa, S.tau, q, u, factors=S.factors)
    torch.cuda.synchronize()
    assert torch.equal(us2.view(torch.int64), us.view(torch.int64))


# ----------------------------------------------------------------------------- whole pipeline
@pytest.mark.parametrize("k", [0, 1, 2, 3, 4])
def test_polynomial_reproduction_gpu(k):
    """Exact polynomial solutions of degree <= k are reproduced by the HIP pipeline with the
    GPU solver (Section 8, last paragraph)."""
    m = make_mesh(3, jitter=0.15, seed=20 + k, dirichlet=("x0", "x1", "z0"), neumann=("y0", "y1", "z1"))
    pb = polynomial_problem(k, seed=k, kappa=2.0, c=1.0, c_linear=True)
    print(f"polynomial reproduction k={k}", flush=True)
    S = gpu_system(m, k, pb)
    r = S.run(rtol=1e-13)
    assert r["info"]["rel_residual"] <= 1e-13
    ex = oracle_expand(m)
    err = OG.errors(ex, pb, k, r["q"].cpu().numpy(), r["u"].cpu().numpy(), S.uhat.cpu().numpy(),
                    r["ustar"].cpu().numpy())
    assert err["e_u"] < 1e-11 and err["e_uhat"] < 1e-11 and err["e_star"] < 1e-11
    if k:
        assert err["e_q"] < 1e-11


def test_pipeline_small_config_against_oracle():
    """The 48-element all-Dirichlet workload end to end: same errors as the oracle."""
    m = make_mesh(2)
    pb = manufactured_sin_pi()
    S = gpu_system(m, 1, pb)
    r = S.run(rtol=1e-12)
    ex = oracle_expand(m)
    out = OG.solve_problem(ex, pb, 1)
    assert rel(S.uhat.cpu().numpy(), out["uhat"]) < 1e-10
    assert rel(r["u"].cpu().numpy(), out["u"]) < 1e-10
    assert rel(r["ustar"].cpu().numpy(), out["ustar"]) < 1e-10


def test_solver_true_residual_smooth():
    m = make_mesh(8, **MIXED)
    pb = manufactured_sin_xyz("c1", "c1")
    S = gpu_system(m, 2, pb)
    S.assemble()
    S.boundary()
    b = S.F.clone()
    info = S.solve(rtol=1e-10)
    Hc, _ = bsr_to_csr(S)
    x = S.uhat.cpu().numpy().ravel()
    bb = b.cpu().numpy().ravel()
    assert np.linalg.norm(bb - Hc @ x) <= 1e-10 * np.linalg.norm(bb) * 1.0001
    assert info["rel_residual"] <= 1e-10
    S.assemble()
    S.uhat.zero_()
    S.boundary()
    info32 = S.solve(rtol=1e-10, precision=1)
    x2 = S.uhat.cpu().numpy().ravel()
    assert np.linalg.norm(bb - Hc @ x2) <= 1e-10 * np.linalg.norm(bb) * 1.0001
