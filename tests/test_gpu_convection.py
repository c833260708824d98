"""GPU parity of the convection-diffusion HDG (Section 9, "Matrices for convection-diffusion
problems") against the oracle through the C ABI: the element face points, the local matrices
C^K, Cf^K and X = A1^{-1} [A2 | Af], the assembled non-symmetric H and F (every face
orientation, a persistent loop that iterates), the GMRES solution against the oracle's
sparse LU, exactness for polynomial data with an affine beta, and beta = 0 against the
diffusion condensation."""
import numpy as np
import pytest
import torch

from hdg_inputs import (convection_polynomial_problem, convection_sin_problem, kuhn_mesh, manufactured_sin_xyz,
                        permute_element_vertices)
from oracle import basis, convection as OC
from _gpu_helpers import OG, OL, bsr_to_csr, csr_rel, gpu_system, oracle_expand, rel

pytestmark = pytest.mark.gpu
TOL = 1e-12
MIXED = dict(dirichlet_sides=("x0", "x1", "z0"), neumann_sides=("y0", "y1", "z1"))


def _perm(n, seed, jitter=0.15):
    return permute_element_vertices(kuhn_mesh(n, jitter=jitter, seed=seed, **MIXED), seed=seed)


def _zero_beta(p):
    p.beta = lambda x, y, z: (0.0 * x, 0.0 * x, 0.0 * x)
    return p


def test_elem_face_points_match_oracle():
    from paper_1305_1489_amd import _lib as L
    m = _perm(2, 5)
    for k in (0, 3):
        S = gpu_system(m, k, convection_sin_problem())
        y = L.hdg_elem_face_qp_coords(S.disc, S.mesh).cpu().numpy()
        ex = oracle_expand(m)
        ref = OC.element_face_points(ex, np.arange(ex.nelt), OL.rules(k))
        assert np.abs(y - ref).max() < 1e-15 * max(1.0, np.abs(ref).max())


@pytest.mark.parametrize("k", [0, 1, 2, 3])
def test_cd_local_matrices_match_oracle(k):
    from paper_1305_1489_amd import _lib as L
    m = _perm(2, 20 + k)
    pb = convection_sin_problem(beta_scale=2.0)
    print(f"cd local k={k}", flush=True)
    S = gpu_system(m, k, pb)
    bv, bf = S.convection_fields()
    ex = oracle_expand(m)
    elems = np.arange(ex.nelt)
    Cg, Cfg, Xg = L.hdg_export_local_cd(S.disc, S.mesh, S.kappa, S.c, S.f, bv, bf, S.tau, elems, want_x=True)
    C, Cf = OC.condense(ex, pb, k)
    A1, A2, Af, A3, _ = OC.cd_matrices(ex, pb, OL.rules(k))
    X = np.linalg.solve(A1, np.concatenate([A2, Af[:, :, None]], axis=2))
    assert rel(Cg.cpu().numpy(), C) < TOL
    assert rel(Cfg.cpu().numpy(), Cf) < TOL
    assert rel(Xg.cpu().numpy().reshape(X.shape), X) < TOL
    # the trace matrix of a convection problem is not symmetric
    assert np.abs(C - C.transpose(0, 2, 1)).max() > 1e-6 * np.abs(C).max()


@pytest.mark.parametrize("k,n", [(0, 3), (1, 3), (2, 3), (3, 3), (1, 8), (3, 8)])
def test_cd_system_matches_oracle(k, n):
    """n = 8 (3072 elements) makes the persistent grid iterate."""
    m = _perm(n, 40 + k, jitter=0.1)
    pb = convection_sin_problem(beta_scale=1.5)
    print(f"cd system k={k} n={n}", flush=True)
    S = gpu_system(m, k, pb)
    S.H.fill_(float("nan"))
    S.F.fill_(float("nan"))
    S.assemble_cd()
    torch.cuda.synchronize()
    ex = oracle_expand(m)
    C, Cf = OC.condense(ex, pb, k)
    H, F = OG.assemble(ex, k, C, Cf)
    Hg, _ = bsr_to_csr(S)
    assert csr_rel(Hg, H) < TOL
    assert rel(S.F.cpu().numpy().ravel(), F) < TOL


@pytest.mark.parametrize("k,solver", [(1, "gmres"), (2, "gmres"), (3, "gmres"), (1, "bicgstab"), (3, "bicgstab")])
def test_cd_solution_matches_oracle(k, solver):
    """Condensation, boundary data, GMRES or BiCGStab, and the reconstruction against the
    oracle's sparse-LU solution of the same discrete problem."""
    m = _perm(3, 60 + k)
    pb = convection_sin_problem(beta_scale=2.0)
    print(f"cd solve k={k} {solver}", flush=True)
    S = gpu_system(m, k, pb)
    r = S.run_cd(rtol=1e-13, restart=40, solver=solver)
    assert r["info"]["rel_residual"] <= 1e-13
    ex = oracle_expand(m)
    ref = OC.solve_problem(ex, pb, k)
    assert rel(S.uhat.cpu().numpy(), ref["uhat"]) < 1e-10
    assert rel(r["q"].cpu().numpy(), ref["q"]) < 1e-10
    assert rel(r["u"].cpu().numpy(), ref["u"]) < 1e-10


@pytest.mark.parametrize("k", [0, 1, 2, 3])
def test_cd_polynomial_exactness_gpu(k):
    """u in P_k, constant kappa and c, affine beta (exact quadrature): q_h = q, u_h = u and
    uhat = u through the whole GPU chain."""
    m = _perm(2, 80 + k)
    pb = convection_polynomial_problem(k, seed=k, kappa=1.3, c=0.7, beta_scale=1.5)
    S = gpu_system(m, k, pb)
    r = S.run_cd(rtol=1e-14, restart=40)
    ex = oracle_expand(m)
    err = OG.errors(ex, pb, k, r["q"].cpu().numpy(), r["u"].cpu().numpy(), S.uhat.cpu().numpy())
    assert err["e_q"] < 1e-10 and err["e_u"] < 1e-10 and err["e_uhat"] < 1e-10, err


@pytest.mark.parametrize("k", [1, 3])
def test_cd_beta_zero_is_diffusion(k):
    """beta = 0: the convection-diffusion condensation equals the diffusion one."""
    m = _perm(3, 90 + k)
    pb = _zero_beta(manufactured_sin_xyz("c1", "c1"))
    S = gpu_system(m, k, pb)
    S.assemble()
    torch.cuda.synchronize()
    H0, F0 = S.H.clone(), S.F.clone()
    S.assemble_cd()
    torch.cuda.synchronize()
    assert rel(S.H.cpu().numpy(), H0.cpu().numpy()) < 1e-13
    assert rel(S.F.cpu().numpy(), F0.cpu().numpy()) < 1e-13


def test_bicgstab_polynomial_exactness_and_errors():
    """BiCGStab through the whole chain on polynomial data (exact), and its argument checks."""
    from paper_1305_1489_amd import _lib as L
    k = 2
    m = _perm(2, 83)
    pb = convection_polynomial_problem(k, seed=k, kappa=1.3, c=0.7, beta_scale=1.5)
    S = gpu_system(m, k, pb)
    r = S.run_cd(rtol=1e-14, solver="bicgstab")
    ex = oracle_expand(m)
    err = OG.errors(ex, pb, k, r["q"].cpu().numpy(), r["u"].cpu().numpy(), S.uhat.cpu().numpy())
    assert err["e_q"] < 1e-10 and err["e_u"] < 1e-10 and err["e_uhat"] < 1e-10, err
    with pytest.raises(L.HdgError) as e:
        L.hdg_solve_bicgstab(S.disc, S.mesh, S.H, S.F, S.uhat, check_every=0)
    assert e.value.name == "HDG_ERR_INVALID_ARG"
    out = L.hdg_solve_bicgstab(S.disc, S.mesh, S.H, S.F, S.uhat, rtol=1e-300, max_iter=3, check_every=1,
                               raise_on_fail=False)
    assert L.STATUS[out["status"]] == "HDG_ERR_NOT_CONVERGED"


def test_gmres_on_symmetric_system_matches_pcg():
    """On the diffusion system GMRES and PCG reach the same solution."""
    from paper_1305_1489_amd import _lib as L
    m = _perm(4, 7)
    S = gpu_system(m, 2, manufactured_sin_xyz("c1", "c1"))
    S.assemble()
    S.boundary()
    b = S.F.clone()
    u0 = S.uhat.clone()
    S.solve(rtol=1e-13)
    x_cg = S.uhat.clone()
    S.uhat.copy_(u0)
    info = L.hdg_solve_gmres(S.disc, S.mesh, S.H, b, S.uhat, rtol=1e-13, restart=30)
    assert info["rel_residual"] <= 1e-13
    assert rel(S.uhat.cpu().numpy(), x_cg.cpu().numpy()) < 1e-10


def test_cd_errors():
    from paper_1305_1489_amd import _lib as L
    m = _perm(2, 3)
    S = gpu_system(m, 4, convection_sin_problem())
    bv, bf = S.convection_fields()
    with pytest.raises(L.HdgError) as e:
        L.hdg_assemble_condense_cd(S.disc, S.mesh, S.kappa, S.c, S.f, bv, bf, S.tau, S.H, S.F)
    assert e.value.name == "HDG_ERR_UNSUPPORTED_DEGREE"
    S = gpu_system(m, 1, convection_sin_problem())
    S.assemble_cd()
    S.boundary()
    for bad in (0, 65):
        with pytest.raises(L.HdgError) as e:
            L.hdg_solve_gmres(S.disc, S.mesh, S.H, S.F, S.uhat, restart=bad)
        assert e.value.name == "HDG_ERR_INVALID_ARG"
    out = L.hdg_solve_gmres(S.disc, S.mesh, S.H, S.F, S.uhat, rtol=1e-14, max_iter=2, restart=10,
                            raise_on_fail=False)
    assert out["status"] == 10 and out["iterations"] == 2  # HDG_ERR_NOT_CONVERGED, iterate still written
    import ctypes as C
    small = torch.empty(8, dtype=torch.uint8, device="cuda")
    info = L.hdg_solve_info()
    code = L.lib().hdg_solve_gmres(S.disc.handle, C.byref(S.mesh.struct), L._ptr(S.H), L._ptr(S.F), L._ptr(S.uhat),
                                   C.c_double(1e-10), C.c_int(100), C.c_int(10), C.byref(info), L._ptr(small),
                                   C.c_size_t(8), L._stream())
    assert L.STATUS[code] == "HDG_ERR_WORKSPACE"
