"""GPU parity of the hybridized BDM element (Section 9, "BDM") against the oracle through the
C ABI: the trace system H, F (eq 6.5 with the BDM local solvers), the reconstruction on the
oracle's trace solution, and the mixed method's polynomial exactness through the GPU solver,
on meshes with every face orientation and with persistent loops that iterate."""
import numpy as np
import pytest
import torch

from hdg_inputs import kuhn_mesh, manufactured_sin_xyz, permute_element_vertices, polynomial_problem
from hdg_inputs.mesh import SIDES
from oracle import basis, bdm
from _gpu_helpers import OG, bsr_to_csr, csr_rel, gpu_system, make_mesh, oracle_expand, rel

pytestmark = pytest.mark.gpu
TOL = 1e-12
MIXED = dict(dirichlet_sides=("x0", "x1", "z0"), neumann_sides=("y0", "y1", "z1"))


def _perm(n, seed):
    return permute_element_vertices(kuhn_mesh(n, jitter=0.15, seed=seed, **MIXED), seed=seed)


@pytest.mark.parametrize("k,n,wpc", [(1, 3, 4), (2, 3, 4), (3, 3, 4), (1, 6, 1), (3, 6, 1)])
def test_bdm_system_and_recovery_match_oracle(k, n, wpc):
    from paper_1305_1489_amd import _lib as L
    m = _perm(n, 60 + k)
    pb = manufactured_sin_xyz("c1", "c1")
    print(f"bdm k={k} n={n} workgroups/CU={wpc}", flush=True)
    ex = oracle_expand(m)
    out = bdm.solve_problem(ex, pb, k)
    S = gpu_system(m, k, pb)
    saved = L.hdg_get_launch_config(k)
    try:
        L.hdg_set_launch_config(k, wpc, 1, 1)
        for t in (S.H, S.F, S.factors):
            t.fill_(float("nan"))
        S.assemble(method="bdm")
        torch.cuda.synchronize()
    finally:
        L.hdg_set_launch_config(k, saved["workgroups_per_cu"], saved["xcd_remap"], saved["waves_per_element"])
    Hg, _ = bsr_to_csr(S)
    assert csr_rel(Hg, out["H"]) < TOL
    assert rel(S.F.cpu().numpy().ravel(), out["F"]) < TOL
    assert (Hg - Hg.T).count_nonzero() == 0 or abs(Hg - Hg.T).max() == 0
    S.uhat.copy_(torch.as_tensor(out["uhat"]))
    q, u, _ = S.recover(postprocess=False)
    torch.cuda.synchronize()
    assert rel(q.cpu().numpy(), out["q"]) < TOL
    assert rel(u.cpu().numpy(), out["u"]) < TOL
    low = basis.dim3(k) - basis.dim2(k)
    assert not u[:, low:].any()  # u in P_{k-1}(K)


@pytest.mark.parametrize("k", [1, 2, 3])
def test_bdm_polynomial_exactness_gpu(k):
    """Constant kappa and c, u in P_k: q_h = q and uhat = u on the faces through the whole GPU
    chain (condensation, boundary data, PCG, reconstruction), u_h = the oracle's."""
    m = _perm(3, 80 + k)
    pb = polynomial_problem(k, seed=k, kappa=1.7, c=0.6)
    S = gpu_system(m, k, pb)
    r = S.run(rtol=1e-13, method="bdm")
    assert r["info"]["rel_residual"] <= 1e-13
    ex = oracle_expand(m)
    err = OG.errors(ex, pb, k, r["q"].cpu().numpy(), r["u"].cpu().numpy(), S.uhat.cpu().numpy())
    assert err["e_q"] < 1e-11 and err["e_uhat"] < 1e-11, err
    ref = bdm.solve_problem(ex, pb, k)
    assert rel(r["u"].cpu().numpy(), ref["u"]) < 1e-10


def test_bdm_rejections():
    from paper_1305_1489_amd import _lib as L
    m = make_mesh(2)
    for k in (0, 4):
        S = gpu_system(m, k, manufactured_sin_xyz("c1", "c1"))
        with pytest.raises(L.HdgError) as e:
            L.hdg_assemble_condense_bdm(S.disc, S.mesh, S.kappa, S.c, S.f, S.H, S.F, S.factors)
        assert e.value.name == "HDG_ERR_UNSUPPORTED_DEGREE"
    mn = make_mesh(2, dirichlet=(), neumann=SIDES)
    S = gpu_system(mn, 2, polynomial_problem(1, kappa=1.0, c=0.0))
    with pytest.raises(L.HdgError) as e:
        L.hdg_assemble_condense_bdm(S.disc, S.mesh, S.kappa, S.c, S.f, S.H, S.F, S.factors)
    assert e.value.name == "HDG_ERR_SINGULAR"
