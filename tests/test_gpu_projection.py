"""GPU parity of the local projections and the superconvergence diagnostics (Section 9;
eq 9.12, 9.13, 10.2) against the oracle, through the C ABI.

The oracle solves the paper's square 4 d3 system per element with quadrature mass
matrices; the library uses the orthonormal basis (unit mass |K| I) and the factorisation of
the face equations through the inverse top-mode blocks of DP_{mu,l}.  Both take the fields at
the same quadrature points (the library's own, evaluated by the caller)."""
import math

import numpy as np
import pytest
import torch

from hdg_inputs import kuhn_mesh, manufactured_sin_xyz, permute_element_vertices, polynomial_problem
from oracle import local as OLL, projection as PR
from _gpu_helpers import OG, gpu_system, oracle_expand, rel

pytestmark = pytest.mark.gpu
TOL = 1e-12
MIXED = dict(dirichlet_sides=("x0", "x1"), neumann_sides=("y0", "y1", "z0", "z1"))


def _fields_at_points(S, pb):
    """(q, u) at the volume points [nelt][nqd][4] and at the points of every face
    [nfc][nqd2][4], and u alone at both, evaluated with torch on the device."""
    from paper_1305_1489_amd import _lib as L
    xv = S.qp
    faces = torch.arange(S.mesh.nfc, dtype=torch.int32, device="cuda")
    xf = L.hdg_face_qp_coords(S.disc, S.mesh, faces)
    out = []
    for x in (xv, xf):
        X, Y, Z = x[..., 0], x[..., 1], x[..., 2]
        q = [c * torch.ones_like(X) for c in pb.q(X, Y, Z)]
        u = pb.u(X, Y, Z) * torch.ones_like(X)
        out.append(torch.stack(q + [u], dim=-1).contiguous())
    return out[0], out[1]


@pytest.mark.parametrize("k", [0, 1, 2, 3, 4])
def test_projections_match_oracle(k):
    from paper_1305_1489_amd import _lib as L
    m = permute_element_vertices(kuhn_mesh(3, jitter=0.15, seed=20 + k, **MIXED), seed=20 + k)
    pb = manufactured_sin_xyz("c1", "c1")
    pb.tau = np.random.default_rng(30 + k).uniform(0.3, 2.0, size=(m.nelt, 4))
    if k == 2:  # tau on one face only (Section 1 allows it; W stays invertible)
        t = np.zeros_like(pb.tau)
        t[np.arange(m.nelt), np.random.default_rng(1).integers(0, 4, m.nelt)] = 1.3
        pb.tau = t
    print(f"projections k={k}", flush=True)
    S = gpu_system(m, k, pb)
    quv, quf = _fields_at_points(S, pb)
    Pq, Pu = L.hdg_project_hdg(S.disc, S.mesh, S.tau, quv, quf)
    Pt = L.hdg_project_trace(S.disc, S.mesh, quf[..., 3].contiguous())
    torch.cuda.synchronize()
    ex = oracle_expand(m)
    R = OLL.rules(k)
    Pq_o, Pu_o = PR.hdg_projection(ex, pb.q, pb.u, pb.tau, R)
    Pt_o = PR.trace_projection(ex, pb.u, R)
    assert rel(Pq.cpu().numpy(), Pq_o) < TOL
    assert rel(Pu.cpu().numpy(), Pu_o) < TOL
    assert rel(Pt.cpu().numpy()[:, 0], Pt_o) < TOL
    # four fields at once give the same moments as one at a time
    Pt4 = L.hdg_project_trace(S.disc, S.mesh, quf)
    torch.cuda.synchronize()
    assert torch.equal(Pt4[:, 3], Pt[:, 0])


@pytest.mark.parametrize("k", [1, 3])
def test_superconvergence_norms_match_oracle(k):
    """The squared norms on the same inputs (the oracle's own projections and solution) as
    the oracle's eps_u, eps_uhat with the same quadrature rule."""
    from paper_1305_1489_amd import _lib as L
    m = kuhn_mesh(3, jitter=0.1, seed=5, **MIXED)
    pb = manufactured_sin_xyz("c1", "c1")
    ex = oracle_expand(m)
    out = OG.solve_problem(ex, pb, k, with_post=False)
    R = OLL.rules(k)
    Pq_o, Pu_o = PR.hdg_projection(ex, pb.q, pb.u, pb.tau, R)
    Pt_o = PR.trace_projection(ex, pb.u, R)
    ref = PR.superconvergence_errors(ex, pb.u, k, Pu_o, out["u"], Pt_o, out["uhat"], nq=k + 2)
    S = gpu_system(m, k, pb)
    quv, quf = _fields_at_points(S, pb)
    dev = lambda a: torch.as_tensor(np.ascontiguousarray(a), device="cuda")
    nrm = L.hdg_superconvergence_norms(S.disc, S.mesh, dev(Pu_o), dev(out["u"]), dev(Pt_o), dev(out["uhat"]),
                                       quv[..., 3].contiguous(), quf[..., 3].contiguous())
    n2 = L.hdg_superconvergence_norms(S.disc, S.mesh, dev(Pu_o), dev(out["u"]), dev(Pt_o), dev(out["uhat"]),
                                      quv[..., 3].contiguous(), quf[..., 3].contiguous())
    torch.cuda.synchronize()
    a = nrm.cpu().numpy()
    assert torch.equal(nrm, n2)  # fixed-order reductions
    assert abs(math.sqrt(a[0] / a[1]) - ref["eps_u"]) <= TOL * ref["eps_u"] * 10
    assert abs(math.sqrt(a[2] / a[3]) - ref["eps_uhat"]) <= TOL * ref["eps_uhat"] * 10


@pytest.mark.parametrize("k", [1, 2])
def test_gpu_superconvergence_rates(k):
    """The whole chain on the GPU (condensation, solve, reconstruction, projections, norms)
    reproduces the k + 2 superconvergence of eq 10.2 on n = 2, 4, 8 (Tables 2-3)."""
    from paper_1305_1489_amd import _lib as L
    pb = manufactured_sin_xyz("c1", "c1")
    errs = []
    for n in (2, 4, 8):
        m = kuhn_mesh(n, **MIXED)
        print(f"superconvergence k={k} n={n}", flush=True)
        S = gpu_system(m, k, pb)
        r = S.run(rtol=1e-13)
        quv, quf = _fields_at_points(S, pb)
        Pq, Pu = L.hdg_project_hdg(S.disc, S.mesh, S.tau, quv, quf)
        Pt = L.hdg_project_trace(S.disc, S.mesh, quf[..., 3].contiguous())[:, 0].contiguous()
        a = L.hdg_superconvergence_norms(S.disc, S.mesh, Pu, r["u"], Pt, S.uhat, quv[..., 3].contiguous(),
                                         quf[..., 3].contiguous()).cpu().numpy()
        errs.append((math.sqrt(a[0] / a[1]), math.sqrt(a[2] / a[3])))
    for j in range(2):
        rate = math.log2(errs[1][j] / errs[2][j])
        assert rate >= k + 2 - 0.35, (j, errs, rate)
