"""Condensation with FP32 local factors and FP64 iterative refinement against the FP64 oracle.

The refinement stops once the correction is at most 1e-15 of the local solution X, so X
carries FP64-level error: about cond(A1) times the FP64 rounding of the residual.  The
bar is therefore the FP64 path's own, 1e-12 relative to the largest entry per field.
"""
import numpy as np
import pytest
import torch

from _gpu_helpers import OG, OL, bsr_to_csr, gpu_system, make_mesh, oracle_expand, rel
from test_gpu_parity import MIXED, _problem_random_tau

pytestmark = pytest.mark.gpu

TOL_IR = 1e-12


@pytest.mark.parametrize("k,n,jit", [(1, 3, 0.1), (2, 3, 0.15), (3, 3, 0.1), (3, 1, 0.0)])
def test_ir_condensation_and_recovery_match_oracle(k, n, jit):
    from paper_1305_1489_amd import _lib as L
    m = make_mesh(n, jitter=jit, seed=17 + k, **MIXED)
    pb = _problem_random_tau(m, seed=30 + k)
    print(f"ir k={k} n={n}", flush=True)
    S = gpu_system(m, k, pb)
    nelt = S.mesh.nelt
    X = torch.full((nelt, L.hdg_ir_store_len(S.disc)), float("nan"), dtype=torch.float64, device="cuda")
    sweeps = torch.zeros(nelt, dtype=torch.int32, device="cuda")
    S.H.fill_(float("nan"))
    L.hdg_assemble_condense_ir(S.disc, S.mesh, S.kappa, S.c, S.f, S.tau, S.H, S.F, X, 8, sweeps)
    torch.cuda.synchronize()
    ex = oracle_expand(m)
    R = OL.rules(k)
    C, Cf = OL.condense_all(ex, pb, R)
    H, F = OG.assemble(ex, k, C, Cf)
    Hg, _ = bsr_to_csr(S)
    eH = rel(Hg.toarray(), H.toarray())
    eF = rel(S.F.cpu().numpy().ravel(), F)
    sw = sweeps.cpu().numpy()
    # local solutions against the oracle's dense solve
    b = OL.local_blocks(ex, pb, R, np.arange(nelt))
    A1, A2, Af, _ = OL.local_solver_matrices(b)
    Xref = np.linalg.solve(A1, np.concatenate([A2, Af[:, :, None]], axis=2))
    eX = rel(X.cpu().numpy().reshape(Xref.shape), Xref)
    # reconstruction on the oracle's traces
    out = OG.solve_problem(ex, pb, k, with_post=False)
    uh = torch.as_tensor(out["uhat"], device="cuda").contiguous()
    q, u = L.hdg_recover_ir(S.disc, S.mesh, X, uh)
    torch.cuda.synchronize()
    eq, eu = rel(q.cpu().numpy(), out["q"]), rel(u.cpu().numpy(), out["u"])
    print(f"  rel errors: H {eH:.2e} F {eF:.2e} X {eX:.2e} q {eq:.2e} u {eu:.2e}; sweeps {sw.min()}..{sw.max()}",
          flush=True)
    assert np.isfinite(Hg.toarray()).all() and abs(Hg - Hg.T).max() == 0
    assert max(eH, eF, eX, eq, eu) < TOL_IR
    assert sw.max() < 8  # every element met the stopping rule


def test_ir_rejects_unsupported_degrees():
    from paper_1305_1489_amd import _lib as L
    m = make_mesh(1)
    pb = _problem_random_tau(m, seed=1)
    for k in (0, 4):
        S = gpu_system(m, k, pb)
        with pytest.raises(L.HdgError):
            L.hdg_assemble_condense_ir(S.disc, S.mesh, S.kappa, S.c, S.f, S.tau, S.H, S.F)
