"""Condensation at the full size of the throughput workload (82,944 jittered elements, the
n = 24 Kuhn mesh), where every persistent workgroup sweeps many element groups.

* The atomic scatter (hdg_assemble_condense) and the atomic-free one
  (hdg_assemble_condense_ws) give the same H, F and factor store bit for bit, k = 1..3.
  Both run the same element kernel; the first copies its divergence tables into LDS
  space that held the element weights a moment earlier, and these tests are the
  regression check for the ordering of that copy after the weights' last reads.
* 256 seeded elements per degree: the H blocks and F entries they touch, and their
  reconstruction and postprocess, against the oracle (eq 5.5-5.6, eq 6.5, eq 5.3,
  eq 9.11) at 1e-12, k = 1..4.
"""
import numpy as np
import pytest
import torch

from hdg_inputs import manufactured_sin_xyz
from _gpu_helpers import gpu_system, make_mesh, oracle_expand, sampled_h_f_errors, sampled_recovery_errors

pytestmark = pytest.mark.gpu
TOL = 1e-12
MIXED = dict(dirichlet=("x0", "x1"), neumann=("y0", "y1", "z0", "z1"))


@pytest.fixture(scope="module")
def full_mesh():
    m = make_mesh(24, jitter=0.15, seed=0, **MIXED)
    return m, oracle_expand(m)


def _bits(t):
    return t.view(torch.int64)


@pytest.mark.parametrize("k", [1, 2, 3, 4])
def test_full_size_scatter_forms_and_oracle_samples(full_mesh, k):
    m, ex = full_mesh
    pb = manufactured_sin_xyz("c1", "c1")
    print(f"full size k={k}: {m.nelt} elements", flush=True)
    S = gpu_system(m, k, pb)
    nan = float("nan")
    for t in (S.H, S.F, S.factors):
        t.fill_(nan)
    S.assemble(atomic=True)
    torch.cuda.synchronize()
    H0, F0, X0 = S.H.clone(), S.F.clone(), S.factors.clone()
    assert not torch.isnan(H0).any() and not torch.isnan(F0).any()
    for t in (S.H, S.F, S.factors):
        t.fill_(nan)
    S.assemble(atomic=(k == 4))  # degree 4 has only the atomic form: a second run must repeat it
    torch.cuda.synchronize()
    assert torch.equal(_bits(S.H), _bits(H0)), f"k={k}: H differs between the scatter forms"
    assert torch.equal(_bits(S.F), _bits(F0)), f"k={k}: F differs between the scatter forms"
    assert torch.equal(_bits(S.factors), _bits(X0)), f"k={k}: factor store differs between the scatter forms"
    del H0, F0, X0
    elems = np.sort(np.random.default_rng(100 + k).choice(m.nelt, size=256, replace=False))
    err = sampled_h_f_errors(S, ex, pb, k, elems)
    print("H/F errors", err, flush=True)
    assert max(err.values()) < TOL, err
    uhat = np.random.default_rng(200 + k).normal(size=(ex.nfc, S.disc.d2))
    err = sampled_recovery_errors(S, ex, pb, k, elems, uhat)
    print("recovery errors", err, flush=True)
    assert max(err.values()) < TOL, err
