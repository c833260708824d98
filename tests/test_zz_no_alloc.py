"""hdg_assemble_condense_noalloc (the library's static workspace) against
hdg_assemble_condense_ws (the caller's workspace) through the C ABI: the same H, F and
factor store bit for bit, on two calls in a row on one device, the second with a smaller
mesh; a mesh whose workspace exceeds the static capacity is refused before any launch."""
import numpy as np
import pytest
import torch

from hdg_inputs import manufactured_sin_xyz
from _gpu_helpers import gpu_system, make_mesh

pytestmark = pytest.mark.gpu
MIXED = dict(dirichlet=("x0", "x1"), neumann=("y0", "y1", "z0", "z1"))


def _bits(t):
    return t.view(torch.int64)


def _reference_and_noalloc(S):
    from paper_1305_1489_amd import _lib as L
    outs = []
    for fn in (lambda H, F, X: L.hdg_assemble_condense_ws(S.disc, S.mesh, S.kappa, S.c, S.f, S.tau, H, F, X),
               lambda H, F, X: L.hdg_assemble_condense_noalloc(S.disc, S.mesh, S.kappa, S.c, S.f, S.tau, H, F, X)):
        H = torch.full_like(S.H, float("nan"))
        F = torch.full_like(S.F, float("nan"))
        X = torch.full_like(S.factors, float("nan"))
        fn(H, F, X)
        torch.cuda.synchronize()
        outs.append((H, F, X))
    return outs


@pytest.mark.parametrize("k", [1, 2, 3, 4])
def test_noalloc_equals_workspace_form_two_calls(k):
    from paper_1305_1489_amd import _lib as L
    assert L.hdg_condense_noalloc_capacity() == 256 << 20
    pb = manufactured_sin_xyz("c1", "c1")
    for n in (8, 5):  # second call: a smaller mesh, over whatever the first left in the array
        m = make_mesh(n, jitter=0.1, seed=n + 10 * k, **MIXED)
        pb.tau = np.random.default_rng(n).uniform(0.3, 2.0, size=(m.nelt, 4))
        print(f"no-alloc k={k} n={n} ({m.nelt} elements)", flush=True)
        S = gpu_system(m, k, pb)
        (H0, F0, X0), (H1, F1, X1) = _reference_and_noalloc(S)
        assert not torch.isnan(H0).any()
        assert torch.equal(_bits(H1), _bits(H0)), f"k={k} n={n}: H"
        assert torch.equal(_bits(F1), _bits(F0)), f"k={k} n={n}: F"
        assert torch.equal(_bits(X1), _bits(X0)), f"k={k} n={n}: factors"


def test_noalloc_refuses_a_mesh_beyond_capacity():
    from paper_1305_1489_amd import _lib as L
    m = make_mesh(27)  # 118,098 elements: 291 MB of workspace at k = 3
    M = L.hdg_mesh_expand(m.coordinates, m.elements, m.dirichlet, m.neumann)
    disc = L.hdg_disc_create(3)
    assert L.hdg_condense_workspace_size(disc, M) > L.hdg_condense_noalloc_capacity()
    d2, nqd = disc.d2, disc.nqd
    f64 = dict(dtype=torch.float64, device="cuda")
    coef = torch.ones((M.nelt, nqd), **f64)
    tau = torch.ones((M.nelt, 4), **f64)
    H = torch.zeros((M.nnzb, d2, d2), **f64)
    F = torch.zeros((M.nfc, d2), **f64)
    X = torch.zeros((M.nelt, disc.factor_len), **f64)
    with pytest.raises(L.HdgError) as e:
        L.hdg_assemble_condense_noalloc(disc, M, coef, coef, coef, tau, H, F, X)
    assert e.value.name == "HDG_ERR_WORKSPACE"
    torch.cuda.synchronize()
    assert not H.any() and not F.any()  # refused before any launch: nothing written
