"""Relabelling the elements (a permutation of the element list).

The trace unknowns do not depend on the element order: faces are numbered by their vertex
keys.  A face's own parametrisation (its stored vertex order, Section 2) is taken from the
first element that holds it, so relabelling can rotate or reflect the parametrisation of
some interior faces, which changes their basis and so the corresponding blocks of H.
What must hold:
  * the same faces in the same order (as vertex sets);
  * bit for bit the same H blocks and F entries wherever both faces kept their
    parametrisation (one writer per off-diagonal block, at most two order-independent
    addends per diagonal block and F entry, and per-element work that does not depend on
    the element's position in its tile or workgroup);
  * the same q and u per element after solving each system (to the solver's accuracy)."""
import numpy as np
import pytest
import torch

from hdg_inputs import kuhn_mesh, manufactured_sin_xyz
from _gpu_helpers import gpu_system, rel

pytestmark = pytest.mark.gpu


@pytest.mark.parametrize("k", [0, 1, 2, 3, 4])
def test_element_permutation(k):
    m = kuhn_mesh(4, jitter=0.12, seed=31, dirichlet_sides=("x0", "x1"), neumann_sides=("y0", "y1", "z0", "z1"))
    perm = np.random.default_rng(100 + k).permutation(m.elements.shape[0])
    pb = manufactured_sin_xyz("c1", "c1")
    print(f"element order k={k}", flush=True)
    A = gpu_system(m, k, pb)
    from paper_1305_1489_amd.driver import HDGSystem
    B = HDGSystem(m.coordinates, m.elements[perm], m.dirichlet, m.neumann, k, pb)
    for S in (A, B):
        S.assemble()
    torch.cuda.synchronize()
    fa, fb = A.mesh.faces.cpu().numpy(), B.mesh.faces.cpu().numpy()
    assert np.array_equal(np.sort(fa, axis=1), np.sort(fb, axis=1))
    assert torch.equal(A.mesh.row_ptr, B.mesh.row_ptr) and torch.equal(A.mesh.col_idx, B.mesh.col_idx)
    same = np.all(fa == fb, axis=1)
    assert same.mean() > 0.3  # boundary faces keep their listed orientation
    rp = A.mesh.row_ptr.cpu().numpy()
    ci = A.mesh.col_idx.cpu().numpy()
    rows = np.repeat(np.arange(A.mesh.nfc), np.diff(rp))
    keep = same[rows] & same[ci]
    Ha, Hb = A.H.cpu().numpy(), B.H.cpu().numpy()
    assert np.array_equal(Ha[keep], Hb[keep])
    assert np.array_equal(A.F.cpu().numpy()[same], B.F.cpu().numpy()[same])
    out = []
    for S in (A, B):
        S.boundary()
        S.solve(rtol=1e-13)
        q, u, _ = S.recover(postprocess=False)
        out.append((q.cpu().numpy(), u.cpu().numpy()))
    assert rel(out[0][0][perm], out[1][0]) < 1e-10
    assert rel(out[0][1][perm], out[1][1]) < 1e-10
