"""Shared set-up for the GPU parity tests: build the same synthetic problem for the HIP
library (through the C-ABI binding) and for the CPU oracle."""
from __future__ import annotations

import numpy as np

from hdg_inputs import kuhn_mesh
from oracle import globalsys as OG, local as OL, mesh as OM


def rel(a, b):
    a = np.asarray(a, dtype=np.float64)
    b = np.asarray(b, dtype=np.float64)
    den = np.abs(b).max()
    return float(np.abs(a - b).max() / (den if den > 0 else 1.0))


def make_mesh(n, jitter=0.0, seed=0, dirichlet=("x0", "x1", "y0", "y1", "z0", "z1"), neumann=()):
    return kuhn_mesh(n, jitter=jitter, seed=seed, dirichlet_sides=dirichlet, neumann_sides=neumann)


def gpu_system(m, k, problem):
    from paper_1305_1489_amd.driver import HDGSystem
    return HDGSystem(m.coordinates, m.elements, m.dirichlet, m.neumann, k, problem)


def oracle_expand(m):
    return OM.expand(m.coordinates, m.elements, m.dirichlet, m.neumann)


def bsr_to_csr(S):
    """Host CSR copy of the library's block-sparse H."""
    import scipy.sparse as sp
    m = S.mesh
    d2 = S.disc.d2
    rp = m.row_ptr.cpu().numpy()
    ci = m.col_idx.cpu().numpy()
    Hb = S.H.cpu().numpy()
    rows = np.repeat(np.arange(m.nfc), np.diff(rp))
    return sp.bsr_matrix((Hb, ci, rp), shape=(m.nfc * d2, m.nfc * d2)).tocsr(), rows


def oracle_rules(k):
    return OL.rules(k)


__all__ = ["rel", "make_mesh", "gpu_system", "oracle_expand", "bsr_to_csr", "oracle_rules", "sampled_h_f_errors",
           "sampled_recovery_errors", "csr_rel", "OG", "OL", "OM"]


def sampled_h_f_errors(S, ex, problem, k, elems):
    """Relative errors of the H blocks and F entries that the listed elements touch, against
    the oracle's element blocks (eq 5.5-5.6) summed per face as in eq 6.5.

    Off-diagonal blocks have one contributing element; a diagonal block and an F entry take
    the contributions of every element holding the face, so the oracle condenses those
    neighbours too.  Only the needed blocks are gathered from the device."""
    import torch
    d2 = S.disc.d2
    fbe = ex.facebyele
    assert np.array_equal(S.mesh.facebyele.cpu().numpy()[elems], fbe[elems])
    faces = np.unique(fbe[elems])
    holders = np.nonzero(np.isin(fbe, faces).any(axis=1))[0]
    C, Cf = OL.condense(OL.local_blocks(ex, problem, OL.rules(k), holders))
    at = {int(K): i for i, K in enumerate(holders)}
    slot = S.mesh.slot.cpu().numpy().reshape(-1, 4, 4)
    diag = S.mesh.diag.cpu().numpy()
    off_idx, off_ref = [], []
    for K in elems:
        CK = C[at[int(K)]]
        for l in range(4):
            for m in range(4):
                if l != m:
                    off_idx.append(slot[K, l, m])
                    off_ref.append(CK[l * d2:(l + 1) * d2, m * d2:(m + 1) * d2])
    dref = np.zeros((faces.size, d2, d2))
    fref = np.zeros((faces.size, d2))
    fpos = {int(f): i for i, f in enumerate(faces)}
    for K in holders:
        for l in range(4):
            f = int(fbe[K, l])
            if f in fpos:
                dref[fpos[f]] += C[at[int(K)]][l * d2:(l + 1) * d2, l * d2:(l + 1) * d2]
                fref[fpos[f]] += Cf[at[int(K)]][l * d2:(l + 1) * d2]
    dev = S.H.device
    Hoff = S.H[torch.as_tensor(np.array(off_idx), device=dev, dtype=torch.long)].cpu().numpy()
    Hdia = S.H[torch.as_tensor(diag[faces], device=dev, dtype=torch.long)].cpu().numpy()
    Fg = S.F[torch.as_tensor(faces, device=dev, dtype=torch.long)].cpu().numpy()
    return dict(H_off=rel(Hoff, np.array(off_ref)), H_diag=rel(Hdia, dref), F=rel(Fg, fref))


def sampled_recovery_errors(S, ex, problem, k, elems, uhat):
    """q, u (eq 5.3) and u* (eq 9.11) of the listed elements from the library's
    reconstruction with the trace uhat, against the oracle's local solves."""
    import torch
    R = OL.rules(k)
    S.uhat.copy_(torch.as_tensor(uhat))
    q, u, us = S.recover()
    b = OL.local_blocks(ex, problem, R, elems)
    qo, uo = OL.recover(b, uhat[ex.facebyele[elems]].reshape(len(elems), -1))
    uso = OG.postprocess(ex, problem, R, qo, uo, elems)
    idx = torch.as_tensor(np.asarray(elems), device=q.device, dtype=torch.long)
    return dict(q=rel(q[idx].cpu().numpy(), qo), u=rel(u[idx].cpu().numpy(), uo),
                ustar=rel(us[idx].cpu().numpy(), uso))


def csr_rel(Hg, H):
    """max |Hg - H| / max |H| for two scipy sparse matrices."""
    d = abs(Hg - H)
    return float((d.max() if d.nnz else 0.0) / abs(H).max())
