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


__all__ = ["rel", "make_mesh", "gpu_system", "oracle_expand", "bsr_to_csr", "oracle_rules", "OG", "OL", "OM"]
