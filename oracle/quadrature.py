"""Quadrature on the reference tetrahedron and triangle (oracle).

The paper leaves the rules open (eq 3.1 only asks for points p_q and weights
summing to 1; Section 4 does the same for the triangle).  The reading used here:
Stroud conical-product Gauss-Jacobi rules with ``n`` points per collapsed
direction (n = k + 2 by default), exact for polynomials of degree 2n - 1.

Tetrahedron: collapsed (a, b, c) in [-1, 1]^3 with Gauss-Jacobi nodes for the
weights (1-a)^0, (1-b)^1, (1-c)^2; xi1 = (1+a)(1-b)(1-c)/4 - 1,
xi2 = (1+b)(1-c)/2 - 1, xi3 = c on the enlarged element 2K - (1,1,1); reference
point x = (xi + 1) / 2.  Node order: a slowest, then b, then c.
Triangle: (1-a)^0, (1-b)^1; xi1 = (1+a)(1-b)/2 - 1, xi2 = b; (s, t) = (xi + 1)/2;
a slowest.  Weights are normalised to sum to 1.
"""
from __future__ import annotations

import numpy as np
from scipy.special import roots_jacobi


def tet_rule(n: int):
    """Points (Nq, 3) in the reference tetrahedron and weights (Nq,) summing to 1 (eq 3.1)."""
    a, wa = roots_jacobi(n, 0.0, 0.0)
    b, wb = roots_jacobi(n, 1.0, 0.0)
    c, wc = roots_jacobi(n, 2.0, 0.0)
    A, B, C = np.meshgrid(a, b, c, indexing="ij")
    W = wa[:, None, None] * wb[None, :, None] * wc[None, None, :]
    xi1 = (1 + A) * (1 - B) * (1 - C) / 4 - 1
    xi2 = (1 + B) * (1 - C) / 2 - 1
    xi3 = C
    pts = np.stack([xi1.ravel(), xi2.ravel(), xi3.ravel()], axis=1)
    pts = (pts + 1) / 2
    w = W.ravel()
    return pts, w / w.sum()


def tri_rule(n: int):
    """Points (Nq2, 2) in the reference triangle and weights summing to 1 (Section 4)."""
    a, wa = roots_jacobi(n, 0.0, 0.0)
    b, wb = roots_jacobi(n, 1.0, 0.0)
    A, B = np.meshgrid(a, b, indexing="ij")
    W = wa[:, None] * wb[None, :]
    xi1 = (1 + A) * (1 - B) / 2 - 1
    xi2 = B
    pts = (np.stack([xi1.ravel(), xi2.ravel()], axis=1) + 1) / 2
    w = W.ravel()
    return pts, w / w.sum()

