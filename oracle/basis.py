"""Orthonormal hierarchical Dubiner bases as exact polynomials (oracle).

Eq 3.3 pushes forward a Dubiner basis written on the enlarged element
2K - (1,1,1); Section 4 does the same on 2K_2 - (1,1).  The paper asks only for
L2-orthogonality and hierarchical order.  The reading used here (normalisation,
order and sign are not fixed by the paper):

  3-D, on xi in the enlarged tetrahedron, collapsed coordinates
      a = 2(1+xi1)/(-xi2-xi3) - 1,  b = 2(1+xi2)/(1-xi3) - 1,  c = xi3,
      psi_pqr = P_p(a) ((1-b)/2)^p P_q^{(2p+1,0)}(b) ((1-c)/2)^{p+q} P_r^{(2p+2q+2,0)}(c),
      Phat_pqr = psi_pqr sqrt((2p+1)(2p+2q+2)(2p+2q+2r+3)/6);
  2-D, a = 2(1+xi1)/(1-xi2) - 1, b = xi2,
      psi_pq = P_p(a) ((1-b)/2)^p P_q^{(2p+1,0)}(b),  Dhat_pq = psi_pq sqrt((2p+1)(p+q+1)).

With this scaling the bases are orthonormal for the normalised measures
(sum_q w_q Phat_i Phat_j = delta_ij with weights summing to 1), Phat_1 = Dhat_1 = 1.
Order: total degree n = 0..k, then p = 0..n, q = 0..n-p (r = n-p-q).

Each function is expanded here into monomials of the reference coordinates,
which removes the collapsed-coordinate singularity: values and gradients are
evaluated as plain polynomials.  The homogenised form used for the expansion is
    psi_pqr = [P_p(X/Y) Y^p] [P_q(U/V) V^q] P_r(xi3) / 2^{p+q},
X = 2 + 2xi1 + xi2 + xi3, Y = -xi2 - xi3, U = 1 + 2xi2 + xi3, V = 1 - xi3.
"""
from __future__ import annotations

from functools import lru_cache
from math import comb, sqrt

import numpy as np

from .poly import Poly, jacobi_poly1, stack_eval


def dim3(k: int) -> int:
    return comb(k + 3, 3)


def dim2(k: int) -> int:
    return comb(k + 2, 2)


def indices3(k):
    return [(p, q, n - p - q) for n in range(k + 1) for p in range(n + 1) for q in range(n - p + 1)]


def indices2(k):
    return [(p, n - p) for n in range(k + 1) for p in range(n + 1)]


def _homog(coefs, X, Y, n):
    """sum_j coefs[j] X^j Y^(n-j)  (coefs ascending)."""
    out = None
    for j, cj in enumerate(coefs):
        if cj == 0.0:
            continue
        t = (X ** j) * (Y ** (n - j)) * cj
        out = t if out is None else out + t
    return out if out is not None else X * 0.0


def _jac_of(poly_arg, n, alpha):
    """P_n^{(alpha,0)}(g) for a polynomial g."""
    co = jacobi_poly1(n, alpha, 0.0)
    out = Poly.const(0.0, poly_arg.ndim)
    for j, cj in enumerate(co):
        out = out + (poly_arg ** j) * cj
    return out


@lru_cache(maxsize=None)
def dubiner3(k: int):
    """List of Poly (3 variables: reference x, y, z) for Phat_1..Phat_d3."""
    # xi = 2 x - 1
    xi1 = Poly.var(0, 3, 2.0, -1.0)
    xi2 = Poly.var(1, 3, 2.0, -1.0)
    xi3 = Poly.var(2, 3, 2.0, -1.0)
    X = xi1 * 2.0 + xi2 + xi3 + 2.0
    Y = -(xi2 + xi3)
    U = xi2 * 2.0 + xi3 + 1.0
    V = 1.0 - xi3
    out = []
    for (p, q, r) in indices3(k):
        A = _homog(jacobi_poly1(p, 0.0, 0.0), X, Y, p)
        B = _homog(jacobi_poly1(q, 2 * p + 1.0, 0.0), U, V, q)
        C = _jac_of(xi3, r, 2 * p + 2 * q + 2.0)
        psi = A * B * C * (1.0 / 2 ** (p + q))
        out.append(psi * sqrt((2 * p + 1) * (2 * p + 2 * q + 2) * (2 * p + 2 * q + 2 * r + 3) / 6.0))
    return out


@lru_cache(maxsize=None)
def dubiner2(k: int):
    """List of Poly (2 variables: reference s, t) for Dhat_1..Dhat_d2."""
    xi1 = Poly.var(0, 2, 2.0, -1.0)
    xi2 = Poly.var(1, 2, 2.0, -1.0)
    X = xi1 * 2.0 + xi2 + 1.0
    Y = 1.0 - xi2
    out = []
    for (p, q) in indices2(k):
        A = _homog(jacobi_poly1(p, 0.0, 0.0), X, Y, p)
        B = _jac_of(xi2, q, 2 * p + 1.0)
        psi = A * B * (1.0 / 2 ** p)
        out.append(psi * sqrt((2 * p + 1) * (p + q + 1)))
    return out


@lru_cache(maxsize=None)
def _grad3(k):
    return tuple([b.deriv(j) for b in dubiner3(k)] for j in range(3))


def eval3(k, pts):
    """Phat_j at reference points pts (..., 3) -> (..., d3)  (the matrix P of eq 3.5)."""
    return stack_eval(dubiner3(k), pts)


def grad3(k, pts):
    """Reference gradients (3, ..., d3): P^x, P^y, P^z of eq 3.66."""
    return np.stack([stack_eval(g, pts) for g in _grad3(k)])


def eval2(k, pts):
    """Dhat_i at reference triangle points (..., 2) -> (..., d2)  (the matrix D of eq 4.7)."""
    return stack_eval(dubiner2(k), pts)
