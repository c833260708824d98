"""Dense polynomials in d variables with float64 coefficients (oracle helper).

A polynomial is an ndarray ``c`` with c[a1, ..., ad] the coefficient of
x1^a1 ... xd^ad.  Products use direct (not FFT) N-d convolution so that
coefficients are exact sums of products.
"""
from __future__ import annotations

import numpy as np
from scipy.signal import convolve


class Poly:
    def __init__(self, coef):
        self.c = np.asarray(coef, dtype=np.float64)

    @property
    def ndim(self):
        return self.c.ndim

    @staticmethod
    def const(v, ndim):
        return Poly(np.full((1,) * ndim, float(v)))

    @staticmethod
    def var(i, ndim, scale=1.0, shift=0.0):
        """scale * x_i + shift."""
        shape = [1] * ndim
        shape[i] = 2
        c = np.zeros(shape)
        idx0 = (0,) * ndim
        idx1 = tuple(1 if j == i else 0 for j in range(ndim))
        c[idx0] = shift
        c[idx1] = scale
        return Poly(c)

    def _pad(self, shape):
        out = np.zeros(shape)
        out[tuple(slice(0, s) for s in self.c.shape)] = self.c
        return out

    def __add__(self, o):
        if not isinstance(o, Poly):
            o = Poly.const(o, self.ndim)
        shape = tuple(max(a, b) for a, b in zip(self.c.shape, o.c.shape))
        return Poly(self._pad(shape) + o._pad(shape))

    __radd__ = __add__

    def __neg__(self):
        return Poly(-self.c)

    def __sub__(self, o):
        return self + (-o if isinstance(o, Poly) else -float(o))

    def __rsub__(self, o):
        return (-self) + o

    def __mul__(self, o):
        if not isinstance(o, Poly):
            return Poly(self.c * float(o))
        return Poly(convolve(self.c, o.c, method="direct"))

    __rmul__ = __mul__

    def __pow__(self, n):
        out = Poly.const(1.0, self.ndim)
        for _ in range(n):
            out = out * self
        return out

    def deriv(self, i):
        c = self.c
        if c.shape[i] == 1:
            return Poly(np.zeros((1,) * self.ndim))
        idx = [slice(None)] * self.ndim
        idx[i] = slice(1, None)
        d = c[tuple(idx)]
        e = np.arange(1, c.shape[i], dtype=np.float64)
        sh = [1] * self.ndim
        sh[i] = -1
        return Poly(d * e.reshape(sh))

    def degree_shape(self, shape):
        return Poly(self._pad(tuple(max(a, b) for a, b in zip(self.c.shape, shape))))


def stack_eval(polys, pts):
    """Evaluate polynomials (list of Poly, same ndim) at points pts (..., ndim).

    Returns an array (..., len(polys))."""
    pts = np.asarray(pts, dtype=np.float64)
    nd = polys[0].ndim
    shape = tuple(max(p.c.shape[j] for p in polys) for j in range(nd))
    C = np.stack([p._pad(shape) for p in polys])  # (nb, n1, ..., nd)
    lead = pts.shape[:-1]
    P = pts.reshape(-1, nd)
    out = C.reshape(len(polys), -1)
    # monomial values at points
    pw = [P[:, j:j + 1] ** np.arange(shape[j])[None, :] for j in range(nd)]
    M = pw[0]
    for j in range(1, nd):
        M = (M[:, :, None] * pw[j][:, None, :]).reshape(P.shape[0], -1)
    return (M @ out.T).reshape(lead + (len(polys),))


def jacobi_poly1(n: int, alpha: float, beta: float) -> np.ndarray:
    """Monomial coefficients (ascending) of the Jacobi polynomial P_n^{(alpha,beta)}(x),
    from the explicit sum  sum_m C(n+a, n-m) C(n+b, m) ((x-1)/2)^m ((x+1)/2)^(n-m)."""
    from numpy.polynomial import polynomial as npp
    from scipy.special import binom
    out = np.zeros(n + 1)
    for m in range(n + 1):
        term = np.array([binom(n + alpha, n - m) * binom(n + beta, m)])
        term = npp.polymul(term, npp.polypow([-0.5, 0.5], m))
        term = npp.polymul(term, npp.polypow([0.5, 0.5], n - m))
        out[:len(term)] += term
    return out
