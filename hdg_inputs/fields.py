"""Coefficient fields and manufactured solutions for the model problem eq 1.1:

    kappa^{-1} q + grad u = 0,  div q + c u = f  in Omega,
    u = u_D on Gamma_D,  -q . nu = g_N . nu on Gamma_N.

A :class:`Problem` bundles kappa(x), c(x), f(x), u_D(x), the Neumann vector
field g_N(x) (only its normal component is used, Section 1), the stabilisation
tau (a constant, or one value per (element, local face)), and -- when known --
the exact u and q for error measurement.

Every field is a plain function of coordinate arrays.  The functions accept
numpy arrays or torch tensors (same expression, evaluated with whichever
library owns the input), so the same definition can be evaluated on the host
for the oracle or on the device for the library's tests and benchmarks.
"""
from __future__ import annotations

import math
from dataclasses import dataclass, field
from typing import Callable, Optional

import numpy as np


def _xp(x):
    if isinstance(x, np.ndarray) or np.isscalar(x):
        return np
    import torch
    return torch


def _full_like(x, v):
    xp = _xp(x)
    return xp.full_like(x, float(v)) if xp is np else x * 0 + float(v)


@dataclass
class Problem:
    kappa: Callable
    c: Callable
    f: Callable
    uD: Callable
    gN: Callable                      # returns a tuple (gx, gy, gz)
    tau: object = 1.0                 # float or array (Nelt, 4)
    u: Optional[Callable] = None      # exact solution (if known)
    q: Optional[Callable] = None      # exact flux q = -kappa grad u (tuple)
    name: str = ""
    meta: dict = field(default_factory=dict)


# --------------------------------------------------------------------------------------
# manufactured smooth solutions
# --------------------------------------------------------------------------------------
def _manufactured(u, grad_u, lap_u, kappa, grad_kappa, c, name, tau=1.0):
    def q(x, y, z):
        k = kappa(x, y, z)
        gx, gy, gz = grad_u(x, y, z)
        return (-k * gx, -k * gy, -k * gz)

    def f(x, y, z):
        k = kappa(x, y, z)
        kx, ky, kz = grad_kappa(x, y, z)
        gx, gy, gz = grad_u(x, y, z)
        return -(kx * gx + ky * gy + kz * gz + k * lap_u(x, y, z)) + c(x, y, z) * u(x, y, z)

    def gN(x, y, z):
        k = kappa(x, y, z)
        gx, gy, gz = grad_u(x, y, z)
        return (k * gx, k * gy, k * gz)

    return Problem(kappa=kappa, c=c, f=f, uD=u, gN=gN, tau=tau, u=u, q=q, name=name)


def _sin_xyz():
    def u(x, y, z):
        return _xp(x).sin(x * y * z)

    def grad_u(x, y, z):
        cc = _xp(x).cos(x * y * z)
        return (cc * y * z, cc * x * z, cc * x * y)

    def lap_u(x, y, z):
        return -_xp(x).sin(x * y * z) * (y * y * z * z + x * x * z * z + x * x * y * y)

    return u, grad_u, lap_u


def manufactured_sin_xyz(kappa_kind: str = "c1", c_kind: str = "c1", tau=1.0) -> Problem:
    """u = sin(xyz) (the exact solution of the paper's experiments, Section 8).

    kappa_kind "c1": kappa = 1 + 0.5 sin(2 pi x) cos(2 pi y); "paper":
    kappa = 2 + sin x sin y sin z; "one": kappa = 1.
    c_kind "c1": c = 1 + |x|^2; "paper": c = 1 + |x|^2 / 2; "zero": c = 0.
    """
    u, grad_u, lap_u = _sin_xyz()
    if kappa_kind == "c1":
        def kappa(x, y, z):
            xp = _xp(x)
            return 1.0 + 0.5 * xp.sin(2 * math.pi * x) * xp.cos(2 * math.pi * y)

        def grad_kappa(x, y, z):
            xp = _xp(x)
            return (math.pi * xp.cos(2 * math.pi * x) * xp.cos(2 * math.pi * y),
                    -math.pi * xp.sin(2 * math.pi * x) * xp.sin(2 * math.pi * y), _full_like(x, 0.0))
    elif kappa_kind == "paper":
        def kappa(x, y, z):
            xp = _xp(x)
            return 2.0 + xp.sin(x) * xp.sin(y) * xp.sin(z)

        def grad_kappa(x, y, z):
            xp = _xp(x)
            sx, sy, sz = xp.sin(x), xp.sin(y), xp.sin(z)
            return (xp.cos(x) * sy * sz, sx * xp.cos(y) * sz, sx * sy * xp.cos(z))
    elif kappa_kind == "one":
        def kappa(x, y, z):
            return _full_like(x, 1.0)

        def grad_kappa(x, y, z):
            return (_full_like(x, 0.0),) * 3
    else:
        raise ValueError(kappa_kind)
    if c_kind == "c1":
        def c(x, y, z):
            return 1.0 + x * x + y * y + z * z
    elif c_kind == "paper":
        def c(x, y, z):
            return 1.0 + 0.5 * (x * x + y * y + z * z)
    elif c_kind == "zero":
        def c(x, y, z):
            return _full_like(x, 0.0)
    else:
        raise ValueError(c_kind)
    return _manufactured(u, grad_u, lap_u, kappa, grad_kappa, c, f"sin_xyz/{kappa_kind}/{c_kind}", tau)


def manufactured_sin_pi(tau=1.0) -> Problem:
    """u = sin(pi x) sin(pi y) sin(pi z), kappa = 1, c = 0, f = 3 pi^2 u (u = 0 on the cube's boundary)."""
    def u(x, y, z):
        xp = _xp(x)
        return xp.sin(math.pi * x) * xp.sin(math.pi * y) * xp.sin(math.pi * z)

    def grad_u(x, y, z):
        xp = _xp(x)
        sx, sy, sz = xp.sin(math.pi * x), xp.sin(math.pi * y), xp.sin(math.pi * z)
        cx, cy, cz = xp.cos(math.pi * x), xp.cos(math.pi * y), xp.cos(math.pi * z)
        return (math.pi * cx * sy * sz, math.pi * sx * cy * sz, math.pi * sx * sy * cz)

    def lap_u(x, y, z):
        return -3 * math.pi ** 2 * u(x, y, z)

    def kappa(x, y, z):
        return _full_like(x, 1.0)

    def grad_kappa(x, y, z):
        return (_full_like(x, 0.0),) * 3

    def c(x, y, z):
        return _full_like(x, 0.0)

    return _manufactured(u, grad_u, lap_u, kappa, grad_kappa, c, "sin_pi", tau)


# --------------------------------------------------------------------------------------
# polynomial exact solutions (Section 8, last paragraph: exact polynomial solutions)
# --------------------------------------------------------------------------------------
def polynomial_problem(degree: int, seed: int = 0, kappa: float = 2.0, c: float = 1.0,
                       c_linear: bool = False, tau=1.0) -> Problem:
    """u = a random polynomial of total degree <= ``degree`` with constant kappa.

    c is the constant ``c``; with ``c_linear`` it is c (1 + x + 2y - z / 2) instead
    (reproduction still holds for a variable c, only kappa must be constant).
    """
    rng = np.random.Generator(np.random.PCG64(seed))
    exps = [(a, b, g) for a in range(degree + 1) for b in range(degree + 1 - a) for g in range(degree + 1 - a - b)]
    coef = rng.uniform(-1.0, 1.0, size=len(exps))

    def mono(x, a):
        return x ** a if a else _full_like(x, 1.0)

    def u(x, y, z):
        s = 0.0 * x
        for (a, b, g), cc in zip(exps, coef):
            s = s + cc * mono(x, a) * mono(y, b) * mono(z, g)
        return s

    def grad_u(x, y, z):
        gx = 0.0 * x
        gy = 0.0 * x
        gz = 0.0 * x
        for (a, b, g), cc in zip(exps, coef):
            if a:
                gx = gx + cc * a * mono(x, a - 1) * mono(y, b) * mono(z, g)
            if b:
                gy = gy + cc * b * mono(x, a) * mono(y, b - 1) * mono(z, g)
            if g:
                gz = gz + cc * g * mono(x, a) * mono(y, b) * mono(z, g - 1)
        return (gx, gy, gz)

    def lap_u(x, y, z):
        s = 0.0 * x
        for (a, b, g), cc in zip(exps, coef):
            if a > 1:
                s = s + cc * a * (a - 1) * mono(x, a - 2) * mono(y, b) * mono(z, g)
            if b > 1:
                s = s + cc * b * (b - 1) * mono(x, a) * mono(y, b - 2) * mono(z, g)
            if g > 1:
                s = s + cc * g * (g - 1) * mono(x, a) * mono(y, b) * mono(z, g - 2)
        return s

    kap = float(kappa)

    def kappa_f(x, y, z):
        return _full_like(x, kap)

    def grad_kappa(x, y, z):
        return (_full_like(x, 0.0),) * 3

    if c_linear:
        def c_f(x, y, z):
            return c * (1.0 + x + 2.0 * y - 0.5 * z)
    else:
        def c_f(x, y, z):
            return _full_like(x, float(c))

    p = _manufactured(u, grad_u, lap_u, kappa_f, grad_kappa, c_f, f"poly{degree}", tau)
    p.meta = {"exps": exps, "coef": coef}
    return p


# --------------------------------------------------------------------------------------
# random Fourier-feature Gaussian fields (log-normal kappa workloads)
# --------------------------------------------------------------------------------------
def rff_field(seed: int, corr_len: float, n_features: int = 512):
    """Gaussian random field g with unit variance and covariance exp(-r^2 / (2 l^2)),
    by random Fourier features: g(x) = sqrt(2/M) sum_m cos(w_m . x + phi_m),
    w_m ~ N(0, l^-2 I), phi_m ~ U[0, 2 pi); drawn from numpy's PCG64(seed)."""
    rng = np.random.Generator(np.random.PCG64(seed))
    w = rng.normal(0.0, 1.0 / corr_len, size=(n_features, 3))
    phi = rng.uniform(0.0, 2.0 * math.pi, size=n_features)
    scale = math.sqrt(2.0 / n_features)

    def g(x, y, z):
        xp = _xp(x)
        if xp is np:
            shp = np.shape(x)
            X = np.stack([np.ravel(x), np.ravel(y), np.ravel(z)], axis=1)
            out = np.empty(X.shape[0])
            for s in range(0, X.shape[0], 65536):
                out[s:s + 65536] = scale * np.cos(X[s:s + 65536] @ w.T + phi).sum(axis=1)
            return out.reshape(shp)
        import torch
        shp = x.shape
        X = torch.stack([x.reshape(-1), y.reshape(-1), z.reshape(-1)], dim=1)
        W = torch.as_tensor(w.T, dtype=X.dtype, device=X.device)
        P = torch.as_tensor(phi, dtype=X.dtype, device=X.device)
        out = torch.empty(X.shape[0], dtype=X.dtype, device=X.device)
        for s in range(0, X.shape[0], 1 << 20):
            out[s:s + (1 << 20)] = scale * torch.cos(X[s:s + (1 << 20)] @ W + P).sum(dim=1)
        return out.reshape(shp)

    return g


def constant_rhs_problem(kappa_sigma: float, corr_len: float, field_seed: int, c: float, tau=1.0) -> Problem:
    """kappa = exp(sigma g) with g a random Fourier-feature field, constant c, f = 1,
    homogeneous Dirichlet data; no exact solution."""
    g = rff_field(field_seed, corr_len)

    def kappa(x, y, z):
        return _xp(x).exp(kappa_sigma * g(x, y, z))

    def c_f(x, y, z):
        return _full_like(x, float(c))

    def f(x, y, z):
        return _full_like(x, 1.0)

    def uD(x, y, z):
        return _full_like(x, 0.0)

    def gN(x, y, z):
        z0 = _full_like(x, 0.0)
        return (z0, z0, z0)

    return Problem(kappa=kappa, c=c_f, f=f, uD=uD, gN=gN, tau=tau, name=f"lognormal(s={kappa_sigma},l={corr_len},seed={field_seed})")


# --------------------------------------------------------------------------------------
# convection-diffusion: div(q + beta u) + c u = f with q = -kappa grad u
# --------------------------------------------------------------------------------------
def _affine_beta(b0, Bm):
    """beta(x) = b0 + Bm x (a tuple of three fields) and its divergence trace(Bm)."""
    b0 = np.asarray(b0, dtype=np.float64)
    Bm = np.asarray(Bm, dtype=np.float64)

    def beta(x, y, z):
        X = (x, y, z)
        return tuple(b0[i] + Bm[i, 0] * X[0] + Bm[i, 1] * X[1] + Bm[i, 2] * X[2] for i in range(3))

    return beta, float(np.trace(Bm))


def convection_problem(u, grad_u, lap_u, kappa_const, beta_b0, beta_B, c, tau, name):
    """Manufactured data for a constant kappa, an affine beta and a constant c: f and the
    Neumann field g_N = kappa grad u - beta u, whose normal component is the total outward
    flux -(q + beta u).nu.  ``tau`` is the stabilisation (a constant or per (element, face))."""
    beta, divb = _affine_beta(beta_b0, beta_B)
    kap = float(kappa_const)

    def q(x, y, z):
        g = grad_u(x, y, z)
        return tuple(-kap * gi for gi in g)

    def f(x, y, z):
        g = grad_u(x, y, z)
        b = beta(x, y, z)
        uu = u(x, y, z)
        return -kap * lap_u(x, y, z) + b[0] * g[0] + b[1] * g[1] + b[2] * g[2] + (divb + c) * uu

    def gN(x, y, z):
        g = grad_u(x, y, z)
        b = beta(x, y, z)
        uu = u(x, y, z)
        return tuple(kap * g[i] - b[i] * uu for i in range(3))

    p = Problem(kappa=lambda x, y, z: _full_like(x, kap), c=lambda x, y, z: _full_like(x, float(c)), f=f,
                uD=u, gN=gN, tau=tau, u=u, q=q, name=name)
    p.beta = beta
    p.meta = {"beta_b0": list(map(float, beta_b0)), "beta_B": np.asarray(beta_B, dtype=float).tolist(),
              "div_beta": divb}
    return p


def convection_sin_problem(beta_scale=1.0, kappa=1.0, c=1.0, tau=None) -> Problem:
    """u = sin(xyz) with kappa constant, beta = beta_scale ((1, 0.5, -0.3) + (0.5 y, -0.4 z, 0.3 x))
    (divergence free) and c constant; tau = 1 + max |beta| on the unit cube unless given."""
    b0 = beta_scale * np.array([1.0, 0.5, -0.3])
    B = beta_scale * np.array([[0.0, 0.5, 0.0], [0.0, 0.0, -0.4], [0.3, 0.0, 0.0]])
    bmax = float(np.abs(b0).sum() + np.abs(B).sum())
    xp = lambda a: _xp(a)

    def u(x, y, z):
        return xp(x).sin(x * y * z)

    def grad_u(x, y, z):
        cc = xp(x).cos(x * y * z)
        return (y * z * cc, x * z * cc, x * y * cc)

    def lap_u(x, y, z):
        return -xp(x).sin(x * y * z) * ((y * z) ** 2 + (x * z) ** 2 + (x * y) ** 2)

    return convection_problem(u, grad_u, lap_u, kappa, b0, B, c, 1.0 + bmax if tau is None else tau,
                              f"convection_sin(beta x{beta_scale})")


def convection_polynomial_problem(degree: int, seed: int = 0, kappa: float = 1.5, c: float = 1.0,
                                  beta_scale: float = 1.0, tau=None) -> Problem:
    """u a random polynomial of total degree <= ``degree``, constant kappa and c, affine beta
    (seeded, with a non-zero divergence); tau = 1 + max |beta| on the unit cube unless given."""
    rng = np.random.Generator(np.random.PCG64(seed))
    base = polynomial_problem(degree, seed=seed, kappa=kappa, c=c)
    exps, coef = base.meta["exps"], base.meta["coef"]
    b0 = beta_scale * rng.uniform(-1.0, 1.0, size=3)
    B = beta_scale * rng.uniform(-0.5, 0.5, size=(3, 3))
    bmax = float(np.abs(b0).sum() + np.abs(B).sum())

    def mono(x, a):
        return x ** a if a else _full_like(x, 1.0)

    def grad_u(x, y, z):
        gx = 0.0 * x
        gy = 0.0 * x
        gz = 0.0 * x
        for (a, b, g), cc in zip(exps, coef):
            if a:
                gx = gx + cc * a * mono(x, a - 1) * mono(y, b) * mono(z, g)
            if b:
                gy = gy + cc * b * mono(x, a) * mono(y, b - 1) * mono(z, g)
            if g:
                gz = gz + cc * g * mono(x, a) * mono(y, b) * mono(z, g - 1)
        return (gx, gy, gz)

    def lap_u(x, y, z):
        s = 0.0 * x
        for (a, b, g), cc in zip(exps, coef):
            if a > 1:
                s = s + cc * a * (a - 1) * mono(x, a - 2) * mono(y, b) * mono(z, g)
            if b > 1:
                s = s + cc * b * (b - 1) * mono(x, a) * mono(y, b - 2) * mono(z, g)
            if g > 1:
                s = s + cc * g * (g - 1) * mono(x, a) * mono(y, b) * mono(z, g - 2)
        return s

    return convection_problem(base.u, grad_u, lap_u, kappa, b0, B, c, 1.0 + bmax if tau is None else tau,
                              f"convection_poly{degree}")
