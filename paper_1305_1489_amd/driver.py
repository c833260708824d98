"""End-to-end driver over the C-ABI: mesh expansion, tables, coefficients at the quadrature
points, assembly + condensation + scatter, boundary conditions, global solve,
reconstruction and postprocess.

Only marshalling and orchestration happen here.  The coefficient fields are whatever
callables the caller hands in (functions of device tensors X, Y, Z); they are evaluated
at the physical quadrature points that the library computes.
"""
from __future__ import annotations

import numpy as np
import torch

from . import _lib as L


def _field(fn, X, Y, Z):
    v = fn(X, Y, Z)
    if not isinstance(v, torch.Tensor):
        v = torch.as_tensor(v, dtype=torch.float64, device=X.device)
    return (v * torch.ones_like(X)).to(torch.float64).contiguous()


class HDGSystem:
    """Device state of one HDG problem (mesh, degree, data)."""

    def __init__(self, coords, elements, dirichlet, neumann, k, problem, device="cuda", stream=None, disc=None):
        self.device = torch.device(device)
        self.stream = stream
        self.mesh = L.hdg_mesh_expand(coords, elements, dirichlet, neumann, device=device, stream=stream)
        if disc is not None and disc.k != k:
            raise ValueError(f"disc has degree {disc.k}, expected {k}")
        self.disc = disc if disc is not None else L.hdg_disc_create(k)
        self.k = k
        self.problem = problem
        xyz = L.hdg_qp_coords(self.disc, self.mesh, stream=stream)
        X, Y, Z = xyz[..., 0], xyz[..., 1], xyz[..., 2]
        self.qp = xyz
        self.kappa = _field(problem.kappa, X, Y, Z)
        self.c = _field(problem.c, X, Y, Z)
        self.f = _field(problem.f, X, Y, Z)
        tau = problem.tau
        if np.isscalar(tau):
            self.tau = torch.full((self.mesh.nelt, 4), float(tau), dtype=torch.float64, device=self.device)
        else:
            self.tau = torch.as_tensor(np.asarray(tau, dtype=np.float64).reshape(-1, 4)).to(self.device).contiguous()
        m = self.mesh
        nqd2 = self.disc.nqd2
        if m.ndir:
            y = L.hdg_face_qp_coords(self.disc, m, m.dirfaces[: m.ndir], stream=stream)
            self.uD = _field(problem.uD, y[..., 0], y[..., 1], y[..., 2])
        else:
            self.uD = torch.zeros((1, nqd2), dtype=torch.float64, device=self.device)
        if m.nneu:
            y = L.hdg_face_qp_coords(self.disc, m, m.neufaces[: m.nneu], stream=stream)
            g = problem.gN(y[..., 0], y[..., 1], y[..., 2])
            self.gN = torch.stack([_field(lambda a, b, c, gi=gi: gi, y[..., 0], y[..., 1], y[..., 2]) for gi in g],
                                  dim=-1).contiguous()
        else:
            self.gN = torch.zeros((1, nqd2, 3), dtype=torch.float64, device=self.device)
        d2 = self.disc.d2
        self.H = torch.empty((m.nnzb, d2, d2), dtype=torch.float64, device=self.device)
        self.F = torch.empty((m.nfc, d2), dtype=torch.float64, device=self.device)
        self.factors = torch.empty((m.nelt, self.disc.factor_len), dtype=torch.float64, device=self.device)
        self.uhat = torch.zeros((m.nfc, d2), dtype=torch.float64, device=self.device)
        # per-(element, face) buffer of the atomic-free condensation (empty for k = 0, 4)
        self.condense_ws = torch.empty(max(L.hdg_condense_workspace_size(self.disc, m), 1), dtype=torch.uint8,
                                       device=self.device)

    # ---- stages
    def assemble(self, atomic=False, method="hdg"):
        """Condensation into H, F, factors; atomic=True selects the atomic scatter (same bits);
        method="bdm" the hybridized BDM element (tau = 0, u in P_{k-1})."""
        if method == "bdm":
            L.hdg_assemble_condense_bdm(self.disc, self.mesh, self.kappa, self.c, self.f, self.H, self.F,
                                        self.factors, ws=self.condense_ws, stream=self.stream)
        elif atomic:
            L.hdg_assemble_condense(self.disc, self.mesh, self.kappa, self.c, self.f, self.tau, self.H, self.F,
                                    self.factors, stream=self.stream)
        else:
            L.hdg_assemble_condense_ws(self.disc, self.mesh, self.kappa, self.c, self.f, self.tau, self.H, self.F,
                                       self.factors, ws=self.condense_ws, stream=self.stream)

    # ---- convection-diffusion (problem.beta: a callable returning the three components)
    def convection_fields(self):
        """beta at the volume points and at every element's own face points (evaluated once)."""
        if getattr(self, "beta_vol", None) is None:
            X, Y, Z = self.qp[..., 0], self.qp[..., 1], self.qp[..., 2]
            self.beta_vol = torch.stack([_field(lambda a, b, c, g=g: g, X, Y, Z) for g in self.problem.beta(X, Y, Z)],
                                        dim=-1).contiguous()
            y = L.hdg_elem_face_qp_coords(self.disc, self.mesh, stream=self.stream)
            Yx, Yy, Yz = y[..., 0], y[..., 1], y[..., 2]
            self.beta_face = torch.stack([_field(lambda a, b, c, g=g: g, Yx, Yy, Yz)
                                          for g in self.problem.beta(Yx, Yy, Yz)], dim=-1).contiguous()
            self.X = torch.empty((self.mesh.nelt, L.hdg_ir_store_len(self.disc)), dtype=torch.float64,
                                 device=self.device)
        return self.beta_vol, self.beta_face

    def assemble_cd(self):
        bv, bf = self.convection_fields()
        L.hdg_assemble_condense_cd(self.disc, self.mesh, self.kappa, self.c, self.f, bv, bf, self.tau, self.H, self.F,
                                   self.X, stream=self.stream)

    def run_cd(self, rtol=1e-10, restart=40, max_iter=20000, solver="gmres"):
        """Convection-diffusion: condensation, boundary data, GMRES(restart) or BiCGStab,
        reconstruction from X."""
        self.assemble_cd()
        self.boundary()
        if solver == "bicgstab":
            info = L.hdg_solve_bicgstab(self.disc, self.mesh, self.H, self.F, self.uhat, rtol=rtol,
                                        max_iter=max_iter, check_every=5, stream=self.stream)
        else:
            info = L.hdg_solve_gmres(self.disc, self.mesh, self.H, self.F, self.uhat, rtol=rtol, max_iter=max_iter,
                                     restart=restart, stream=self.stream)
        q, u = L.hdg_recover_ir(self.disc, self.mesh, self.X, self.uhat, stream=self.stream)
        return dict(info=info, q=q, u=u)

    def boundary(self):
        L.hdg_boundary(self.disc, self.mesh, self.uD, self.gN, self.H, self.F, self.uhat, stream=self.stream)

    def solve(self, rtol=1e-10, max_iter=200000, check_every=20, precision=0):
        return L.hdg_solve(self.disc, self.mesh, self.H, self.F, self.uhat, rtol=rtol, max_iter=max_iter,
                           check_every=check_every, precision=precision, stream=self.stream)

    def recover(self, postprocess=True):
        return L.hdg_recover(self.disc, self.mesh, self.kappa, self.tau, self.factors, self.uhat,
                             postprocess=postprocess, stream=self.stream)

    def run(self, rtol=1e-10, precision=0, method="hdg"):
        self.assemble(method=method)
        self.boundary()
        info = self.solve(rtol=rtol, precision=precision)
        q, u, us = self.recover()
        return dict(info=info, q=q, u=u, ustar=us)

    def batch_item(self):
        """This system's arrays as an item of a batched condensation (hdg_batch_create)."""
        return dict(disc=self.disc, mesh=self.mesh, kappa=self.kappa, c=self.c, f=self.f, tau=self.tau, H=self.H,
                    F=self.F, factors=self.factors)
