"""Learned face-graph preconditioner: parameters, training loop, checkpoints.

The network, its loss and its gradient run in the library's kernels (hdg_gnn_*).  This
module holds the parameter vector, draws the probe vectors and calls Adam; checkpoints are
written and read by the library (hdg_gnn_save, hdg_gnn_load: the safetensors layout).

Training data follows the log-normal workload family: Kuhn cubes n ~ U{8..16}, degree 2,
kappa = exp(1.5 g) with a fresh Gaussian random field per system (correlation length
0.1), c = 0.1, f = 1, homogeneous Dirichlet data, tau = 1.  Each system is generated,
condensed, used for `steps_per_system` optimiser steps, and dropped.

    python -m paper_1305_1489_amd.gnn --systems 2000 --out <checkpoint.safetensors>
"""
from __future__ import annotations

import argparse
import json
import math
import time

import torch

from . import _lib as L

F0 = 5


def param_layout(d2: int, hidden: int, layers: int):
    """(name, shape) in the library's order (hdg_gnn_param_count is the authority)."""
    h, fe = hidden, d2 * d2
    lay = [("W0", (h, F0)), ("c0", (h,)), ("We", (h, fe)), ("ce", (h,))]
    for l in range(layers):
        lay += [(f"Wm{l}", (h, 3 * h)), (f"cm{l}", (h,)), (f"Wu{l}", (h, 2 * h)), (f"cu{l}", (h,))]
    fb = d2 * (d2 + 1) // 2
    lay += [("Wo", (fe, 3 * h)), ("co", (fe,)), ("Wb", (fb, h)), ("cb", (fb,))]
    return lay


class LearnedPreconditioner:
    def __init__(self, d2: int, hidden: int = 32, layers: int = 3, seed: int = 0, device="cuda", params=None):
        self.d2, self.hidden, self.layers = d2, hidden, layers
        self.shape = (d2, hidden, layers)
        self.device = torch.device(device)
        n = L.hdg_gnn_param_count(self.shape)
        if params is None:
            gen = torch.Generator().manual_seed(seed)
            parts = []
            for name, sh in param_layout(d2, hidden, layers):
                if name.startswith("W") and name not in ("Wo", "Wb"):  # He initialisation; both heads start at zero
                    parts.append(torch.randn(sh, generator=gen, dtype=torch.float64).ravel() * math.sqrt(2.0 / sh[1]))
                else:
                    parts.append(torch.zeros(int(torch.tensor(sh).prod())), )
            params = torch.cat([p.double() for p in parts]).float()
        if params.numel() != n:
            raise ValueError(f"parameter vector has {params.numel()} entries, the shape needs {n}")
        self.params = params.to(self.device).contiguous()
        self.meta = {}
        self._ws = {}

    # ---- inference
    def prepare(self, disc, mesh, H, stream=None):
        """Graph of the system, the factor N and the block scaling B (for
        hdg_solve(..., learned=(N, B, graph)))."""
        g = L.hdg_gnn_build_graph(disc, mesh, H, stream=stream)
        N, B = L.hdg_gnn_forward(self.shape, self.params, mesh, g, ws=self._workspace(mesh, 0), stream=stream)
        return g, N, B

    def _workspace(self, mesh, nprobe):
        key = (id(mesh), nprobe)
        if key not in self._ws:
            self._ws = {key: L.hdg_gnn_workspace(self.shape, mesh, nprobe)}  # one system at a time
        return self._ws[key]

    def loss(self, mesh, graph, nprobe=16, seed=0):
        z = self.probes(mesh, nprobe, seed)
        loss, _, _, _ = L.hdg_gnn_loss_grad(self.shape, self.params, mesh, graph, z, want_grad=False,
                                            ws=self._workspace(mesh, nprobe))
        return float(loss.item())

    def probes(self, mesh, nprobe, seed):
        gen = torch.Generator(device=self.device).manual_seed(int(seed))
        z = torch.randint(0, 2, (nprobe, mesh.nfc, self.d2), generator=gen, device=self.device, dtype=torch.int32)
        return (2 * z - 1).float().contiguous()

    # ---- training
    def train(self, systems, steps_per_system=1, lr=1e-3, nprobe=8, seed=0, log=None):
        """systems: iterable of (disc, mesh, H) (H after hdg_boundary).  Returns the loss history."""
        m = torch.zeros_like(self.params)
        v = torch.zeros_like(self.params)
        grad = torch.empty_like(self.params)
        hist, t = [], 0
        t0 = time.perf_counter()
        for si, (disc, mesh, H) in enumerate(systems):
            g = L.hdg_gnn_build_graph(disc, mesh, H)
            ws = self._workspace(mesh, nprobe)
            for _ in range(steps_per_system):
                t += 1
                z = self.probes(mesh, nprobe, seed * 1000003 + t)
                loss, _, _, _ = L.hdg_gnn_loss_grad(self.shape, self.params, mesh, g, z, grad=grad, ws=ws)
                L.hdg_gnn_adam(self.params, grad, m, v, t, lr=lr)
                hist.append(loss)
            if log and (si + 1) % 100 == 0:
                torch.cuda.synchronize()
                log(f"system {si + 1}: loss {hist[-1].item():.5f}, {time.perf_counter() - t0:.1f} s")
        torch.cuda.synchronize()
        self.meta.update(train_steps=t, train_seconds=time.perf_counter() - t0, lr=lr, nprobe=nprobe)
        return [float(x.item()) for x in hist]

    # ---- checkpoints
    def save(self, path):
        """Through the library's checkpoint writer (safetensors layout, metadata as JSON strings)."""
        meta = {k: json.dumps(v) for k, v in self.meta.items()}
        L.hdg_gnn_save(path, self.shape, self.params, meta)

    @classmethod
    def load(cls, path, device="cuda"):
        (d2, hidden, layers), params = L.hdg_gnn_load(path)
        obj = cls(d2, hidden, layers, device=device, params=params)
        obj.meta = {}
        for key in ("systems", "train_seconds", "train_steps", "first_loss", "last_loss", "lr", "nprobe", "data"):
            try:
                obj.meta[key] = json.loads(L.hdg_gnn_checkpoint_meta(path, key))
            except L.HdgError:
                pass
        return obj


def generated_systems(count, n_range=(8, 16), k=2, field_seed0=10000, seed=0, sigma=1.5, corr=0.1, c=0.1):
    """Fresh condensed systems of the log-normal family, one at a time."""
    import numpy as np
    from hdg_inputs import kuhn_mesh
    from hdg_inputs.fields import constant_rhs_problem
    from hdg_inputs.mesh import SIDES
    from .driver import HDGSystem
    rng = np.random.Generator(np.random.PCG64(seed))
    disc = L.hdg_disc_create(k)
    meshes = {}
    for i in range(count):
        n = int(rng.integers(n_range[0], n_range[1] + 1))
        if n not in meshes:
            meshes[n] = kuhn_mesh(n, dirichlet_sides=SIDES, neumann_sides=())
        m = meshes[n]
        S = HDGSystem(m.coordinates, m.elements, m.dirichlet, m.neumann, k,
                      constant_rhs_problem(sigma, corr, field_seed0 + i, c), disc=disc)
        S.assemble()
        S.boundary()
        yield S.disc, S.mesh, S.H


def main():
    ap = argparse.ArgumentParser(description=__doc__, formatter_class=argparse.RawDescriptionHelpFormatter)
    ap.add_argument("--systems", type=int, default=2000)
    ap.add_argument("--steps-per-system", type=int, default=1)
    ap.add_argument("--hidden", type=int, default=32)
    ap.add_argument("--layers", type=int, default=3)
    ap.add_argument("--lr", type=float, default=1e-3)
    ap.add_argument("--nprobe", type=int, default=8)
    ap.add_argument("--seed", type=int, default=0)
    ap.add_argument("--out", required=True)
    a = ap.parse_args()
    lp = LearnedPreconditioner(6, a.hidden, a.layers, seed=a.seed)
    hist = lp.train(generated_systems(a.systems, seed=a.seed), a.steps_per_system, a.lr, a.nprobe, a.seed,
                    log=lambda s: print(s, flush=True))
    lp.meta.update(systems=a.systems, first_loss=hist[0], last_loss=sum(hist[-50:]) / min(50, len(hist)),
                   data="log-normal family: n ~ U{8..16}, k=2, kappa=exp(1.5 g), corr. length 0.1, "
                        "field seeds 10000+i, c=0.1, f=1, all Dirichlet")
    lp.save(a.out)
    print(json.dumps(lp.meta), flush=True)


if __name__ == "__main__":
    main()
