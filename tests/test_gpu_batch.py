"""Batched condensation of meshes of mixed degree: the persistent batched kernels, eager and
graph-captured, and after autotuning, give every mesh exactly (bit for bit) what a separate
hdg_assemble_condense gives it."""
import numpy as np
import pytest
import torch

from hdg_inputs import kuhn_mesh
from hdg_inputs.fields import constant_rhs_problem
from hdg_inputs.mesh import SIDES

pytestmark = pytest.mark.gpu

# (n, k, seed): every degree, ragged element counts (6 n^3 is not a multiple of 4 for odd n)
SPECS = [(3, 4, 0), (2, 1, 1), (3, 2, 2), (1, 3, 3), (2, 0, 4), (3, 3, 5), (2, 4, 6), (3, 1, 7)]


def _systems():
    from paper_1305_1489_amd import _lib as L
    from paper_1305_1489_amd.driver import HDGSystem
    discs, out = {}, []
    for n, k, seed in SPECS:
        m = kuhn_mesh(n, jitter=0.1 if n > 1 else 0.0, seed=seed, dirichlet_sides=SIDES, neumann_sides=())
        pb = constant_rhs_problem(1.0, 0.3, 500 + seed, 0.5)
        pb.tau = np.random.default_rng(seed).uniform(0.3, 2.0, size=(m.elements.shape[0], 4))
        disc = discs.setdefault(k, L.hdg_disc_create(k))
        out.append(HDGSystem(m.coordinates, m.elements, m.dirichlet, m.neumann, k, pb, disc=disc))
    return out


def _nan_fill(systems):
    for S in systems:
        S.H.fill_(float("nan"))
        S.F.fill_(float("nan"))
        S.factors.fill_(float("nan"))


def _bits(t):
    return t.view(torch.int64)


def _references(systems):
    _nan_fill(systems)
    for S in systems:
        S.assemble()
    torch.cuda.synchronize()
    return [(S.H.clone(), S.F.clone(), S.factors.clone()) for S in systems]


def _assert_same(systems, refs, what):
    for i, (S, (H, F, X)) in enumerate(zip(systems, refs)):
        assert torch.equal(_bits(S.H), _bits(H)), f"{what}: H of mesh {i} (k={S.k})"
        assert torch.equal(_bits(S.F), _bits(F)), f"{what}: F of mesh {i}"
        assert torch.equal(_bits(S.factors), _bits(X)), f"{what}: factors of mesh {i}"
        assert not torch.isnan(S.H).any() and not torch.isnan(S.F).any()


def test_batch_equals_per_mesh_launches_bitwise():
    from paper_1305_1489_amd import _lib as L
    systems = _systems()
    refs = _references(systems)
    b = L.hdg_batch_create([S.batch_item() for S in systems])
    for k in range(5):
        nm, ne = L.hdg_batch_info(b, k)
        assert nm == sum(1 for n, kk, _ in SPECS if kk == k)
        assert ne == sum(6 * n ** 3 for n, kk, _ in SPECS if kk == k)
    print("batch eager", flush=True)
    _nan_fill(systems)
    L.hdg_batch_condense(b)
    torch.cuda.synchronize()
    _assert_same(systems, refs, "eager")
    # every launch shape gives the same bits
    for wpc, remap, waves in ((1, 0, 1), (3, 1, 2), (16, 1, 8), (2, 0, 4)):
        for k in range(5):
            L.hdg_batch_set_config(b, k, wpc, remap, waves if k in (0, 4) else 1)
        _nan_fill(systems)
        L.hdg_batch_condense(b)
        torch.cuda.synchronize()
        _assert_same(systems, refs, f"eager wpc={wpc} remap={remap} waves={waves}")


def test_batch_graph_replays_and_autotune():
    from paper_1305_1489_amd import _lib as L
    systems = _systems()
    refs = _references(systems)
    b = L.hdg_batch_create([S.batch_item() for S in systems])
    print("batch graph", flush=True)
    for rep in range(3):
        _nan_fill(systems)  # eager work between the replays
        torch.cuda.synchronize()
        L.hdg_batch_launch(b)
        torch.cuda.synchronize()
        _assert_same(systems, refs, f"graph replay {rep}")
        systems[rep].assemble()  # unrelated eager launch on the same arrays, then restore by replay
        torch.cuda.synchronize()
    print("autotune", flush=True)
    for k in range(5):
        res = L.hdg_autotune(b, k, reps=1)
        assert len(res["candidates"]) == (16 if k in (0, 4) else 10)
        assert res["best_ms"] > 0
        keys = ("workgroups_per_cu", "xcd_remap", "waves_per_element")
        assert res["best"] in [{kk: c[kk] for kk in keys} for c in res["candidates"]]
        assert res["best_ms"] == min(c["ms"] for c in res["candidates"])
        assert L.hdg_batch_get_config(b, k) == res["best"]
    for rep in range(2):
        _nan_fill(systems)
        L.hdg_batch_launch(b)  # recaptured with the tuned shapes
        torch.cuda.synchronize()
        _assert_same(systems, refs, f"tuned graph replay {rep}")


def test_batch_rejects_bad_items():
    from paper_1305_1489_amd import _lib as L
    systems = _systems()[:2]
    items = [S.batch_item() for S in systems]
    items[1] = dict(items[1], H=items[1]["H"][:, :1, :])  # non-contiguous
    with pytest.raises(ValueError):
        L.hdg_batch_create(items)
    b = L.hdg_batch_create([S.batch_item() for S in systems])
    with pytest.raises(L.HdgError):
        L.hdg_batch_set_config(b, 1, 0, 0)
    with pytest.raises(L.HdgError):
        L.hdg_batch_set_config(b, 1, 4, 0, 2)  # the tile kernels run one wavefront per four elements
    with pytest.raises(L.HdgError):
        L.hdg_autotune(b, 2, reps=1)  # no mesh of degree 2 in this batch


def test_single_mesh_launch_shapes_bitwise():
    """hdg_assemble_condense under every library-wide launch shape gives the same bits."""
    from paper_1305_1489_amd import _lib as L
    systems = _systems()
    refs = _references(systems)
    saved = {k: L.hdg_get_launch_config(k) for k in range(5)}
    try:
        for wpc, remap, waves in ((1, 0, 1), (16, 1, 2), (3, 1, 4), (2, 0, 8)):
            for k in range(5):
                L.hdg_set_launch_config(k, wpc, remap, waves if k in (0, 4) else 1)
            _nan_fill(systems)
            for S in systems:
                S.assemble()
            torch.cuda.synchronize()
            _assert_same(systems, refs, f"single-mesh wpc={wpc} remap={remap} waves={waves}")
        with pytest.raises(L.HdgError):
            L.hdg_set_launch_config(2, 4, 1, 4)
    finally:
        for k, c in saved.items():
            L.hdg_set_launch_config(k, c["workgroups_per_cu"], c["xcd_remap"], c["waves_per_element"])


def test_workspace_condensation_equals_atomic_scatter_bitwise():
    """hdg_assemble_condense_ws (per-face sums of the stored contributions) gives the bits of
    hdg_assemble_condense (atomic adds onto zeros) for every degree, under two launch shapes;
    a short workspace is refused."""
    from paper_1305_1489_amd import _lib as L
    systems = _systems()
    saved = {k: L.hdg_get_launch_config(k) for k in range(5)}
    try:
        for wpc, remap in ((4, 1), (1, 0)):
            for k in range(1, 4):
                L.hdg_set_launch_config(k, wpc, remap, 1)
            for i, S in enumerate(systems):
                need = L.hdg_condense_workspace_size(S.disc, S.mesh)
                d2 = S.disc.d2
                # per-(element, face) upper triangles and F entries, 256-byte aligned, then
                # 48-double geometry records per element
                per_face = (4 * S.mesh.nelt * (d2 * (d2 + 1) // 2 + d2) * 8 + 255) // 256 * 256
                assert need == (per_face + 48 * 8 * S.mesh.nelt if 1 <= S.k <= 3 else 0)
                H0, F0, X0 = L.hdg_assemble_condense(S.disc, S.mesh, S.kappa, S.c, S.f, S.tau)
                H1 = torch.full_like(H0, float("nan"))
                F1 = torch.full_like(F0, float("nan"))
                X1 = torch.full_like(X0, float("nan"))
                ws = torch.full((max(need, 1) // 8,), float("nan"), dtype=torch.float64, device="cuda")
                L.hdg_assemble_condense_ws(S.disc, S.mesh, S.kappa, S.c, S.f, S.tau, H1, F1, X1,
                                           ws=ws.view(torch.uint8))
                torch.cuda.synchronize()
                what = f"mesh {i} (k={S.k}) wpc={wpc} remap={remap}"
                assert torch.equal(_bits(H0), _bits(H1)), what
                assert torch.equal(_bits(F0), _bits(F1)), what
                assert torch.equal(_bits(X0), _bits(X1)), what
                if need:
                    with pytest.raises(L.HdgError):
                        L.hdg_assemble_condense_ws(S.disc, S.mesh, S.kappa, S.c, S.f, S.tau, H1, F1, X1,
                                                   ws=ws.view(torch.uint8)[: need - 8])
    finally:
        for k, c in saved.items():
            L.hdg_set_launch_config(k, c["workgroups_per_cu"], c["xcd_remap"], c["waves_per_element"])
