"""Host-side pieces of the learned preconditioner: parameter layout, checkpoints."""
import torch

from oracle import gnn as OGN
from paper_1305_1489_amd import _lib as L
from paper_1305_1489_amd.gnn import LearnedPreconditioner, param_layout


def test_layout_agrees_with_library_and_oracle():
    for d2, h, l in ((6, 32, 3), (3, 8, 0), (10, 64, 4), (1, 5, 1)):
        lay = param_layout(d2, h, l)
        n = sum(int(torch.tensor(sh).prod()) for _, sh in lay)
        assert n == L.hdg_gnn_param_count((d2, h, l))
        assert lay == OGN.param_layout(OGN.Shape(d2, h, l))


def test_shape_errors():
    import pytest
    for bad in ((5, 32, 3), (6, 0, 3), (6, 65, 3), (6, 32, 9)):
        with pytest.raises(L.HdgError):
            L.hdg_gnn_param_count(bad)


def test_checkpoint_round_trip(tmp_path):
    lp = LearnedPreconditioner(6, hidden=8, layers=2, seed=3, device="cpu")
    # both heads (Wo, co, Wb, cb) start at zero, the other weights are random
    lay = param_layout(6, 8, 2)
    assert [n for n, _ in lay[-4:]] == ["Wo", "co", "Wb", "cb"]
    o = sum(int(torch.tensor(sh).prod()) for _, sh in lay[:-4])
    assert not lp.params[o:].any() and lp.params[:o].abs().sum() > 0
    lp.meta.update(systems=7, train_seconds=1.5)
    p = str(tmp_path / "g.safetensors")
    lp.save(p)
    lq = LearnedPreconditioner.load(p, device="cpu")
    assert (lq.d2, lq.hidden, lq.layers) == (6, 8, 2)
    assert torch.equal(lq.params, lp.params)
    assert lq.meta["systems"] == 7 and lq.meta["train_seconds"] == 1.5


def test_packaged_checkpoint_loads():
    import os
    from bench import GNN_CHECKPOINT
    assert os.path.exists(GNN_CHECKPOINT)
    lp = LearnedPreconditioner.load(GNN_CHECKPOINT, device="cpu")
    assert lp.d2 == 6 and lp.meta.get("systems") == 2000
    assert torch.isfinite(lp.params).all()
    assert lp.meta["last_loss"] < lp.meta["first_loss"]  # training lowered the objective


def test_checkpoint_io_agrees_with_the_safetensors_library(tmp_path):
    """The library's checkpoint writer and reader against the independent safetensors
    package: files written by either are read by the other with the same values and
    metadata, and the packaged checkpoint loads in both."""
    from safetensors import safe_open
    from safetensors.torch import save_file
    from bench import GNN_CHECKPOINT
    shape = (6, 8, 2)
    n = L.hdg_gnn_param_count(shape)
    params = torch.randn(n, generator=torch.Generator().manual_seed(5))
    p1 = str(tmp_path / "lib.safetensors")
    L.hdg_gnn_save(p1, shape, params, {"note": 'quoted "text" \\ and\nnewline', "systems": "7"})
    with safe_open(p1, framework="pt") as fh:
        meta = fh.metadata()
        assert torch.equal(fh.get_tensor("params"), params)
    assert meta["d2"] == "6" and meta["hidden"] == "8" and meta["layers"] == "2"
    assert meta["note"] == 'quoted "text" \\ and\nnewline' and meta["systems"] == "7"
    p2 = str(tmp_path / "ref.safetensors")
    save_file({"params": params}, p2, metadata={"d2": "6", "hidden": "8", "layers": "2", "x": "y"})
    shp, h = L.hdg_gnn_load(p2)
    assert shp == shape and torch.equal(h, params)
    assert L.hdg_gnn_checkpoint_meta(p2, "x") == "y"
    shp, h = L.hdg_gnn_load(GNN_CHECKPOINT)
    with safe_open(GNN_CHECKPOINT, framework="pt") as fh:
        assert torch.equal(fh.get_tensor("params"), h)
    import pytest
    with pytest.raises(L.HdgError):
        L.hdg_gnn_save(p1, (6, 8, 3), params)  # count does not match the shape
    bad = tmp_path / "bad.safetensors"
    bad.write_bytes(b"\x05\x00\x00\x00\x00\x00\x00\x00{oops")
    with pytest.raises(L.HdgError):
        L.hdg_gnn_load(str(bad))
