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
