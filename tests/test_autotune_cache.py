"""The JSON cache of tuned launch shapes (host logic only; the tuner is replaced by a stub)."""
import json

from paper_1305_1489_amd import autotune as AT


def _stub(calls):
    def tuner(batch, k, reps, stream):
        calls.append(("tune", k, reps))
        return {"best": {"workgroups_per_cu": 2 * k + 1, "xcd_remap": k % 2}, "best_ms": 0.5 * k,
                "candidates": [{"workgroups_per_cu": 1, "xcd_remap": 0, "ms": 1.0}]}

    def apply(batch, k, cfg):
        calls.append(("apply", k, cfg["workgroups_per_cu"], cfg["xcd_remap"]))
    return tuner, apply


def test_key_format_strips_target_features():
    assert AT.cache_key("gfx950:sramecc+:xnack-", 3) == "gfx950|k3|fp64"
    assert AT.cache_key("gfx950", 1, "fp32ir") == "gfx950|k1|fp32ir"


def test_tune_then_reuse_then_force(tmp_path):
    path = str(tmp_path / "tune.json")
    calls = []
    tuner, apply = _stub(calls)
    out = AT.tune_batch(None, [3, 1, 3], arch="gfx950", cache_path=path, reps=2, tuner=tuner, apply=apply)
    assert calls == [("tune", 1, 2), ("tune", 3, 2)]
    assert out[3]["workgroups_per_cu"] == 7 and out[3]["xcd_remap"] == 1
    data = json.load(open(path))
    assert set(data) == {"gfx950|k1|fp64", "gfx950|k3|fp64"}
    assert data["gfx950|k1|fp64"]["ms"] == 0.5
    # a second batch on the same architecture reuses the cached shapes without timing
    calls.clear()
    out2 = AT.tune_batch(None, [1, 3, 4], arch="gfx950", cache_path=path, tuner=tuner, apply=apply)
    assert calls == [("apply", 1, 3, 1), ("apply", 3, 7, 1), ("tune", 4, 3)]
    assert out2[1] == out[1]
    # another architecture, or force, re-tunes
    calls.clear()
    AT.tune_batch(None, [1], arch="gfx942", cache_path=path, tuner=tuner, apply=apply)
    AT.tune_batch(None, [1], arch="gfx950", cache_path=path, tuner=tuner, apply=apply, force=True)
    assert calls == [("tune", 1, 3), ("tune", 1, 3)]
    assert set(json.load(open(path))) == {"gfx950|k1|fp64", "gfx950|k3|fp64", "gfx950|k4|fp64", "gfx942|k1|fp64"}


def test_unreadable_cache_is_empty(tmp_path):
    p = tmp_path / "bad.json"
    p.write_text("{not json")
    assert AT.load_cache(str(p)) == {}
    assert AT.load_cache(str(tmp_path / "missing.json")) == {}
