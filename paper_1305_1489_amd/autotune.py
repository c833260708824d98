"""Launch shapes of the batched condensation, tuned on the device and cached on disk.

The library's own tuner (``hdg_autotune``) times every candidate shape of one degree's
persistent kernel on a real batch and keeps the fastest.  This module persists the
winners in a JSON file keyed by ``"<arch>|k<degree>|<precision>"`` (e.g.
``"gfx950|k3|fp64"``), so that later batches on the same architecture start from the
tuned shape without re-timing.  An entry records the chosen shape, its time, the batch
size it was measured on and every candidate's time.
"""
from __future__ import annotations

import json
import os
import tempfile

DEFAULT_CACHE = os.environ.get("HDG_AUTOTUNE_CACHE",
                               os.path.join(os.path.expanduser("~"), ".cache", "hdg_autotune.json"))


def cache_key(arch: str, k: int, precision: str = "fp64") -> str:
    return f"{arch.split(':')[0]}|k{int(k)}|{precision}"


def load_cache(path: str = DEFAULT_CACHE) -> dict:
    try:
        with open(path) as fh:
            data = json.load(fh)
        return data if isinstance(data, dict) else {}
    except (OSError, ValueError):
        return {}


def save_cache(data: dict, path: str = DEFAULT_CACHE) -> None:
    """Atomic replace, so a concurrent reader never sees a half-written file."""
    d = os.path.dirname(os.path.abspath(path))
    os.makedirs(d, exist_ok=True)
    fd, tmp = tempfile.mkstemp(dir=d, prefix=".hdg_autotune.", suffix=".json")
    with os.fdopen(fd, "w") as fh:
        json.dump(data, fh, indent=1, sort_keys=True)
    os.replace(tmp, path)


def device_arch() -> str:
    import torch
    return torch.cuda.get_device_properties(torch.cuda.current_device()).gcnArchName.split(":")[0]


def tune_batch(batch, degrees, arch: str | None = None, cache_path: str = DEFAULT_CACHE, reps: int = 3,
               force: bool = False, precision: str = "fp64", tuner=None, apply=None, stream=None) -> dict:
    """Set a tuned launch shape for every degree in `degrees` on `batch`.

    A cached entry is applied as it is unless `force`; otherwise the tuner runs and the
    cache is updated.  `tuner(batch, k, reps, stream) -> {"best", "best_ms", "candidates"}`
    and `apply(batch, k, cfg)` default to the library calls.  Returns {k: entry}.
    """
    from . import _lib as L
    tuner = tuner or (lambda b, k, r, s: L.hdg_autotune(b, k, reps=r, stream=s))
    apply = apply or (lambda b, k, cfg: L.hdg_batch_set_config(b, k, cfg["workgroups_per_cu"], cfg["xcd_remap"],
                                                               cfg.get("waves_per_element", 1)))
    arch = arch or device_arch()
    cache = load_cache(cache_path)
    out, dirty = {}, False
    for k in sorted(set(int(x) for x in degrees)):
        key = cache_key(arch, k, precision)
        ent = cache.get(key)
        if ent is None or force:
            res = tuner(batch, k, reps, stream)
            ent = {"workgroups_per_cu": int(res["best"]["workgroups_per_cu"]),
                   "xcd_remap": int(res["best"]["xcd_remap"]),
                   "waves_per_element": int(res["best"].get("waves_per_element", 1)), "ms": float(res["best_ms"]),
                   "candidates": res.get("candidates", [])}
            cache[key] = ent
            dirty = True
        else:
            apply(batch, k, ent)
        out[k] = ent
    if dirty:
        save_cache(cache, cache_path)
    return out
