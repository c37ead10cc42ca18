"""Autotuner for the tile side (32 or 64 sites) a lattice or a replica table
is labelled in.

The choice changes no result -- only speed: 64-wide tiles move less data
across tile edges, 32-wide tiles give small lattices more workgroups.  The
tuner times a few sweeps of every allowed choice on the current GPU, keeps
the fastest, and caches the decision per device and workload in a JSON file
(``$SWMI_TUNE_CACHE``, default ``~/.cache/paper_2302_14720_amd/tune.json``).
"""
from __future__ import annotations

import hashlib
import json
import os
import time

import numpy as np

from . import SW_INIT_HOT, Batch, Sim


def cache_path() -> str:
    return os.environ.get("SWMI_TUNE_CACHE",
                          os.path.join(os.path.expanduser("~"), ".cache", "paper_2302_14720_amd", "tune.json"))


def _load() -> dict:
    try:
        with open(cache_path()) as f:
            return json.load(f)
    except (OSError, ValueError):
        return {}


def _store(key: str, entry: dict) -> None:
    path = cache_path()
    data = _load()
    data[key] = entry
    os.makedirs(os.path.dirname(path), exist_ok=True)
    tmp = path + ".tmp"
    with open(tmp, "w") as f:
        json.dump(data, f, indent=1, sort_keys=True)
    os.replace(tmp, path)


def _device() -> str:
    import torch

    return torch.cuda.get_device_name(torch.cuda.current_device())


def _time(make, warmup: int, sweeps: int) -> float:
    """Milliseconds per sweep of a fresh Sim or Batch built by make()."""
    import torch

    obj = make()
    try:
        obj.sweep(warmup)
        obj.sync()
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        obj.sweep(sweeps)
        obj.sync()
        return (time.perf_counter() - t0) * 1e3 / sweeps
    finally:
        obj.close()


def tune_batch(L, beta, J=1.0, seed=0, *, sweeps: int = 10, warmup: int = 3, use_cache: bool = True):
    """Tile side for a replica table; returns (tile, {tile: ms per sweep})."""
    La = np.asarray(L, dtype=np.int32)
    options = [64, 32] if np.all(La % 64 == 0) else [32]
    digest = hashlib.sha1(np.sort(La).tobytes()).hexdigest()[:16]
    key = f"{_device()}|batch|n={La.size}|L={digest}"
    if use_cache:
        hit = _load().get(key)
        if hit and int(hit["tile"]) in options:
            return int(hit["tile"]), {int(k): v for k, v in hit["ms"].items()}
    ms = {t: _time(lambda t=t: Batch(La, beta, J, seed, init=SW_INIT_HOT, ring=64, tile=t), warmup, sweeps)
          for t in options}
    best = min(ms, key=ms.get)
    _store(key, {"tile": best, "ms": {str(k): v for k, v in ms.items()}})
    return best, ms


def tune_sim(L: int, beta: float, J: float = 1.0, seed: int = 0, *, sweeps: int = 10, warmup: int = 3,
             use_cache: bool = True):
    """Tile side for one lattice; returns (tile, {tile: ms per sweep})."""
    options = [64, 32] if L % 64 == 0 else [32]
    key = f"{_device()}|sim|L={L}"
    if use_cache:
        hit = _load().get(key)
        if hit and int(hit["tile"]) in options:
            return int(hit["tile"]), {int(k): v for k, v in hit["ms"].items()}
    ms = {t: _time(lambda t=t: Sim(L, beta, J, seed, tile=t, ring=64), warmup, sweeps) for t in options}
    best = min(ms, key=ms.get)
    _store(key, {"tile": best, "ms": {str(k): v for k, v in ms.items()}})
    return best, ms
