"""Autotuner for the tile side (32 or 64 sites) a lattice or a replica table
is labelled in, and, per lattice side of a batch, for the merge schedule
(the whole merge of a replica in one workgroup's LDS, or the global merge).

The choices change no result -- only speed: 64-wide tiles move less data
across tile edges, 32-wide tiles give small lattices more workgroups; the
LDS merge saves a small replica four launches' worth of dependent steps.
The tuner times a few sweeps of every allowed choice on the current GPU,
keeps the fastest, and caches the decision per device and workload in a JSON
file (``$SWMI_TUNE_CACHE``, default ``~/.cache/paper_2302_14720_amd/tune.json``).
"""
from __future__ import annotations

import hashlib
import json
import os
import time

import numpy as np

from . import SW_INIT_HOT, SW_MERGE_GLOBAL, SW_MERGE_LDS, Batch, Sim


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


SMALL_TILES = 16  # replicas of at most this many tiles may take the LDS merge


def _options(L: int, q: int):
    tiles = [64, 32] if (L % 64 == 0 and q <= 4) else [32]
    out = []
    for t in tiles:
        out.append((t, SW_MERGE_GLOBAL))
        if (L // t) ** 2 <= SMALL_TILES:
            out.append((t, SW_MERGE_LDS))
    return out


def tune_batch_per_side(L, beta, J=1.0, seed=0, q=None, *, sweeps: int = 10, warmup: int = 3,
                        use_cache: bool = True):
    """Tile side and merge for every replica of a table, chosen per lattice
    side (and Potts q): the replicas of each side are timed as a batch of
    their own under every allowed (tile, merge) pair and the fastest pair is
    kept.  Returns (tiles, merges, {(L, q): {(tile, merge): ms per sweep}})."""
    La = np.asarray(L, dtype=np.int32)
    n = La.size
    ba = np.broadcast_to(np.asarray(beta, dtype=np.float64), (n,))
    Ja = np.broadcast_to(np.asarray(J, dtype=np.float64), (n,))
    sa = np.broadcast_to(np.asarray(seed, dtype=np.uint64), (n,))
    qa = np.zeros(n, dtype=np.int32) if q is None else np.broadcast_to(np.asarray(q, dtype=np.int32), (n,))
    tiles = np.zeros(n, dtype=np.int32)
    merges = np.zeros(n, dtype=np.int32)
    table = {}
    for side, qq in sorted({(int(a), int(b)) for a, b in zip(La, qa)}):
        idx = np.nonzero((La == side) & (qa == qq))[0]
        key = f"{_device()}|batch-side|L={side}|q={qq}|n={idx.size}"
        opts = _options(side, qq)
        hit = _load().get(key) if use_cache else None
        if hit and tuple(hit["best"]) in opts:
            best = tuple(hit["best"])
            ms = {tuple(int(x) for x in k.split(",")): v for k, v in hit["ms"].items()}
        else:
            ms = {}
            for t, m in opts:
                ms[(t, m)] = _time(lambda t=t, m=m: Batch(La[idx], ba[idx], Ja[idx], sa[idx], init=SW_INIT_HOT,
                                                          ring=64, q=qa[idx], tiles=t, merge=m),
                                   warmup, sweeps)
            best = min(ms, key=ms.get)
            _store(key, {"best": list(best), "ms": {f"{k[0]},{k[1]}": v for k, v in ms.items()}})
        tiles[idx], merges[idx] = best
        table[(side, qq)] = ms
    return tiles, merges, table


def tune_batch_table(L, beta, J=1.0, seed=0, q=None, *, sweeps: int = 10, warmup: int = 3,
                     use_cache: bool = True):
    """Tile side and merge for every replica of a table: the per-side choices
    of tune_batch_per_side, then a check on the whole table against the same
    tiles with every merge global and against the widest allowed tile with
    either merge rule (a side that is fastest alone may cost the mixed batch
    an extra launch group or a longer merge).  Returns (tiles, merges,
    {"per_side": ..., "batch": {name: ms per sweep}, "choice": name})."""
    La = np.asarray(L, dtype=np.int32)
    n = La.size
    ba = np.broadcast_to(np.asarray(beta, dtype=np.float64), (n,))
    Ja = np.broadcast_to(np.asarray(J, dtype=np.float64), (n,))
    sa = np.broadcast_to(np.asarray(seed, dtype=np.uint64), (n,))
    qa = np.zeros(n, dtype=np.int32) if q is None else np.broadcast_to(np.asarray(q, dtype=np.int32), (n,))
    tiles, merges, per_side = tune_batch_per_side(La, ba, Ja, sa, q=qa, sweeps=sweeps, warmup=warmup,
                                                  use_cache=use_cache)
    wide = np.where((La % 64 == 0) & (qa <= 4), 64, 32).astype(np.int32)
    cands = {
        "per_side": (tiles, merges),
        "per_side_tiles_global_merge": (tiles, np.full(n, SW_MERGE_GLOBAL, dtype=np.int32)),
        "widest_tiles_auto_merge": (wide, np.zeros(n, dtype=np.int32)),
        "widest_tiles_global_merge": (wide, np.full(n, SW_MERGE_GLOBAL, dtype=np.int32)),
    }
    digest = hashlib.sha1(La.tobytes() + qa.tobytes()).hexdigest()[:16]
    key = f"{_device()}|batch-table|n={n}|{digest}"
    hit = _load().get(key) if use_cache else None
    if hit and hit.get("choice") in cands:
        ms, choice = hit["ms"], hit["choice"]
    else:
        ms = {name: _time(lambda t=t, m=m: Batch(La, ba, Ja, sa, init=SW_INIT_HOT, ring=64, q=qa, tiles=t, merge=m),
                          warmup, sweeps) for name, (t, m) in cands.items()}
        choice = min(ms, key=ms.get)
        _store(key, {"choice": choice, "ms": ms})
    t, m = cands[choice]
    return t, m, {"per_side": per_side, "batch": ms, "choice": choice}
