"""Replica tables for batched runs (inputs only: no part of a sweep).

``grid_table`` is the temperature-scan workload the batched path is measured
on: n replicas, replica r at beta_k = beta_lo + (beta_hi - beta_lo) * k / 31
with k = r // 8 (a 32-point grid, endpoints included, eight replicas per
temperature), lattice side {64, 128, 256, 512, 1024}[r mod 5] and seed
base_seed + r.  Deterministic, so a batched run and per-replica plain runs
see identical inputs.
"""
from __future__ import annotations

import numpy as np

SIDES = (64, 128, 256, 512, 1024)


def grid_table(n: int = 256, base_seed: int = 1000, beta_lo: float = 0.40, beta_hi: float = 0.48,
               sides=SIDES):
    """(L, beta, seed) arrays of an n-replica temperature grid."""
    r = np.arange(n)
    k = r // 8
    beta = beta_lo + (beta_hi - beta_lo) * k / 31.0
    L = np.asarray(sides, dtype=np.int32)[r % len(sides)]
    seed = (base_seed + r).astype(np.uint64)
    return L, beta.astype(np.float64), seed
