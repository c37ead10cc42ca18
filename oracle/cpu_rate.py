"""Rate of the CPU oracle on bounded samples of the benchmark workloads.

TEST INFRASTRUCTURE: this times the plain sequential oracle as the reported
CPU baseline; it is never part of the product path.  It runs as a child
process (``python -m oracle.cpu_rate``) so that its worker processes start
from an interpreter that has never touched the GPU, and prints one JSON
object:

* ``L64``    -- L = 64, beta_c, hot start seed 1, all 1000 sweeps, one core;
* ``L1024``  -- L = 1024 at beta = 0.30, beta_c, 0.60 (seeds 10, 11, 12), hot
  start, the first ``--l1024-sweeps`` of the 2000 sweeps each, one core;
* ``L16384`` -- L = 16384, beta_c, hot start seed 4, ``--l16384-sweeps``
  sweeps, one core (the rate of the 200-sweep run is extrapolated from them);
* ``phi4_L28`` -- the O(4) phi^4 multicluster update on the 28^4 lattice at
  kappa = 0.304, hot start, ``--phi4-sweeps`` updates, one core;
* ``grid``   -- the 256-replica temperature grid, ``--grid-sweeps`` sweeps
  of every replica, replicas spread over ``--cores`` worker processes (one
  sequential oracle each, largest replicas first onto the least loaded
  worker); the rate is total site updates over the wall time of the pool.

Every rate is site updates (sites x sweeps) per second of wall time.
"""
from __future__ import annotations

import argparse
import json
import math
import multiprocessing as mp
import os
import sys
import time

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
if ROOT not in sys.path:
    sys.path.insert(0, ROOT)

BETA_C = math.log(1.0 + math.sqrt(2.0)) / 2.0


def _chain(L: int, beta: float, seed: int, sweeps: int) -> float:
    """Seconds for `sweeps` oracle sweeps of one hot-start lattice."""
    import oracle

    T = oracle.threshold(beta, 1.0)
    spins = oracle.init(L, seed)
    t0 = time.perf_counter()
    oracle.run(L, 1.0, T, seed, 0, sweeps, spins)
    return time.perf_counter() - t0


def _worker(jobs):
    return sum(_chain(L, beta, seed, n) for (L, beta, seed, n) in jobs)


def single(L: int, betas, seeds, sweeps: int) -> dict:
    secs = [_chain(L, b, s, sweeps) for b, s in zip(betas, seeds)]
    total = sum(secs)
    return {"value": len(secs) * L * L * sweeps / total, "unit": "site-updates/s", "cores": 1,
            "L": L, "betas": list(betas), "seeds": list(seeds), "sweeps_each": sweeps, "seconds": total}


def phi4(L: int, kappa: float, seed: int, sweeps: int) -> dict:
    """The O(4) phi^4 multicluster oracle on the L^4 lattice, one core."""
    import oracle

    phi = oracle.phi4_init(4, L, seed)
    t0 = time.perf_counter()
    oracle.phi4_run(4, L, kappa, seed, 0, sweeps, phi)
    dt = time.perf_counter() - t0
    return {"value": L ** 4 * sweeps / dt, "unit": "site-updates/s", "cores": 1, "L": L, "kappa": kappa,
            "seed": seed, "sweeps": sweeps, "seconds": dt}


def grid(sweeps: int, cores: int) -> dict:
    from paper_2302_14720_amd.replicas import grid_table

    L, beta, seed = grid_table(256, 1000)
    jobs = sorted(((int(L[r]), float(beta[r]), int(seed[r]), sweeps) for r in range(len(L))),
                  key=lambda j: -j[0])
    bins = [[] for _ in range(cores)]
    load = [0] * cores
    for j in jobs:  # largest first onto the least loaded worker
        w = load.index(min(load))
        bins[w].append(j)
        load[w] += j[0] * j[0]
    sites = int(sum(int(x) ** 2 for x in L))
    ctx = mp.get_context("fork")
    t0 = time.perf_counter()
    with ctx.Pool(cores) as pool:
        busy = pool.map(_worker, bins)
    wall = time.perf_counter() - t0
    return {"value": sites * sweeps / wall, "unit": "site-updates/s", "cores": cores,
            "replicas": len(L), "sites": sites, "sweeps_each": sweeps, "seconds": wall,
            "worker_busy_seconds": [round(b, 3) for b in busy]}


def main() -> int:
    ap = argparse.ArgumentParser(description=__doc__)
    ap.add_argument("--cores", type=int, default=0, help="worker processes of the grid leg (0: all usable, at most 16)")
    ap.add_argument("--l1024-sweeps", type=int, default=20)
    ap.add_argument("--l16384-sweeps", type=int, default=1)
    ap.add_argument("--grid-sweeps", type=int, default=10)
    ap.add_argument("--phi4-sweeps", type=int, default=5)
    args = ap.parse_args()
    usable = len(os.sched_getaffinity(0))
    cores = args.cores or min(usable, 16)
    out = {"usable_cores": usable}
    out["L64"] = single(64, [BETA_C], [1], 1000)
    out["L1024"] = single(1024, [0.30, BETA_C, 0.60], [10, 11, 12], args.l1024_sweeps)
    out["L16384"] = single(16384, [BETA_C], [4], args.l16384_sweeps)
    out["grid"] = grid(args.grid_sweeps, cores)
    out["phi4_L28"] = phi4(28, 0.304, 6028, args.phi4_sweeps)
    print(json.dumps(out))
    return 0


if __name__ == "__main__":
    sys.exit(main())
