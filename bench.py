"""Benchmark: Swendsen-Wang site-updates/s of the 2D Ising model at
L = 16384, beta_c, on one MI355X.

One step = one full sweep of the lattice (bond formation, cluster labelling,
new cluster spins, per-sweep record: Sec. 2 of the paper).  The timed region
is `steps` consecutive sweeps of one device-resident lattice, issued as one
sw_sweep call (graph-replayed sweeps plus the closing pass that leaves final
+-1 spins and measures them), bracketed by device synchronisation.

Prints one JSON line.  Besides the headline rate it reports the roofline of
the dominant kernel (per-kernel durations from HIP events on the sim's own
stream, in a profiled continuation of the same chain), the cold-start rate of
the first sweeps, and the CPU oracle's rate on a bounded sample.
"""
from __future__ import annotations

import argparse
import hashlib
import json
import math
import os
import sys
import time

ROOT = os.path.dirname(os.path.abspath(__file__))
if ROOT not in sys.path:
    sys.path.insert(0, ROOT)

METRIC = "SW site-updates/s at L=16384 βc (1 GPU, % HBM roofline); batched vs plain"
BETA_C = math.log(1.0 + math.sqrt(2.0)) / 2.0

# MI355X published peaks
HBM_PEAK_GBS = 8000.0
# Integer VALU peak: 256 CUs x 4 SIMDs x 32 lanes x 2.4 GHz = 78.6 Tops/s,
# one 32-bit op per lane per clock: the lane rate behind the published
# 157.3 TFLOP/s FP32 vector peak (an FMA is two flops).  A wave64 VALU
# instruction takes a SIMD two clocks.
ALU_PEAK_TOPS = 256 * 4 * 32 * 2.4e9 / 1e12

# Algorithmic work of k_tile per site.  Bytes: the spin byte read and the
# spin byte written.  Integer ops: Philox4x32-10 costs 10 rounds x (2 wide
# multiplies + 4 xors) = 60 ops per call; a site needs 1/2 call for its two
# bond words plus 1/TW of a call for the flip bits of its tile row.
TILE_BYTES_PER_SITE = 2.0
# Stream model of one sweep of a bond / label / flip pipeline, bytes per
# site-update: bonds 2 (spin in, mask out), labels 5 (mask in, 32-bit label
# out), flip 5 (label in, spin out).
MODEL_BYTES_PER_SITE = 12.0
PHILOX_OPS = 60.0
# Paths with 32-bit labels in HBM, algorithmic bytes per site and sweep.
# Label equivalence: bonds 2 (spins in, mask out), label init 4, every pass
# 9 (scan: mask 1 + label 4; analysis: label 4), roots 4, flip 6 (labels 4,
# new spin 1 gathered, spin 1 out), statistics 5 (spin 1, label 4).
# Cubic bricks: bricks 6 (spin 1 in, mask 1 and label 4 out), face unions
# 27/16 (3/16 of the sites on a +face: mask 1, two labels 8), flatten 1
# (mask), relabel 10 (mask 1, label 4 in and out, spin 1 out), statistics 5.
LE_BYTES_FIXED, LE_BYTES_PER_PASS = 21.0, 9.0
BRICK_BYTES_PER_SITE = 6.0 + 27.0 / 16.0 + 1.0 + 10.0 + 5.0


def hbm_fields(rate: float, bytes_per_site: float) -> dict:
    gbs = rate * bytes_per_site / 1e9
    return {"algorithmic_bytes_per_site": bytes_per_site, "hbm_GBs": gbs, "hbm_frac": gbs / HBM_PEAK_GBS}


def kernel_source_sha() -> str:
    p = os.path.join(ROOT, "paper_2302_14720_amd", "csrc", "sw_kernels.hip")
    with open(p, "rb") as f:
        return hashlib.sha256(f.read()).hexdigest()


def load_counters(L: int):
    """The committed rocprofv3 counter summary of k_tile (HBM bytes and
    instruction counts per launch), if it was taken on the current kernel
    source; else None."""
    p = os.path.join(ROOT, "profiles", f"k_tile_L{L}_counters.json")
    if not os.path.exists(p):
        return None
    with open(p) as f:
        d = json.load(f)
    if d.get("kernel_source_sha256") != kernel_source_sha():
        return None
    return d


# Instruction-throughput ceilings of the chip for wave64 integer work, as
# measured by throughput probes (independent add/xor chains: 1.35 VALU
# wave-instructions per CU per clock; scalar chains: 0.86 SALU per CU per
# clock, issued beside the VALU), at the 2.4 GHz clock.
VALU_ISSUE_PEAK = 256 * 2.4e9 * 1.35
SALU_ISSUE_PEAK = 256 * 2.4e9 * 0.86


def cpu_baseline(args):
    """The sequential C oracle timed on bounded samples of the workloads, in a
    child process that never touches the GPU (oracle/cpu_rate.py): the
    headline lattice, L = 64 and L = 1024 on one core each, and the
    256-replica grid over all usable host cores (at most 16)."""
    import subprocess

    cmd = [sys.executable, "-m", "oracle.cpu_rate", "--l16384-sweeps", "1",
           "--l1024-sweeps", str(args.cpu_l1024_sweeps), "--grid-sweeps", str(args.cpu_grid_sweeps)]
    res = subprocess.run(cmd, cwd=ROOT, capture_output=True, text=True, timeout=900)
    if res.returncode != 0:
        raise RuntimeError(f"oracle timing failed: {res.stderr[-2000:]}")
    legs = json.loads(res.stdout.strip().splitlines()[-1])
    head = legs["L16384"]
    return {
        "value": head["value"],
        "unit": "site-updates/s",
        "cores": 1,
        "kind": "oracle",
        "sample": f"one sweep of the L=16384 beta_c lattice from a hot start (seed 4), sequential C "
                  f"oracle on one core, {head['seconds']:.1f} s; the 200-sweep rate is extrapolated from it",
        "legs": {
            "L64_beta_c_1000_sweeps_1_core": legs["L64"],
            "L1024_three_betas_1_core": legs["L1024"],
            "grid_256_replicas_all_cores": legs["grid"],
            "phi4_L28_kappa_0.304_1_core": legs["phi4_L28"],
        },
        "usable_host_cores": legs["usable_cores"],
    }


def batched_vs_plain(args):
    """The 256-replica temperature grid swept as one batch (the kernels of a
    sweep launched once per launch group for all replicas, tile width and
    merge autotuned per lattice side) and as 256 plain sims (one sw_sweep(n)
    per replica stream, and one sw_sweep(1) per replica per sweep)."""
    import torch

    import paper_2302_14720_amd as sw
    from paper_2302_14720_amd.replicas import grid_table

    from paper_2302_14720_amd import autotune

    L, beta, seed = grid_table(256, 1000)
    sites = int((L.astype("int64") ** 2).sum())
    tiles, merges, tune = autotune.tune_batch_table(L, beta, 1.0, seed, sweeps=10, use_cache=False)
    tune_ms = tune["per_side"]
    choice = {int(side): {"tile": int(tiles[L == side][0]),
                          "merge": "lds" if int(merges[L == side][0]) == sw.SW_MERGE_LDS else "global"}
              for side in sorted(set(L.tolist()))}
    print(f"[bench] batched: {len(L)} replicas, {sites} sites; autotuned {tune['choice']}: {choice} "
          f"(whole-table candidates, ms per sweep: {tune['batch']})", file=sys.stderr, flush=True)
    b = sw.Batch(L, beta, 1.0, seed, tiles=tiles, merge=merges)
    b.sweep(args.warmup)
    b.sync()
    t0 = time.perf_counter()
    b.sweep(args.batch_steps)
    b.sync()
    bdt = time.perf_counter() - t0
    recs = b.observables()
    assert int(recs["sweep"][0]) == args.warmup + args.batch_steps - 1
    b.close()
    print(f"[bench] batched: {bdt * 1e3:.2f} ms for {args.batch_steps} sweeps", file=sys.stderr, flush=True)

    # plain: one sim per replica, each on its own stream, driven by one
    # sw_sweep(n) per replica (n sweeps replayed from the sim's own graph)
    sims = [sw.Sim(int(L[r]), float(beta[r]), 1.0, int(seed[r])) for r in range(len(L))]
    for s_ in sims:
        s_.sweep(2)
    for s_ in sims:
        s_.sync()
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    for s_ in sims:
        s_.sweep(args.batch_steps)
    for s_ in sims:
        s_.sync()
    pdt = time.perf_counter() - t0
    # the same sims driven one sweep at a time, replica after replica (as a
    # caller that steps every replica in lockstep would)
    t0 = time.perf_counter()
    for _ in range(args.plain_steps):
        for s_ in sims:
            s_.sweep(1)
    for s_ in sims:
        s_.sync()
    idt = time.perf_counter() - t0
    for s_ in sims:
        s_.close()
    print(f"[bench] plain: {pdt * 1e3:.2f} ms for {args.batch_steps} sweeps per replica stream; "
          f"{idt * 1e3:.2f} ms for {args.plain_steps} lockstep sweeps", file=sys.stderr, flush=True)
    bval = sites * args.batch_steps / bdt
    pval = sites * args.batch_steps / pdt
    ival = sites * args.plain_steps / idt
    return {
        "workload": "256 replicas, L = {64,128,256,512,1024}[r mod 5], beta_k = 0.40 + 0.08 k/31 "
                    "(k = r // 8), seed 1000 + r, hot start, J = 1",
        "replicas": len(L), "sites": sites, "per_side": choice, "autotune_choice": tune["choice"],
        "autotune_table_ms_per_sweep": tune["batch"],
        "autotune_ms_per_sweep": {f"L={k[0]}": {f"tile{t}_{'lds' if m == sw.SW_MERGE_LDS else 'global'}": v
                                                for (t, m), v in ms.items()} for k, ms in tune_ms.items()},
        "value": bval, "unit": "site-updates/s", "sweeps": args.batch_steps,
        "ms_per_step": bdt * 1e3 / args.batch_steps,
        "plain": {"how": "256 plain sims, each on its own stream, one sw_sweep(n) call per replica",
                  "value": pval, "sweeps": args.batch_steps, "ms_per_step": pdt * 1e3 / args.batch_steps},
        "plain_lockstep": {"how": "the same sims, one sw_sweep(1) per replica per sweep",
                           "value": ival, "sweeps": args.plain_steps, "ms_per_step": idt * 1e3 / args.plain_steps},
        "batched_over_plain": bval / pval,
        "batched_over_plain_lockstep": bval / ival,
    }


def potts_tile(args):
    """The q = 3 Potts model on the tile path at its critical point
    ln(1 + sqrt 3), headline lattice, hot start; per-kernel times from the
    measurement entry point."""
    import paper_2302_14720_amd as sw

    q, L = 3, args.L
    beta_q = math.log(1.0 + math.sqrt(q))
    s = sw.Sim(L, beta_q, 1.0, 11, q=q)
    s.sweep(10)
    s.sync()
    t0 = time.perf_counter()
    s.sweep(args.potts_steps)
    s.sync()
    dt = time.perf_counter() - t0
    prof = s.profile(5)
    tw = s.tile
    s.close()
    out = {"workload": f"2D q=3 Potts, L={L} periodic, J=1, beta=ln(1+sqrt 3), hot start seed 11, "
                       f"tile path ({tw}-wide tiles)",
           "value": L * L * args.potts_steps / dt, "unit": "site-updates/s", "sweeps": args.potts_steps,
           "ms_per_step": dt * 1e3 / args.potts_steps, "kernel_ms": prof}
    print(f"[bench] Potts q=3 tile path L={L}: {out['value']:.4g} site-updates/s, kernel ms {prof}",
          file=sys.stderr, flush=True)
    return out


CUBIC_WORKLOADS = (("ising", 0, 0.2216544), ("potts_q3", 3, 0.5505))

# The paper's own SW timing experiment (its Sec. 5 table): 10^4 sweeps at
# k_B T = 2.5 (beta = 0.4 with J = 1) for L = 128 .. 4096, GPU minutes on its
# Tesla P100.  Context only: other hardware, other code.
PAPER_SW_GPU_MINUTES = {128: 0.112, 256: 0.151, 512: 0.390, 1024: 1.472, 2048: 5.483, 4096: 22.440}


def paper_table(args):
    """The paper's timing experiment re-run here: 10^4 sweeps (by default) at
    beta = 0.4 from a hot start for each lattice side of its table."""
    import paper_2302_14720_amd as sw

    out = {"sweeps": args.paper_sweeps, "beta": 0.4, "unit": "minutes", "rows": []}
    for L, paper_min in PAPER_SW_GPU_MINUTES.items():
        s = sw.Sim(L, 0.4, 1.0, 2500 + L)
        s.sweep(5)
        s.sync()
        t0 = time.perf_counter()
        s.sweep(args.paper_sweeps)
        s.sync()
        dt = time.perf_counter() - t0
        s.close()
        minutes = dt / 60.0 * 1e4 / args.paper_sweeps  # scaled to the table's 10^4 sweeps
        out["rows"].append({"L": L, "minutes_per_1e4_sweeps": minutes, "site_updates_per_s": L * L * args.paper_sweeps / dt,
                            "paper_p100_minutes": paper_min, "ratio_to_paper": paper_min / minutes})
        print(f"[bench] paper table L={L}: {minutes:.4f} min per 10^4 sweeps (paper on P100: {paper_min} min)",
              file=sys.stderr, flush=True)
    return out


def cubic(args):
    """The simple cubic lattice on 16^3 bricks (the default 3D path): 3D
    Ising at its critical coupling (numerical estimate 0.2216544) and 3D q = 3
    Potts near its transition, L = 512 (134 M sites), hot start."""
    import paper_2302_14720_amd as sw

    L = 512
    out = {"unit": "site-updates/s", "sites": L ** 3}
    for name, q, beta in CUBIC_WORKLOADS:
        s = sw.Sim(L, beta, 1.0, 13, q=q, dims=3)
        s.sweep(3)
        s.sync()
        t0 = time.perf_counter()
        s.sweep(args.cubic_steps)
        s.sync()
        dt = time.perf_counter() - t0
        prof = s.profile(3)
        s.close()
        out[name] = {"workload": f"3D {'Ising' if q == 0 else 'q=3 Potts'}, L={L} periodic, J=1, beta={beta}, "
                                 f"hot start seed 13, 16^3 bricks",
                     "value": L ** 3 * args.cubic_steps / dt, "ms_per_step": dt * 1e3 / args.cubic_steps,
                     "sweeps": args.cubic_steps,
                     "roofline": hbm_fields(L ** 3 * args.cubic_steps / dt, BRICK_BYTES_PER_SITE),
                     "kernel_ms": {"bricks": prof["tile"], "face_unions_and_flatten": prof["union"],
                                   "spins_and_sizes": prof["flatten"], "statistics": prof["roots"],
                                   "record": prof["record"]}}
        print(f"[bench] cubic {name} L={L}: {out[name]['value']:.4g} site-updates/s, {out[name]['kernel_ms']}",
              file=sys.stderr, flush=True)
    return out


def serving(args):
    """Continuous batching: jobs arrive as a Poisson process (L log-uniform in
    [128, 4096] rounded to 32, beta uniform in [0.35, 0.55], sweeps uniform in
    [100, 10^4], seeded), wait for room in a 16 GiB device pool, and are swept
    together; latency = finish - arrival on the host clock."""
    import numpy as np

    import paper_2302_14720_amd as sw

    rng = np.random.default_rng(2024)
    n = args.serve_jobs
    gaps = rng.exponential(1.0 / args.serve_rate, n)
    arrive = np.cumsum(gaps) - gaps[0]
    L = (np.round(np.exp(rng.uniform(np.log(128), np.log(4096), n)) / 32).astype(int) * 32).clip(128, 4096)
    beta = rng.uniform(0.35, 0.55, n)
    sweeps = rng.integers(100, 10001, n)
    work = int((L.astype(np.int64) ** 2 * sweeps).sum())
    print(f"[bench] serving: {n} jobs, {work:.3e} site-updates", file=sys.stderr, flush=True)
    srv = sw.Server(16 << 30, max_jobs=256)
    t0 = time.perf_counter()
    nxt, finish, ids = 0, {}, {}
    while len(finish) < n:
        now = time.perf_counter() - t0
        while nxt < n and arrive[nxt] <= now:
            ids[srv.submit(int(L[nxt]), float(beta[nxt]), 1.0, 5000 + nxt, int(sweeps[nxt]))] = nxt
            nxt += 1
        st = srv.status()
        if st["active"] == 0 and st["queued"] == 0:
            time.sleep(max(0.0, min(0.01, arrive[nxt] - now)))
            continue
        for jid in srv.step(20):
            finish[ids[jid]] = time.perf_counter() - t0
            srv.release(jid)
    span = time.perf_counter() - t0
    srv.close()
    lat = np.array([finish[i] - arrive[i] for i in range(n)])
    return {
        "workload": f"{n} jobs, Poisson arrivals at {args.serve_rate} jobs/s, L log-uniform in [128, 4096] "
                    "(multiples of 32), beta U[0.35, 0.55], sweeps U[100, 10000], hot start, 16 GiB pool",
        "jobs": n, "site_updates": work, "makespan_s": span,
        "value": work / span, "unit": "site-updates/s",
        "latency_p50_s": float(np.percentile(lat, 50)), "latency_p99_s": float(np.percentile(lat, 99)),
    }


# The paper's phi^4 timing experiment (its Sec. 5 table): 10^4 multicluster
# updates at kappa = 0.304 on L^4 lattices, GPU minutes on its Tesla P100.
# Context only: other hardware, other code.
PAPER_PHI4_GPU_MINUTES = {16: 0.186, 20: 0.305, 24: 0.619, 28: 1.188}
PHI4_KAPPA = 0.304
# Algorithmic bytes per site and update of the five phi^4 kernels: fields
# 32 B in and projection 8 B, parent and size out (projections); five
# projections in (bonds); root in and out (flatten); fields in and out,
# root and projection in (reflection); five fields, root and size in (record).
PHI4_BYTES_PER_SITE = (32 + 8 + 4 + 4) + 40 + 8 + (32 + 32 + 4 + 8) + (5 * 32 + 8)


def phi4(args):
    """The 4D O(4) phi^4 multicluster update (unit fields) at kappa = 0.304
    on the paper's lattice sides, hot start; per-kernel times from the
    measurement entry point; the paper's P100 times for context."""
    import paper_2302_14720_amd as sw

    out = {"kappa": PHI4_KAPPA, "unit": "site-updates/s", "rows": []}
    for L, paper_min in PAPER_PHI4_GPU_MINUTES.items():
        N = L ** 4
        p = sw.Phi4(L, PHI4_KAPPA, 6000 + L)
        p.sweep(20)
        p.sync()
        t0 = time.perf_counter()
        p.sweep(args.phi4_steps)
        p.sync()
        dt = time.perf_counter() - t0
        prof = p.profile(20)
        rec = p.series(p.next_sweep - 1, 1)[0]
        p.close()
        rate = N * args.phi4_steps / dt
        ms = dt * 1e3 / args.phi4_steps
        paper_ms = paper_min * 60e3 / 1e4
        out["rows"].append({
            "L": L, "sites": N, "sweeps": args.phi4_steps, "value": rate, "ms_per_step": ms,
            "kernel_ms": prof, "roofline": hbm_fields(rate, PHI4_BYTES_PER_SITE),
            "last_action_per_link": float(rec["action"]) / (4 * N),
            "paper_p100_ms_per_update": paper_ms, "ratio_to_paper": paper_ms / ms})
        print(f"[bench] phi4 L={L}: {rate:.4g} site-updates/s, {ms * 1e3:.1f} us per update "
              f"(paper on P100: {paper_ms * 1e3:.0f} us), kernel ms {prof}", file=sys.stderr, flush=True)
    return out


def serving_saturated(args):
    """Serving capacity: every job is queued at time 0 (the queue is never
    empty while jobs remain), so the GPU is never waiting for arrivals; job
    mix as in the Poisson leg (its own seed); latency = finish time."""
    import numpy as np

    import paper_2302_14720_amd as sw

    rng = np.random.default_rng(4048)
    n = args.serve_sat_jobs
    L = (np.round(np.exp(rng.uniform(np.log(128), np.log(4096), n)) / 32).astype(int) * 32).clip(128, 4096)
    beta = rng.uniform(0.35, 0.55, n)
    sweeps = rng.integers(100, 10001, n)
    work = int((L.astype(np.int64) ** 2 * sweeps).sum())
    print(f"[bench] serving (saturated): {n} jobs, {work:.3e} site-updates", file=sys.stderr, flush=True)
    srv = sw.Server(16 << 30, max_jobs=256)
    t0 = time.perf_counter()
    ids = {srv.submit(int(L[i]), float(beta[i]), 1.0, 9000 + i, int(sweeps[i])): i for i in range(n)}
    finish = {}
    while len(finish) < n:
        for jid in srv.step(20):
            finish[ids[jid]] = time.perf_counter() - t0
            srv.release(jid)
    span = time.perf_counter() - t0
    srv.close()
    lat = np.array([finish[i] for i in range(n)])
    return {
        "workload": f"{n} jobs all queued at t = 0, L log-uniform in [128, 4096] (multiples of 32), "
                    "beta U[0.35, 0.55], sweeps U[100, 10000], hot start, 16 GiB pool",
        "jobs": n, "site_updates": work, "makespan_s": span,
        "value": work / span, "unit": "site-updates/s",
        "latency_p50_s": float(np.percentile(lat, 50)), "latency_p99_s": float(np.percentile(lat, 99)),
    }


def label_equivalence(args, tile_rate):
    """The paper's own cluster formation (iterated label equivalence in
    global memory, one cooperative kernel) against the tile pipeline: the
    same sweeps, bit for bit, at the paper's 512^2 / beta = 0.4 and at the
    headline lattice; then the q = 3 Potts model and the simple cubic
    lattice, which run on that path."""
    import paper_2302_14720_amd as sw

    out = {}
    for L, beta, seed in ((512, 0.4, 7), (args.L, BETA_C, args.seed)):
        res = {}
        for name, flags in (("label_equivalence", sw.SW_FLAG_LABEL_EQUIV), ("tile", 0)):
            if name == "tile" and L == args.L:
                res[name] = tile_rate
                continue
            s = sw.Sim(L, beta, 1.0, seed, flags=flags)
            s.sweep(3)
            s.sync()
            t0 = time.perf_counter()
            s.sweep(args.le_steps)
            s.sync()
            dt = time.perf_counter() - t0
            res[name] = L * L * args.le_steps / dt
            if flags:
                res["passes_last_sweep"] = s.label_passes
                res["roofline"] = hbm_fields(res[name], LE_BYTES_FIXED + LE_BYTES_PER_PASS * s.label_passes)
            s.close()
        res["tile_over_label_equivalence"] = res["tile"] / res["label_equivalence"]
        out[f"L{L}_beta{beta:.4f}"] = res
        print(f"[bench] label equivalence L={L}: {res}", file=sys.stderr, flush=True)
    # the q = 3 Potts model (same path) at its critical point ln(1 + sqrt 3)
    q = 3
    beta_q = math.log(1.0 + math.sqrt(q))
    for L in (4096, args.L):
        s = sw.Sim(L, beta_q, 1.0, 11, q=q, flags=sw.SW_FLAG_LABEL_EQUIV)
        s.sweep(3)
        s.sync()
        t0 = time.perf_counter()
        s.sweep(args.le_steps)
        s.sync()
        dt = time.perf_counter() - t0
        rec = s.observables()
        out[f"potts_q3_L{L}"] = {"value": L * L * args.le_steps / dt, "passes_last_sweep": s.label_passes,
                                 "roofline": hbm_fields(L * L * args.le_steps / dt,
                                                        LE_BYTES_FIXED + LE_BYTES_PER_PASS * s.label_passes),
                                 # not an equilibrium value: the lattice is still relaxing from
                                 # its hot start after these few sweeps
                                 "energy_per_site_last_sweep": float(rec["energy"]) / (L * L),
                                 "sweeps_from_hot_start": 3 + args.le_steps}
        s.close()
        print(f"[bench] Potts q=3 L={L}: {out[f'potts_q3_L{L}']}", file=sys.stderr, flush=True)
    # the simple cubic lattice on this path: 3D Ising at its critical
    # coupling (numerical estimate 0.2216544) and 3D q = 3 Potts near its
    # transition (the default 16^3-brick path is timed in its own leg)
    Lc = 512
    for name, q, beta in (("cubic_ising", 0, 0.2216544), ("cubic_potts_q3", 3, 0.5505)):
        s = sw.Sim(Lc, beta, 1.0, 13, q=q, dims=3, flags=sw.SW_FLAG_LABEL_EQUIV)
        s.sweep(3)
        s.sync()
        t0 = time.perf_counter()
        s.sweep(args.le_steps)
        s.sync()
        dt = time.perf_counter() - t0
        key = f"{name}_L{Lc}"
        out[key] = {"value": Lc ** 3 * args.le_steps / dt, "sites": Lc ** 3, "beta": beta,
                    "roofline": hbm_fields(Lc ** 3 * args.le_steps / dt,
                                           LE_BYTES_FIXED + LE_BYTES_PER_PASS * s.label_passes),
                    "passes_last_sweep": s.label_passes, "sweeps_from_hot_start": 3 + args.le_steps}
        s.close()
        print(f"[bench] {key}: {out[key]}", file=sys.stderr, flush=True)
    out["unit"] = "site-updates/s"
    return out


def main() -> int:
    ap = argparse.ArgumentParser(description=__doc__)
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=200)
    ap.add_argument("--warmup", type=int, default=20)
    ap.add_argument("--L", type=int, default=16384)
    ap.add_argument("--seed", type=int, default=4)
    ap.add_argument("--profile-sweeps", type=int, default=20)
    ap.add_argument("--cold-sweeps", type=int, default=10)
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--no-extras", action="store_true",
                    help="skip the per-kernel profile and the cold-start leg (for counter runs)")
    ap.add_argument("--batch-steps", type=int, default=200,
                    help="timed sweeps of the 256-replica batch")
    ap.add_argument("--plain-steps", type=int, default=10,
                    help="timed lockstep sweeps of the same replicas as plain sims, one sw_sweep(1) per replica per sweep")
    ap.add_argument("--no-batched", action="store_true", help="skip the batched-vs-plain leg")
    ap.add_argument("--serve-jobs", type=int, default=48, help="jobs of the serving leg (0 = skip)")
    ap.add_argument("--le-steps", type=int, default=10,
                    help="timed sweeps of the label-equivalence comparison, its Potts and its "
                         "simple cubic runs (0 = skip)")
    ap.add_argument("--serve-rate", type=float, default=8.0, help="Poisson arrival rate of the serving leg, jobs/s")
    ap.add_argument("--serve-sat-jobs", type=int, default=64,
                    help="jobs of the saturated serving leg, all queued at once (0 = skip)")
    ap.add_argument("--phi4-steps", type=int, default=500,
                    help="timed multicluster updates per lattice side of the phi^4 leg (0 = skip)")
    ap.add_argument("--cpu-l1024-sweeps", type=int, default=20,
                    help="oracle sweeps per temperature of the L = 1024 CPU-baseline leg")
    ap.add_argument("--cpu-grid-sweeps", type=int, default=10,
                    help="oracle sweeps per replica of the all-cores grid CPU-baseline leg")
    ap.add_argument("--potts-steps", type=int, default=50,
                    help="timed sweeps of the q = 3 Potts model on the tile path (0 = skip)")
    ap.add_argument("--cubic-steps", type=int, default=20,
                    help="timed sweeps of the simple cubic lattice on 16^3 bricks (0 = skip)")
    ap.add_argument("--paper-sweeps", type=int, default=10000,
                    help="sweeps per lattice of the paper's timing table, L = 128..4096 at beta = 0.4 (0 = skip)")
    ap.add_argument("--calibrate-copy-mib", type=int, default=0,
                    help="first run one plain device copy of this many MiB (reference for "
                         "HBM byte counters)")
    args = ap.parse_args()

    if args.gpus != 1:
        print(f"bench.py runs on exactly one GPU; --gpus {args.gpus} is not supported "
              f"(the sweep of one lattice is a single-GPU workload here)", file=sys.stderr)
        return 2

    import torch

    import paper_2302_14720_amd as sw

    if not torch.cuda.is_available():
        print("bench.py needs a ROCm GPU", file=sys.stderr)
        return 1
    L, N = args.L, args.L * args.L
    print(f"[bench] L={L} beta_c hot start seed={args.seed}: warmup {args.warmup}, "
          f"timed {args.steps} sweeps", file=sys.stderr, flush=True)

    if args.calibrate_copy_mib > 0:
        nb = args.calibrate_copy_mib << 20
        src = torch.ones(nb, dtype=torch.uint8, device="cuda")
        dst = torch.empty_like(src)
        torch.cuda.synchronize()
        dst.copy_(src)
        torch.cuda.synchronize()
        del src, dst
        print(f"[bench] calibration copy of {nb} bytes done", file=sys.stderr, flush=True)

    sim = sw.Sim(L, BETA_C, 1.0, args.seed, init=sw.SW_INIT_HOT)
    sim.sweep(args.warmup)
    sim.sync()
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    sim.sweep(args.steps)
    sim.sync()
    torch.cuda.synchronize()
    dt = time.perf_counter() - t0
    value = N * args.steps / dt
    rec = sim.observables()
    # integer invariants of the last record
    assert (int(rec["e_sum"]) - 2 * N) % 4 == 0 and (int(rec["m_sum"]) - N) % 2 == 0
    assert int(rec["hist_log2"].sum()) == int(rec["n_clusters"])
    print(f"[bench] timed: {dt * 1e3:.2f} ms, {value:.4e} site-updates/s", file=sys.stderr, flush=True)

    tw = sim.tile
    if args.no_extras:
        sim.close()
        print(json.dumps({"metric": METRIC, "value": value, "unit": "site-updates/s", "n_gpus": 1,
                          "steps": args.steps, "warmup": args.warmup, "ms_per_step": dt * 1e3 / args.steps,
                          "note": "counter run: no per-kernel profile, cold start or CPU baseline"}))
        return 0
    prof = sim.profile(args.profile_sweeps)
    sim.close()
    print(f"[bench] kernel ms: {prof}", file=sys.stderr, flush=True)

    # cold start: the first sweeps carry one near-spanning cluster
    cold = sw.Sim(L, BETA_C, 1.0, 3, init=sw.SW_INIT_COLD)
    torch.cuda.synchronize()
    c0 = time.perf_counter()
    cold.sweep(args.cold_sweeps)
    cold.sync()
    cdt = time.perf_counter() - c0
    crec = cold.series(0, 1)[0]
    cold.close()

    per_sweep = {k: v for k, v in prof.items() if k != "resolve"}
    dom = max(per_sweep, key=per_sweep.get)
    t_dom = per_sweep[dom] * 1e-3
    # Roofline against the stream model of a bond / label / flip sweep
    # (12 B per site-update: bonds read a spin and write a mask, labelling
    # reads the mask and writes a 32-bit label, the flip reads the label and
    # writes a spin), credited to the dominant kernel, which does all three
    # for N sites per launch; and the same model over the whole timed sweep.
    model_bytes = MODEL_BYTES_PER_SITE * N
    ach = model_bytes / t_dom / 1e9
    cnt = load_counters(L)
    traffic = cnt.get("hbm_bytes_per_launch") if (cnt and dom == "tile") else None
    valu = cnt.get("valu_wave_instructions_per_launch") if (cnt and dom == "tile") else None
    salu = cnt.get("salu_wave_instructions_per_launch") if (cnt and dom == "tile") else None
    alu_ach = (0.5 + 1.0 / tw) * PHILOX_OPS * N / t_dom / 1e12
    design_ach = TILE_BYTES_PER_SITE * N / t_dom / 1e9
    roofline = {
        "bound": "hbm", "achieved": ach, "peak": HBM_PEAK_GBS, "unit": "GB/s", "frac": ach / HBM_PEAK_GBS,
        "traffic": traffic,
        "kernel": "k_tile" if dom == "tile" else dom, "kernel_ms": per_sweep[dom],
        "algorithmic_bytes_per_launch": model_bytes,
        "model": "12 B per site-update (bond 1R+1W, label 1R+4W, flip 4R+1W) x N sites per launch",
        "traffic_bytes_per_site": (traffic / N) if traffic else None,
        "whole_sweep": {"ms": dt * 1e3 / args.steps, "achieved_GBs": value * MODEL_BYTES_PER_SITE / 1e9,
                        "frac": value * MODEL_BYTES_PER_SITE / 1e9 / HBM_PEAK_GBS},
        "diagnostics": {
            # the bytes this design actually has to move in k_tile (one spin
            # byte in, one out), the Philox integer work, and the issued VALU
            # instructions against the issue ceiling
            "design_bytes_per_site": TILE_BYTES_PER_SITE, "design_GBs": design_ach,
            "design_hbm_frac": design_ach / HBM_PEAK_GBS,
            "philox_alu_Tops": alu_ach, "philox_alu_frac": alu_ach / ALU_PEAK_TOPS,
            "valu_issue_frac": (valu / t_dom / VALU_ISSUE_PEAK) if valu else None,
            "salu_issue_frac": (salu / t_dom / SALU_ISSUE_PEAK) if salu else None,
        },
    }
    # measured HBM bytes of every kernel of a sweep (committed counters of the
    # current kernel source), against the 12 B/site stream model
    sweep_hbm = None
    if cnt and cnt.get("sweep_hbm_bytes_per_site"):
        bps = cnt["sweep_hbm_bytes_per_site"]
        sweep_hbm = {"measured_bytes_per_site": bps, "model_bytes_per_site": MODEL_BYTES_PER_SITE,
                     "GBs": value * bps / 1e9, "frac": value * bps / 1e9 / HBM_PEAK_GBS}

    out = {
        "metric": METRIC,
        "value": value,
        "unit": "site-updates/s",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": dt * 1e3 / args.steps,
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "int8",
        "data": "synthetic",
        "config": {
            "workload": f"plain SW sweep, 2D Ising, L={L} periodic (N={N}), J=1, beta=beta_c, "
                        f"hot start seed {args.seed}, int8 spins, Philox4x32-10",
            "L": L, "beta": BETA_C, "J": 1.0, "tile": tw, "start": "hot",
        },
        "sweep_hbm": sweep_hbm,
        "roofline": roofline,
        "kernel_ms": prof,
        "cold_start": {"sweeps": args.cold_sweeps, "value": N * args.cold_sweeps / cdt,
                       "ms_per_step": cdt * 1e3 / args.cold_sweeps,
                       "first_sweep_max_cluster": int(crec["max_cluster"])},
        "batched": None if args.no_batched else batched_vs_plain(args),
        "serving": serving(args) if args.serve_jobs > 0 else None,
        "serving_saturated": serving_saturated(args) if args.serve_sat_jobs > 0 else None,
        "potts_tile": potts_tile(args) if args.potts_steps > 0 else None,
        "cubic": cubic(args) if args.cubic_steps > 0 else None,
        "phi4": phi4(args) if args.phi4_steps > 0 else None,
        "paper_table": paper_table(args) if args.paper_sweeps > 0 else None,
        "label_equivalence": label_equivalence(args, value) if args.le_steps > 0 else None,
    }
    if not args.no_cpu_baseline:
        print("[bench] timing the CPU oracle (one L=16384 sweep, L=64, L=1024, the replica grid)",
              file=sys.stderr, flush=True)
        out["cpu_baseline"] = cpu_baseline(args)
    print(json.dumps(out))
    return 0


if __name__ == "__main__":
    sys.exit(main())
