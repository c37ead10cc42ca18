"""Batched replicas through the C ABI: every replica's records and spins
must be bit for bit those of a plain sim with the same parameters (which the
parity tests tie to the oracle), and small replicas are also compared with
the oracle directly."""
import math

import numpy as np
import pytest

import oracle
import paper_2302_14720_amd as sw
from paper_2302_14720_amd.replicas import grid_table

pytestmark = pytest.mark.gpu

BETA_C = math.log(1.0 + math.sqrt(2.0)) / 2.0
FIELDS = ("sweep", "e_sum", "energy", "m_sum", "n_clusters", "max_cluster", "sum_sq_sizes")


def _same_records(a, b, where):
    assert len(a) == len(b), where
    for f in FIELDS:
        bad = np.nonzero(a[f] != b[f])[0]
        assert bad.size == 0, f"{where} field {f}: first mismatch at record {bad[0]}"
    assert np.array_equal(a["hist_log2"], b["hist_log2"]), f"{where} hist_log2"


def _batch(L, beta, seed, **kw):
    print(f"\n[case] batch n={len(L)} L={list(L)[:8]} {kw}", flush=True)
    return sw.Batch(L, beta, 1.0, seed, **kw)


def _plain(L, beta, seed, n, chunks=None, tile=0, cold=False):
    with sw.Sim(int(L), float(beta), 1.0, int(seed), tile=tile,
                init=sw.SW_INIT_COLD if cold else sw.SW_INIT_HOT) as s:
        for c in (chunks or [n]):
            s.sweep(c)
        return s.series(0, n), s.spins()


def test_mixed_batch_matches_plain_and_oracle():
    L = [64, 128, 192, 256, 64, 320, 128]
    beta = [BETA_C, 0.30, 0.60, BETA_C, 0.0, 0.45, 5.0]
    seed = [11, 12, 13, 14, 15, 16, 17]
    n = 25
    with _batch(L, beta, seed) as b:
        assert b.tile == 64
        b.sweep(3)
        b.sweep(n - 3)
        last = b.observables()
        for r in range(len(L)):
            assert b.threshold(r) == oracle.threshold(beta[r], 1.0)
            got = b.series(r, 0, n)
            ref, sp = _plain(L[r], beta[r], seed[r], n)
            _same_records(got, ref, f"replica {r}")
            assert np.array_equal(b.spins(r), sp), f"replica {r} spins"
            assert last[r].tobytes() == got[-1].tobytes()
            if L[r] <= 128:
                osp = oracle.init(L[r], seed[r])
                orec = oracle.run(L[r], 1.0, oracle.threshold(beta[r], 1.0), seed[r], 0, n, osp)
                _same_records(got, orec, f"replica {r} vs oracle")
                assert np.array_equal(b.spins(r), osp)


def test_tile32_batch_and_cold_start():
    L = [32, 96, 64, 160]
    beta = [0.35, BETA_C, 0.5, BETA_C]
    seed = [21, 22, 23, 24]
    n = 20
    with _batch(L, beta, seed, init=sw.SW_INIT_COLD, tile=32) as b:
        assert b.tile == 32
        b.sweep(n)
        for r in range(len(L)):
            ref, sp = _plain(L[r], beta[r], seed[r], n, tile=32, cold=True)
            _same_records(b.series(r, 0, n), ref, f"replica {r}")
            assert np.array_equal(b.spins(r), sp)


def test_reset_replays_the_same_chain():
    L, beta, seed = [64, 128, 256], [0.41, 0.44, 0.47], [5, 6, 7]
    with _batch(L, beta, seed) as b:
        b.sweep(7)
        first = [b.series(r, 0, 7) for r in range(3)]
        b.reset()
        assert b.next_sweep == 0
        b.sweep(2)
        b.sweep(5)
        for r in range(3):
            _same_records(b.series(r, 0, 7), first[r], f"replica {r} after reset")


def test_grid_workload_sampled_replicas():
    """The 256-replica temperature grid at its full sizes: a few sweeps of the
    whole batch; sampled replicas against plain sims, every replica against
    the record invariants."""
    L, beta, seed = grid_table()
    n = 4
    with _batch(L, beta, seed) as b:
        b.sweep(n)
        recs = b.observables()
        for r in (0, 1, 2, 3, 4, 9, 130, 254, 255):
            ref, sp = _plain(L[r], beta[r], seed[r], n)
            _same_records(b.series(r, 0, n), ref, f"replica {r}")
            assert np.array_equal(b.spins(r), sp)
    N = L.astype(np.int64) ** 2
    assert np.all(recs["sweep"] == n - 1)
    assert np.all((recs["e_sum"] - 2 * N) % 4 == 0)
    assert np.all((recs["m_sum"] - N) % 2 == 0)
    assert np.all(recs["hist_log2"].sum(axis=1) == recs["n_clusters"])
    assert np.all(recs["max_cluster"] <= N) and np.all(recs["n_clusters"] >= 1)


def test_batch_errors():
    with pytest.raises(sw.SwError) as e:
        sw.Batch([64, 100], 0.4, 1.0, 1)
    assert e.value.code == sw.SW_EINVAL and "replica 1" in str(e.value)
    with pytest.raises(sw.SwError):
        sw.Batch([64], -1.0, 1.0, 1)
    with _batch([64, 64], [0.4, 0.4], [1, 2]) as b:
        with pytest.raises(sw.SwError) as e:
            b.observables()
        assert e.value.code == sw.SW_ESTATE
        b.sweep(1)
        with pytest.raises(sw.SwError) as e:
            b.series(2, 0, 1)
        assert e.value.code == sw.SW_ERANGE
        with pytest.raises(sw.SwError) as e:
            b.series(0, 0, 2)
        assert e.value.code == sw.SW_ERANGE


def test_autotuner_picks_an_allowed_tile(tmp_path, monkeypatch):
    from paper_2302_14720_amd import autotune

    monkeypatch.setenv("SWMI_TUNE_CACHE", str(tmp_path / "tune.json"))
    L = [64, 128, 256]
    tile, ms = autotune.tune_batch(L, [0.41, 0.44, 0.47], 1.0, [1, 2, 3], sweeps=4, warmup=1)
    assert tile in (32, 64) and set(ms) == {32, 64} and all(v > 0 for v in ms.values())
    assert ms[tile] == min(ms.values())
    again, _ = autotune.tune_batch(L, [0.41, 0.44, 0.47], 1.0, [1, 2, 3])
    assert again == tile  # served from the cache
    t2, ms2 = autotune.tune_sim(96, 0.44, sweeps=3, warmup=1)
    assert t2 == 32 and set(ms2) == {32}
    # the tuned tile changes no bit
    with _batch(L, [0.41, 0.44, 0.47], [1, 2, 3], tile=tile) as b1, \
            _batch(L, [0.41, 0.44, 0.47], [1, 2, 3], tile=96 - tile) as b2:
        b1.sweep(6)
        b2.sweep(6)
        for r in range(3):
            _same_records(b1.series(r, 0, 6), b2.series(r, 0, 6), f"replica {r}")
            assert np.array_equal(b1.spins(r), b2.spins(r))


@pytest.mark.parametrize("qs,L,want_tile", [
    ([2, 3, 4, 3, 2], [64, 128, 192, 64, 256], 64),        # q <= 4, multiples of 64
    ([3, 5, 8, 2], [64, 96, 128, 160], 0),                 # q above 4 or L % 64 != 0: mixed widths
])
def test_potts_batch_matches_plain_and_oracle(qs, L, want_tile):
    """A batch of Potts replicas (mixed q and L): every replica's records and
    spins are those of a plain Potts sim, and for the small ones of the Potts
    oracle."""
    n = len(L)
    beta = [math.log(1.0 + math.sqrt(q)) if i % 2 == 0 else 0.4 + 0.3 * i for i, q in enumerate(qs)]
    seed = [600 + i for i in range(n)]
    sweeps = 12
    print(f"\n[case] Potts batch q={qs} L={L}", flush=True)
    with sw.Batch(L, beta, 1.0, seed, q=qs) as b:
        assert b.tile == want_tile
        b.sweep(5)
        b.sweep(sweeps - 5)
        for r in range(n):
            assert b.threshold(r) == oracle.potts_threshold(beta[r], 1.0)
            got = b.series(r, 0, sweeps)
            with sw.Sim(L[r], beta[r], 1.0, seed[r], q=qs[r], tile=b.replica_tile(r)) as s:
                s.sweep(sweeps)
                ref, sp = s.series(0, sweeps), s.spins()
            _same_records(got, ref, f"replica {r}")
            assert np.array_equal(b.spins(r), sp), f"replica {r} spins"
            if L[r] <= 128:
                osp = oracle.potts_init(L[r], seed[r], qs[r])
                orec = oracle.potts_run(L[r], 1.0, oracle.potts_threshold(beta[r], 1.0), qs[r], seed[r], 0,
                                        sweeps, osp)
                _same_records(got, orec, f"replica {r} vs oracle")
                assert np.array_equal(b.spins(r), osp)


def test_potts_batch_errors():
    with pytest.raises(sw.SwError) as e:
        sw.Batch([64, 128], 0.5, 1.0, [1, 2], q=[3, 9])
    assert e.value.code == sw.SW_EINVAL
    with pytest.raises(sw.SwError) as e:
        sw.Batch([64, 128], 0.5, 1.0, [1, 2], q=[3, 6], tile=64)
    assert e.value.code == sw.SW_EINVAL


def test_per_replica_tiles_and_merges_match_plain():
    """Replicas with their own tile width and merge (LDS-resident or global),
    Ising and Potts in one batch: four launch groups, every replica's bits
    those of a plain sim; the same table with every merge global gives the
    same bits."""
    L = [64, 96, 128, 256, 512, 64, 128, 192]
    q = [0, 0, 0, 0, 0, 3, 5, 2]
    tiles = [64, 32, 32, 64, 64, 64, 32, 64]
    merge = [sw.SW_MERGE_LDS, sw.SW_MERGE_AUTO, sw.SW_MERGE_GLOBAL, sw.SW_MERGE_LDS, sw.SW_MERGE_AUTO,
             sw.SW_MERGE_LDS, sw.SW_MERGE_LDS, sw.SW_MERGE_GLOBAL]
    beta = [BETA_C, 0.3, 0.6, BETA_C, 0.45, 1.0050525, 0.9, 0.5]
    seed = [700 + i for i in range(len(L))]
    n = 15
    with _batch(L, beta, seed, q=q, tiles=tiles, merge=merge) as b, \
            _batch(L, beta, seed, q=q, tiles=tiles, merge=sw.SW_MERGE_GLOBAL) as g:
        assert b.tile == 0
        want_merge = [sw.SW_MERGE_LDS, sw.SW_MERGE_LDS, sw.SW_MERGE_GLOBAL, sw.SW_MERGE_LDS, sw.SW_MERGE_GLOBAL,
                      sw.SW_MERGE_LDS, sw.SW_MERGE_LDS, sw.SW_MERGE_GLOBAL]
        for r in range(len(L)):
            assert b.replica_tile(r) == tiles[r] and b.replica_merge(r) == want_merge[r], f"replica {r}"
            assert g.replica_merge(r) == sw.SW_MERGE_GLOBAL
        b.sweep(4)
        b.sweep(n - 4)
        g.sweep(n)
        for r in range(len(L)):
            got = b.series(r, 0, n)
            with sw.Sim(L[r], beta[r], 1.0, seed[r], q=q[r], tile=tiles[r]) as s:
                s.sweep(n)
                ref, sp = s.series(0, n), s.spins()
            _same_records(got, ref, f"replica {r}")
            _same_records(g.series(r, 0, n), ref, f"replica {r}, global merge")
            assert np.array_equal(b.spins(r), sp), f"replica {r} spins"
            assert np.array_equal(g.spins(r), sp), f"replica {r} spins, global merge"


def test_lds_merge_on_giant_and_empty_clusters():
    """The LDS merge at the extremes: a cold start (one cluster spanning every
    tile of a 16-tile replica), beta = 0 (no bonds: only tile-interior
    clusters), and a replica of one tile (every edge wraps onto itself)."""
    L = [256, 256, 64, 128]
    beta = [BETA_C, 0.0, 5.0, 3.0]
    seed = [801, 802, 803, 804]
    n = 6
    for init in (sw.SW_INIT_COLD, sw.SW_INIT_HOT):
        with _batch(L, beta, seed, init=init, merge=sw.SW_MERGE_LDS) as b:
            b.sweep(n)
            for r in range(len(L)):
                assert b.replica_merge(r) == sw.SW_MERGE_LDS
                ref, sp = _plain(L[r], beta[r], seed[r], n, cold=init == sw.SW_INIT_COLD)
                _same_records(b.series(r, 0, n), ref, f"init {init} replica {r}")
                assert np.array_equal(b.spins(r), sp), f"init {init} replica {r} spins"


def test_per_side_autotuner_choices(tmp_path, monkeypatch):
    """The per-side tuner returns, for every replica, a tile width and a
    merge that the replica allows, caches them, and the batch built from
    them runs (its bits are covered by the per-replica test above)."""
    from paper_2302_14720_amd import autotune

    monkeypatch.setenv("SWMI_TUNE_CACHE", str(tmp_path / "tune.json"))
    L = [64, 256, 96, 64, 512]
    q = [0, 0, 0, 3, 0]
    tiles, merges, table = autotune.tune_batch_per_side(L, 0.44, 1.0, [1, 2, 3, 4, 5], q=q, sweeps=3, warmup=1)
    for r in range(len(L)):
        assert (int(tiles[r]), int(merges[r])) in autotune._options(L[r], q[r]), f"replica {r}"
        assert (L[r], q[r]) in table
    assert int(tiles[2]) == 32 and int(merges[4]) == sw.SW_MERGE_GLOBAL
    again = autotune.tune_batch_per_side(L, 0.44, 1.0, [1, 2, 3, 4, 5], q=q)
    assert np.array_equal(again[0], tiles) and np.array_equal(again[1], merges)
    with _batch(L, 0.44, [1, 2, 3, 4, 5], q=q, tiles=tiles, merge=merges) as b:
        b.sweep(3)
        assert int(b.observables()[0]["sweep"]) == 2
