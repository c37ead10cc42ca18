"""q-state Potts sweeps through the C ABI, on the label-equivalence path and
on the tile path (32-wide tiles), bit for bit against the Potts oracle:
records, spins, canonical labels and the dense cluster-size histogram."""
import math

import numpy as np
import pytest

import oracle
import paper_2302_14720_amd as sw

pytestmark = pytest.mark.gpu

FIELDS = ("sweep", "e_sum", "energy", "m_sum", "n_clusters", "max_cluster", "sum_sq_sizes")


def _same_records(a, b, where):
    assert len(a) == len(b), where
    for f in FIELDS:
        bad = np.nonzero(a[f] != b[f])[0]
        assert bad.size == 0, f"{where} field {f}: first mismatch at record {bad[0]}: {a[f][bad[0]]} vs {b[f][bad[0]]}"
    assert np.array_equal(a["hist_log2"], b["hist_log2"]), f"{where} hist_log2"


def _potts(L, q, beta, seed, **kw):
    print(f"\n[case] Potts q={q} L={L} beta={beta} seed={seed} {kw}", flush=True)
    return sw.Sim(L, beta, 1.0, seed, q=q, flags=sw.SW_FLAG_LABEL_EQUIV, **kw)


@pytest.mark.parametrize("q", [2, 3, 4, 8])
@pytest.mark.parametrize("L", [32, 64, 96])
def test_matches_oracle(q, L):
    seed, n = 300 + q + L, 10
    for beta in (math.log(1.0 + math.sqrt(q)), 0.4, 2.5):
        T = oracle.potts_threshold(beta, 1.0)
        sp = oracle.potts_init(L, seed, q)
        ref = oracle.potts_run(L, 1.0, T, q, seed, 0, n - 1, sp)
        last, lab = oracle.potts_sweep(L, 1.0, T, q, seed, n - 1, sp)
        with _potts(L, q, beta, seed) as s:
            assert s.threshold == T
            s.sweep(4)
            s.sweep(n - 4)
            got = s.series(0, n)
            _same_records(got[: n - 1], ref, f"q={q} L={L} beta={beta}")
            _same_records(got[n - 1:], np.array([last], dtype=got.dtype), f"q={q} L={L} last")
            assert np.array_equal(s.spins(), sp)
            assert np.array_equal(s.labels(), lab)


def test_cold_start_and_resume():
    L, q, seed = 64, 3, 12
    beta = math.log(1.0 + math.sqrt(q))
    T = oracle.potts_threshold(beta, 1.0)
    sp = oracle.potts_init(L, seed, q, cold=True)
    ref = oracle.potts_run(L, 1.0, T, q, seed, 0, 6, sp)
    with _potts(L, q, beta, seed, init=sw.SW_INIT_COLD) as s:
        assert np.all(s.spins() == 0)
        s.sweep(6)
        _same_records(s.series(0, 6), ref, "cold")
        assert np.array_equal(s.spins(), sp)
        # resume from a host state at sweep 40
        state = np.random.default_rng(3).integers(0, q, L * L).astype(np.int8)
        s.set_spins(state, 40)
        s.sweep(3)
        ref2 = oracle.potts_run(L, 1.0, T, q, seed, 40, 3, state)
        _same_records(s.series(40, 3), ref2, "resumed")
        assert np.array_equal(s.spins(), state)
        with pytest.raises(sw.SwError):
            s.set_spins(np.full(L * L, q, dtype=np.int8), 0)


def test_potts_configuration_errors():
    with pytest.raises(sw.SwError) as e:
        sw.Sim(64, 1.0, 1.0, 1, q=5, tile=64)  # q > 4 needs 32-wide tiles
    assert e.value.code == sw.SW_EINVAL
    with pytest.raises(sw.SwError) as e:
        sw.Sim(64, 1.0, 1.0, 1, q=9, flags=sw.SW_FLAG_LABEL_EQUIV)
    assert e.value.code == sw.SW_EINVAL
    with pytest.raises(sw.SwError) as e:
        sw.Sim(64, 1.0, 1.0, 1, q=1, flags=sw.SW_FLAG_LABEL_EQUIV)
    assert e.value.code == sw.SW_EINVAL


def _potts_tile(L, q, beta, seed, **kw):
    print(f"\n[case] Potts tile path q={q} L={L} beta={beta} seed={seed} {kw}", flush=True)
    return sw.Sim(L, beta, 1.0, seed, q=q, **kw)


@pytest.mark.parametrize("q", [2, 3, 4, 5, 8])
@pytest.mark.parametrize("L,tile", [(32, 0), (96, 0), (160, 0), (64, 0), (192, 0), (128, 32)])
def test_tile_path_matches_oracle(q, L, tile):
    """Several tiles, ragged tile counts (96 = 3 tiles of 32, 192 = 3 tiles of
    64), periodic wrap; 64-wide tiles for q <= 4 when L allows, else 32-wide;
    beta 0 (no bonds), the critical point, an ordered phase."""
    seed, n = 500 + q + L, 9
    want_tile = tile if tile else (64 if q <= 4 and L % 64 == 0 else 32)
    for beta in (0.0, math.log(1.0 + math.sqrt(q)), 0.4, 2.5):
        T = oracle.potts_threshold(beta, 1.0)
        sp = oracle.potts_init(L, seed, q)
        ref = oracle.potts_run(L, 1.0, T, q, seed, 0, n - 1, sp)
        last, lab = oracle.potts_sweep(L, 1.0, T, q, seed, n - 1, sp)
        with _potts_tile(L, q, beta, seed, tile=tile, flags=sw.SW_FLAG_LABELS | sw.SW_FLAG_DENSE_HIST) as s:
            assert s.threshold == T and s.tile == want_tile
            s.sweep(2)
            s.sweep(n - 2)
            got = s.series(0, n)
            _same_records(got[: n - 1], ref, f"tile q={q} L={L} beta={beta}")
            _same_records(got[n - 1:], np.array([last], dtype=got.dtype), f"tile q={q} L={L} last")
            assert np.array_equal(s.spins(), sp)
            assert np.array_equal(s.labels(), lab)
            h = s.cluster_hist()
            assert int((h * np.arange(len(h))).sum()) == L * L and h.sum() == last["n_clusters"]


def test_tile_path_cold_start_resume_and_label_equivalence_agree():
    L, q, seed = 128, 4, 21
    beta = math.log(1.0 + math.sqrt(q))
    T = oracle.potts_threshold(beta, 1.0)
    sp = oracle.potts_init(L, seed, q, cold=True)
    ref = oracle.potts_run(L, 1.0, T, q, seed, 0, 7, sp)
    with _potts_tile(L, q, beta, seed, init=sw.SW_INIT_COLD) as s, _potts(L, q, beta, seed, init=sw.SW_INIT_COLD) as le:
        s.sweep(7)
        le.sweep(7)
        _same_records(s.series(0, 7), ref, "tile cold")
        _same_records(le.series(0, 7), ref, "label-equivalence cold")
        assert np.array_equal(s.spins(), sp) and np.array_equal(le.spins(), sp)
        state = np.random.default_rng(8).integers(0, q, L * L).astype(np.int8)
        s.set_spins(state, 1000)
        s.sweep(3)
        ref2 = oracle.potts_run(L, 1.0, T, q, seed, 1000, 3, state)
        _same_records(s.series(1000, 3), ref2, "tile resumed")
        assert np.array_equal(s.spins(), state)


@pytest.mark.parametrize("q", [3, 6])
def test_tile_path_large_lattice(q):
    """L = 4096 (4096 tiles of 64 for q = 3, 16384 of 32 for q = 6): two
    sweeps bit for bit from a GPU checkpoint after 20 sweeps; every record
    passes the integer invariants."""
    L, seed = 4096, 77
    beta = math.log(1.0 + math.sqrt(q))
    T = oracle.potts_threshold(beta, 1.0)
    with _potts_tile(L, q, beta, seed) as s:
        s.sweep(20)
        state = s.spins()
        assert state.min() >= 0 and state.max() < q
        s.sweep(2)
        recs = s.series(0, 22)
        ref = oracle.potts_run(L, 1.0, T, q, seed, 20, 2, state)
        _same_records(recs[20:], ref, "L=4096 checkpoint")
        assert np.array_equal(s.spins(), state)
        assert np.all(recs["e_sum"] <= 2 * L * L) and np.all(recs["m_sum"] >= L * L // q)
        assert np.all(recs["hist_log2"].sum(axis=1) == recs["n_clusters"])


def test_tile_path_headline_lattice_one_step():
    """The benchmark's Potts leg (q = 3 at ln(1 + sqrt 3), L = 16384, 64-wide
    tiles, hot start seed 11): the GPU chain runs to sweep 10, and sweep 10
    is compared with one oracle sweep from the GPU's own state -- record,
    spins and every site's canonical label."""
    L, q, seed, t = 16384, 3, 11, 10
    beta = math.log(1.0 + math.sqrt(q))
    T = oracle.potts_threshold(beta, 1.0)
    with _potts_tile(L, q, beta, seed, flags=sw.SW_FLAG_LABELS) as s:
        assert s.threshold == T and s.tile == 64
        s.sweep(t)
        state = s.spins()
        s.sweep(1)
        rec = s.series(t, 1)
        final = s.spins()
        lab = s.labels()
    ref, olab = oracle.potts_sweep(L, 1.0, T, q, seed, t, state)
    assert rec[0].tobytes() == ref.tobytes()
    assert np.array_equal(final, state)
    del state, final
    bad = np.nonzero(lab != olab)[0]
    assert bad.size == 0, f"labels differ at {bad.size} sites, first {bad[0]}"
