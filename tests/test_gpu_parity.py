"""Bit-exact parity of the HIP path (through the C ABI) with the CPU oracle.

Spins, canonical labels, cluster-size histograms and every integer field of
every per-sweep record must be identical; the FP64 energy is -J * e_sum on
both sides and must be identical too.
"""
import math

import numpy as np
import pytest

import oracle
import paper_2302_14720_amd as sw

pytestmark = pytest.mark.gpu

BETA_C = math.log(1.0 + math.sqrt(2.0)) / 2.0
FIELDS = ("sweep", "e_sum", "energy", "m_sum", "n_clusters", "max_cluster", "sum_sq_sizes")


def _assert_records(gpu, ref, where=""):
    assert len(gpu) == len(ref)
    for f in FIELDS:
        bad = np.nonzero(gpu[f] != ref[f])[0]
        assert bad.size == 0, f"{where} field {f}: first mismatch at record {bad[0]}: {gpu[f][bad[0]]} vs {ref[f][bad[0]]}"
    bad = np.nonzero((gpu["hist_log2"] != ref["hist_log2"]).any(axis=1))[0]
    assert bad.size == 0, f"{where} hist_log2 differs at record {bad[0]}"


def _oracle_run(L, beta, seed, n, cold=False, J=1.0):
    sp = oracle.init(L, seed, cold=cold)
    recs = oracle.run(L, J, oracle.threshold(beta, J), seed, 0, n, sp)
    return recs, sp


def _sim(L, beta, seed, **kw):
    print(f"\n[case] L={L} beta={beta} seed={seed} {kw}", flush=True)
    return sw.Sim(L, beta, 1.0, seed, **kw)


@pytest.mark.parametrize("beta", [0.0, 0.3, BETA_C, 0.6, 3.0])
def test_threshold_equals_oracle(beta):
    with _sim(64, beta, 1) as s:
        assert s.threshold == oracle.threshold(beta, 1.0)


@pytest.mark.parametrize("L,cold", [(32, False), (64, False), (96, True), (160, False)])
def test_initial_spins(L, cold):
    seed = 0xDEADBEEF12345
    with _sim(L, 0.4, seed, init=sw.SW_INIT_COLD if cold else sw.SW_INIT_HOT) as s:
        assert np.array_equal(s.spins(), oracle.init(L, seed, cold=cold))


def test_plain_L64_beta_c_1000_sweeps():
    """L = 64 at beta_c, hot start, 1000 sweeps; records of every sweep."""
    L, seed, n = 64, 1, 1000
    ref, sp = _oracle_run(L, BETA_C, seed, n)
    with _sim(L, BETA_C, seed) as s:
        s.sweep(1)
        s.sweep(2)
        s.sweep(n - 3)
        got = s.series(0, n)
        assert np.array_equal(s.spins(), sp)
        last = s.observables()
    _assert_records(got, ref)
    assert last.tobytes() == ref[-1].tobytes()


@pytest.mark.parametrize("L", [32, 96, 128, 160, 256])
@pytest.mark.parametrize("beta", [0.3, BETA_C, 0.6])
def test_small_lattices(L, beta):
    seed, n = 7 + L, 24
    ref, sp = _oracle_run(L, beta, seed, n)
    tiles = [0] + ([32] if L % 64 == 0 else [])
    for tile in tiles:
        with _sim(L, beta, seed, tile=tile) as s:
            for chunk in (1, 5, n - 6):
                s.sweep(chunk)
            _assert_records(s.series(0, n), ref, f"L={L} tile={s.tile}")
            assert np.array_equal(s.spins(), sp)


@pytest.mark.parametrize("L,tile", [(64, 64), (96, 32), (128, 32), (128, 64)])
def test_labels_and_dense_histogram(L, tile):
    seed, beta = 3, BETA_C
    T = oracle.threshold(beta)
    sp = oracle.init(L, seed)
    with _sim(L, beta, seed, tile=tile, flags=sw.SW_FLAG_LABELS | sw.SW_FLAG_DENSE_HIST) as s:
        for t in range(6):
            rec, lab, _, dense = oracle.sweep(L, 1.0, T, seed, t, sp, dense=True)
            s.sweep(1)
            assert np.array_equal(s.labels(), lab), f"labels differ after sweep {t}"
            assert np.array_equal(s.cluster_hist(), dense), f"dense histogram differs after sweep {t}"
            assert np.array_equal(s.spins(), sp)
            assert s.observables().tobytes() == rec.tobytes()


@pytest.mark.parametrize("beta,seed", [(0.30, 10), (BETA_C, 11), (0.60, 12)])
def test_L1024_three_temperatures(beta, seed):
    L, n = 1024, 12
    ref, sp = _oracle_run(L, beta, seed, n)
    with _sim(L, beta, seed) as s:
        s.sweep(n)
        _assert_records(s.series(0, n), ref, f"L=1024 beta={beta}")
        assert np.array_equal(s.spins(), sp)


@pytest.mark.parametrize("L", [2048, 2112])
def test_record_fold_boundary(L):
    """L = 2048: 1024 tiles, 64 groups of 16, the largest lattice whose last
    k_roots workgroup folds the record; L = 2112: 1089 tiles, 69 groups (the
    last one ragged), folded by k_record.  Cold and hot starts, every record
    and the final spins against the oracle."""
    for cold, seed in ((True, 31), (False, 32)):
        n = 4
        ref, sp = _oracle_run(L, BETA_C, seed, n, cold=cold)
        with _sim(L, BETA_C, seed, init=sw.SW_INIT_COLD if cold else sw.SW_INIT_HOT) as s:
            s.sweep(n)
            _assert_records(s.series(0, n), ref, f"L={L} cold={cold}")
            assert np.array_equal(s.spins(), sp)


def test_cold_start_giant_cluster():
    L, seed, n = 256, 3, 10
    ref, sp = _oracle_run(L, BETA_C, seed, n, cold=True)
    with _sim(L, BETA_C, seed, init=sw.SW_INIT_COLD) as s:
        s.sweep(n)
        _assert_records(s.series(0, n), ref)
        assert np.array_equal(s.spins(), sp)
    assert ref["max_cluster"][0] > 0.5 * L * L


@pytest.mark.parametrize("beta", [0.0, 5.0, 40.0])
def test_degenerate_temperatures(beta):
    """beta = 0: no bonds (every site its own cluster); large beta: almost
    every satisfied edge bonded (one cluster)."""
    L, seed, n = 128, 21, 8
    ref, sp = _oracle_run(L, beta, seed, n)
    with _sim(L, beta, seed) as s:
        s.sweep(n)
        _assert_records(s.series(0, n), ref, f"beta={beta}")
        assert np.array_equal(s.spins(), sp)
    if beta == 0.0:
        assert np.all(ref["n_clusters"] == L * L)


def test_set_spins_one_step_and_resume():
    L, seed, beta = 192, 99, BETA_C
    T = oracle.threshold(beta)
    rng = np.random.default_rng(4)
    start = rng.choice(np.array([-1, 1], dtype=np.int8), size=L * L)
    with _sim(L, beta, seed) as s:
        s.set_spins(start, 17)
        assert s.next_sweep == 17
        s.sweep(1)
        ref_sp = start.copy()
        rec, _, _ = oracle.sweep(L, 1.0, T, seed, 17, ref_sp)
        assert np.array_equal(s.spins(), ref_sp)
        assert s.observables().tobytes() == rec.tobytes()
        # checkpoint / resume: 9 straight sweeps == 4 + save + restore + 5
        s.reset(sw.SW_INIT_HOT)
        s.sweep(9)
        straight = s.spins()
        straight_recs = s.series(0, 9)
        s.reset(sw.SW_INIT_HOT)
        s.sweep(4)
        ckpt = s.spins()
    with _sim(L, beta, seed) as s2:
        s2.set_spins(ckpt, 4)
        s2.sweep(5)
        assert np.array_equal(s2.spins(), straight)
        _assert_records(s2.series(4, 5), straight_recs[4:])


def test_api_states_and_errors():
    with _sim(64, 0.4, 5) as s:
        with pytest.raises(sw.SwError) as e:
            s.observables()
        assert e.value.code == sw.SW_ESTATE
        s.sweep(0)
        with pytest.raises(sw.SwError) as e:
            s.observables()
        assert e.value.code == sw.SW_ESTATE
        s.sweep(3)
        assert s.next_sweep == 3
        with pytest.raises(sw.SwError) as e:
            s.series(0, 4)
        assert e.value.code == sw.SW_ERANGE
        with pytest.raises(sw.SwError) as e:
            s.labels()
        assert e.value.code == sw.SW_ESTATE
        bad = np.ones(64 * 64, dtype=np.int8)
        bad[5] = 0
        with pytest.raises(sw.SwError) as e:
            s.set_spins(bad, 0)
        assert e.value.code == sw.SW_EINVAL
        with pytest.raises(sw.SwError) as e:
            sw.sw_sweep(s.handle, -1)
        assert e.value.code == sw.SW_EINVAL


def test_ring_wraps():
    L, seed, n = 64, 8, 50
    ref, _ = _oracle_run(L, 0.45, seed, n)
    with _sim(L, 0.45, seed, ring=16) as s:
        s.sweep(n)
        _assert_records(s.series(n - 16, 16), ref[n - 16:])
        with pytest.raises(sw.SwError):
            s.series(n - 17, 17)


@pytest.mark.parametrize("cold", [False, True])
def test_L4096_one_step(cold):
    """Full-size tiling at L = 4096: 3 sweeps, then one more sweep compared
    with one oracle sweep from the GPU's own state."""
    L, seed = 4096, 5 if cold else 6
    T = oracle.threshold(BETA_C)
    with _sim(L, BETA_C, seed, init=sw.SW_INIT_COLD if cold else sw.SW_INIT_HOT) as s:
        s.sweep(3)
        state = s.spins()
        s.sweep(1)
        got = s.spins()
        rec = s.observables()
    rrec, _, _ = oracle.sweep(L, 1.0, T, seed, 3, state)
    assert np.array_equal(got, state)
    assert rec.tobytes() == rrec.tobytes()


@pytest.mark.parametrize("L,tile,q", [(128, 64, 0), (96, 32, 0), (128, 64, 3), (96, 32, 5)])
def test_profile_runs_the_same_sweeps(L, tile, q):
    """sw_profile launches the sweep's five stages one by one with events
    between them: the sweeps it runs are those of sw_sweep, bit for bit,
    mixed with ordinary sweeps; every stage reports a time."""
    seed, n = 31 + L + q, 9
    beta = BETA_C if q == 0 else 1.0
    if q:
        sp = oracle.potts_init(L, seed, q)
        ref = oracle.potts_run(L, 1.0, oracle.potts_threshold(beta, 1.0), q, seed, 0, n, sp)
    else:
        ref, sp = _oracle_run(L, beta, seed, n)
    with _sim(L, beta, seed, tile=tile, q=q) as s:
        s.sweep(2)
        prof = s.profile(4)
        s.sweep(n - 6)
        assert set(prof) == set(sw.PROFILE_STAGES) and len(sw.PROFILE_STAGES) == 6
        assert all(math.isfinite(v) and v >= 0.0 for v in prof.values())
        assert prof["tile"] > 0.0 and prof["record"] > 0.0
        _assert_records(s.series(0, n), ref, f"profiled L={L} tile={tile} q={q}")
        assert np.array_equal(s.spins(), sp)
