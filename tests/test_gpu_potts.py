"""q-state Potts sweeps (label-equivalence path) through the C ABI, bit for
bit against the Potts oracle: records, spins and canonical labels."""
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
        sw.Sim(64, 1.0, 1.0, 1, q=3)  # needs the label-equivalence path
    assert e.value.code == sw.SW_EINVAL
    with pytest.raises(sw.SwError) as e:
        sw.Sim(64, 1.0, 1.0, 1, q=9, flags=sw.SW_FLAG_LABEL_EQUIV)
    assert e.value.code == sw.SW_EINVAL
    with pytest.raises(sw.SwError) as e:
        sw.Sim(64, 1.0, 1.0, 1, q=1, flags=sw.SW_FLAG_LABEL_EQUIV)
    assert e.value.code == sw.SW_EINVAL
