"""The paper's own cluster formation (iterated label equivalence, Sec. 2.3),
selected with SW_FLAG_LABEL_EQUIV: labels, spins and records must be bit for
bit those of the oracle and of the default tile pipeline."""
import math

import numpy as np
import pytest

import oracle
import paper_2302_14720_amd as sw

pytestmark = pytest.mark.gpu

BETA_C = math.log(1.0 + math.sqrt(2.0)) / 2.0
FIELDS = ("sweep", "e_sum", "energy", "m_sum", "n_clusters", "max_cluster", "sum_sq_sizes")


def _same_records(a, b, where):
    assert len(a) == len(b), where
    for f in FIELDS:
        bad = np.nonzero(a[f] != b[f])[0]
        assert bad.size == 0, f"{where} field {f}: first mismatch at record {bad[0]}"
    assert np.array_equal(a["hist_log2"], b["hist_log2"]), f"{where} hist_log2"


def _le(L, beta, seed, **kw):
    print(f"\n[case] label-equivalence L={L} beta={beta} seed={seed} {kw}", flush=True)
    kw.setdefault("flags", sw.SW_FLAG_LABEL_EQUIV)
    return sw.Sim(L, beta, 1.0, seed, **kw)


@pytest.mark.parametrize("L", [32, 64, 96, 128])
@pytest.mark.parametrize("beta", [0.3, BETA_C, 0.6])
def test_matches_oracle(L, beta):
    seed, n = 50 + L, 12
    sp = oracle.init(L, seed)
    T = oracle.threshold(beta, 1.0)
    ref = oracle.run(L, 1.0, T, seed, 0, n - 1, sp)
    last, lab, _ = oracle.sweep(L, 1.0, T, seed, n - 1, sp)
    with _le(L, beta, seed) as s:
        s.sweep(n - 1)
        s.sweep(1)
        got = s.series(0, n)
        _same_records(got[: n - 1], ref, f"L={L}")
        _same_records(got[n - 1:], np.array([last], dtype=got.dtype), f"L={L} last")
        assert np.array_equal(s.spins(), sp)
        assert np.array_equal(s.labels(), lab)
        assert s.label_passes >= 1


@pytest.mark.parametrize("beta", [0.0, 40.0])
def test_degenerate(beta):
    L, seed, n = 64, 9, 5
    sp = oracle.init(L, seed)
    ref = oracle.run(L, 1.0, oracle.threshold(beta, 1.0), seed, 0, n, sp)
    with _le(L, beta, seed) as s:
        s.sweep(n)
        _same_records(s.series(0, n), ref, f"beta={beta}")
        assert np.array_equal(s.spins(), sp)


@pytest.mark.parametrize("L,beta,cold", [(1024, BETA_C, False), (512, 0.4, False), (256, BETA_C, True)])
def test_matches_tile_pipeline(L, beta, cold):
    seed, n = 77, 8
    init = sw.SW_INIT_COLD if cold else sw.SW_INIT_HOT
    with sw.Sim(L, beta, 1.0, seed, init=init, flags=sw.SW_FLAG_LABELS) as t:
        t.sweep(n)
        ref, sp, lab = t.series(0, n), t.spins(), t.labels()
    with _le(L, beta, seed, init=init) as s:
        s.sweep(n)
        _same_records(s.series(0, n), ref, f"L={L}")
        assert np.array_equal(s.spins(), sp)
        assert np.array_equal(s.labels(), lab)
        passes = s.label_passes
        print(f"[info] L={L} beta={beta:.4f}: {passes} label-equivalence passes in the last sweep", flush=True)
        assert 1 <= passes < 1000


def test_dense_histogram():
    L, seed, n, beta = 96, 21, 6, BETA_C
    sp = oracle.init(L, seed)
    T = oracle.threshold(beta, 1.0)
    oracle.run(L, 1.0, T, seed, 0, n - 1, sp)
    _, _, _, dense = oracle.sweep(L, 1.0, T, seed, n - 1, sp, dense=True)
    with _le(L, beta, seed, flags=sw.SW_FLAG_LABEL_EQUIV | sw.SW_FLAG_DENSE_HIST) as s:
        s.sweep(n)
        assert np.array_equal(s.cluster_hist(), dense)


def test_pass_count_at_the_papers_configuration():
    """Sec. 2.3 reports 5 to 6 scan/analysis passes at 512^2 and k_B T = 2.5
    (beta = 0.4); the pass count depends on the order of the atomic minima,
    so it is checked per sweep within a small band around that."""
    passes = []
    with _le(512, 0.4, 31) as s:
        s.sweep(20)
        for _ in range(12):
            s.sweep(1)
            passes.append(s.label_passes)
    print(f"[info] passes per sweep at 512^2, beta = 0.4: {passes}", flush=True)
    assert all(4 <= p <= 8 for p in passes), passes
    assert 4.5 <= float(np.mean(passes)) <= 7.0, passes
