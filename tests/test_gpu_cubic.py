"""Simple cubic (L x L x L) sweeps through the C ABI, Ising and Potts, on
the 16^3-brick path (the default) and on the label-equivalence path, bit for
bit against the cubic oracle: records, spins and canonical labels; at full
size, properties that hold at any L."""
import math

import numpy as np
import pytest

import oracle
import paper_2302_14720_amd as sw

pytestmark = pytest.mark.gpu

FIELDS = ("sweep", "e_sum", "energy", "m_sum", "n_clusters", "max_cluster", "sum_sq_sizes")
BETA_C3 = 0.2216544  # 3D Ising critical coupling (numerical estimate), a workload parameter


def _same_records(a, b, where):
    assert len(a) == len(b), where
    for f in FIELDS:
        bad = np.nonzero(a[f] != b[f])[0]
        assert bad.size == 0, f"{where} field {f}: first mismatch at record {bad[0]}: {a[f][bad[0]]} vs {b[f][bad[0]]}"
    assert np.array_equal(a["hist_log2"], b["hist_log2"]), f"{where} hist_log2"


PATHS = ["brick", "label_equivalence"]


def _cube(L, beta, seed, q=0, flags=0, path="brick", **kw):
    print(f"\n[case] cubic {path} L={L} q={q} beta={beta} seed={seed} {kw}", flush=True)
    if path == "label_equivalence":
        flags |= sw.SW_FLAG_LABEL_EQUIV
    s = sw.Sim(L, beta, 1.0, seed, q=q, dims=3, flags=flags, **kw)
    assert s.tile == (16 if path == "brick" else 0)
    return s


def _threshold(q, beta):
    return oracle.potts_threshold(beta, 1.0) if q else oracle.threshold(beta, 1.0)


@pytest.mark.parametrize("path", PATHS)
@pytest.mark.parametrize("L", [16, 32, 48])
def test_ising_matches_oracle(L, path):
    seed, n = 700 + L, 8
    for beta in (0.0, 0.1, BETA_C3, 0.5):
        T = _threshold(0, beta)
        sp = oracle.cubic_init(L, seed, 0)
        ref = oracle.cubic_run(L, 1.0, T, 0, seed, 0, n - 1, sp)
        last, lab, _, dense = oracle.cubic_sweep(L, 1.0, T, 0, seed, n - 1, sp, dense=True)
        with _cube(L, beta, seed, flags=sw.SW_FLAG_DENSE_HIST, path=path) as s:
            assert s.threshold == T and sw.lib().sw_sites(s.handle) == L ** 3
            s.sweep(3)
            s.sweep(n - 3)
            got = s.series(0, n)
            _same_records(got[: n - 1], ref, f"L={L} beta={beta}")
            _same_records(got[n - 1:], np.array([last], dtype=got.dtype), f"L={L} beta={beta} last")
            assert np.array_equal(s.spins(), sp)
            assert np.array_equal(s.labels(), lab)
            assert np.array_equal(s.cluster_hist(), dense)


@pytest.mark.parametrize("path", PATHS)
@pytest.mark.parametrize("q", [2, 3, 5])
@pytest.mark.parametrize("L", [16, 32, 48])
def test_potts_matches_oracle(q, L, path):
    seed, n = 900 + q + L, 8
    for beta in (0.3, 0.5505, 1.5):
        T = _threshold(q, beta)
        sp = oracle.cubic_init(L, seed, q)
        ref = oracle.cubic_run(L, 1.0, T, q, seed, 0, n - 1, sp)
        last, lab, _ = oracle.cubic_sweep(L, 1.0, T, q, seed, n - 1, sp)
        with _cube(L, beta, seed, q=q, path=path) as s:
            assert s.threshold == T
            s.sweep(n)
            got = s.series(0, n)
            _same_records(got[: n - 1], ref, f"q={q} L={L} beta={beta}")
            _same_records(got[n - 1:], np.array([last], dtype=got.dtype), f"q={q} L={L} last")
            assert np.array_equal(s.spins(), sp)
            assert np.array_equal(s.labels(), lab)


@pytest.mark.parametrize("path", PATHS)
@pytest.mark.parametrize("q", [0, 3])
def test_cold_start_and_resume(q, path):
    L, seed = 32, 41
    beta = BETA_C3 if q == 0 else 0.5505
    T = _threshold(q, beta)
    sp = oracle.cubic_init(L, seed, q, cold=True)
    ref = oracle.cubic_run(L, 1.0, T, q, seed, 0, 5, sp)
    with _cube(L, beta, seed, q=q, init=sw.SW_INIT_COLD, path=path) as s:
        assert np.all(s.spins() == (0 if q else 1))
        s.sweep(5)
        _same_records(s.series(0, 5), ref, "cold")
        assert np.array_equal(s.spins(), sp)
        rng = np.random.default_rng(q + 5)
        state = (rng.integers(0, q, L ** 3) if q else 1 - 2 * rng.integers(0, 2, L ** 3)).astype(np.int8)
        s.set_spins(state, 77)
        s.sweep(4)
        ref2 = oracle.cubic_run(L, 1.0, T, q, seed, 77, 4, state)
        _same_records(s.series(77, 4), ref2, "resumed")
        assert np.array_equal(s.spins(), state)
        s.reset(sw.SW_INIT_HOT)
        assert np.array_equal(s.spins(), oracle.cubic_init(L, seed, q))


@pytest.mark.parametrize("path", PATHS)
def test_mid_size_bit_exact(path):
    """L = 256 (16.8 M sites, 4096 bricks), two sweeps at the critical coupling."""
    L, seed = 256, 5
    T = _threshold(0, BETA_C3)
    sp = oracle.cubic_init(L, seed, 0)
    ref = oracle.cubic_run(L, 1.0, T, 0, seed, 0, 2, sp)
    with _cube(L, BETA_C3, seed, path=path) as s:
        s.sweep(2)
        _same_records(s.series(0, 2), ref, "L=256")
        assert np.array_equal(s.spins(), sp)


@pytest.mark.parametrize("path", PATHS)
def test_full_size_properties(path):
    """L = 512 (134 M sites): integer invariants at the critical coupling, and
    the high-temperature series <e_sum>/N = 3v + 12 v^3 (1 - v^2), v = tanh
    beta, at beta = 0.05 (one sweep already averages over 1.6e8 edges)."""
    L = 512
    N = L ** 3
    with _cube(L, BETA_C3, 17, path=path) as s:
        s.sweep(12)
        recs = s.series(0, 12)
        assert s.label_passes > 0 or path == "brick"
        assert np.all(recs["e_sum"] % 4 == (3 * N) % 4) and np.all(recs["m_sum"] % 2 == N % 2)
        assert np.all(recs["hist_log2"].sum(axis=1) == recs["n_clusters"])
        assert np.all(recs["max_cluster"] <= N) and np.all(recs["sum_sq_sizes"] >= N)
        assert np.all(recs["sum_sq_sizes"] >= recs["max_cluster"].astype(np.float64) ** 2)
        sp = s.spins()
        assert int(sp.astype(np.int64).sum()) == int(recs["m_sum"][-1])
    beta = 0.05
    v = math.tanh(beta)
    with _cube(L, beta, 18, path=path) as s:
        s.sweep(6)
        e = s.series(1, 5)["e_sum"] / N
        want = 3 * v + 12 * v ** 3 * (1 - v * v)
        err = math.sqrt(3.0 / N / len(e))
        assert abs(e.mean() - want) < 6 * err, (e.mean(), want, err)


@pytest.mark.parametrize("q,beta", [(0, BETA_C3), (3, 0.5505)])
def test_benchmark_lattice_one_step(q, beta):
    """The benchmark's cubic legs (512^3 on bricks, hot start seed 13, Ising
    at 0.2216544 and q = 3 Potts at 0.5505): the GPU chain runs to sweep 3,
    and sweep 3 is compared with one oracle sweep from the GPU's own state
    (record and spins)."""
    L, seed, t = 512, 13, 3
    T = _threshold(q, beta)
    with _cube(L, beta, seed, q=q) as s:
        s.sweep(t)
        state = s.spins()
        s.sweep(1)
        rec = s.series(t, 1)
        final = s.spins()
    ref, _, _ = oracle.cubic_sweep(L, 1.0, T, q, seed, t, state)
    assert rec[0].tobytes() == ref.tobytes()
    assert np.array_equal(final, state)


def test_cubic_configuration_errors():
    cases = [
        dict(dims=3, flags=0, L=40),                         # not a multiple of 16
        dict(dims=3, flags=sw.SW_FLAG_LABEL_EQUIV, L=40),
        dict(dims=3, flags=sw.SW_FLAG_LABEL_EQUIV, L=1632),  # L^3 would reach 2^32
        dict(dims=3, flags=sw.SW_FLAG_LABEL_EQUIV, L=8),
        dict(dims=4, flags=sw.SW_FLAG_LABEL_EQUIV),
        dict(dims=1, flags=sw.SW_FLAG_LABEL_EQUIV),
    ]
    for c in cases:
        L = c.pop("L", 32)
        with pytest.raises(sw.SwError) as e:
            sw.Sim(L, 0.2, 1.0, 1, **c)
        assert e.value.code == sw.SW_EINVAL, c
    with _cube(16, 0.2, 1) as s:
        with pytest.raises(sw.SwError) as e:
            sw.sw_get_spins(s.handle, 16 * 16)
        assert e.value.code == sw.SW_ERANGE


@pytest.mark.parametrize("path", PATHS)
def test_largest_cubic_lattice(path):
    """The largest cubic lattice the library accepts (L = 1616, N = 4.22e9
    sites, just below 2^32): two sweeps; the record invariants; E and M
    recomputed from the spins on the host."""
    L = 1616
    N = L ** 3
    with _cube(L, BETA_C3, 29, path=path) as s:
        s.sweep(2)
        recs = s.series(0, 2)
        sp = s.spins()
    assert np.all(recs["e_sum"] % 4 == (3 * N) % 4) and np.all(recs["m_sum"] % 2 == N % 2)
    assert np.all(recs["hist_log2"].sum(axis=1) == recs["n_clusters"])
    assert np.all(recs["max_cluster"] <= N) and np.all(recs["sum_sq_sizes"] >= N)
    assert int(sp.sum(dtype=np.int64)) == int(recs["m_sum"][-1])
    g = sp.reshape(L, L, L)
    e = 0
    for ax in range(3):
        e += int(np.sum(g * np.roll(g, -1, axis=ax), dtype=np.int64))
    assert e == int(recs["e_sum"][-1])
