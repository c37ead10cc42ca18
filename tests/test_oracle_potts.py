"""Pins of the q-state Potts oracle (spins 0..q-1, H = -J sum delta(s_i, s_j),
bonds with p = 1 - exp(-beta J), uniform new value per cluster), checked
against exact enumeration, the Ising model it reduces to at q = 2, the
infinite-temperature limit and the exact critical energy; CPU only."""
import math
from decimal import Decimal, getcontext

import numpy as np
import pytest

import exact
import oracle


def potts_beta_c(q: int) -> float:
    return math.log(1.0 + math.sqrt(q))


def test_threshold_closed_form():
    """At beta_c = ln(1 + sqrt q): p = sqrt(q) / (1 + sqrt(q)), in 60 digits."""
    getcontext().prec = 60
    for q in (2, 3, 4, 8):
        sq = Decimal(q).sqrt()
        want = int((sq / (1 + sq) * Decimal(2) ** 32).to_integral_value(rounding="ROUND_FLOOR"))
        assert oracle.potts_threshold(potts_beta_c(q), 1.0) == want
    assert oracle.potts_threshold(0.0) == 0
    # Potts coupling beta J equals an Ising coupling beta J / 2
    for b in (0.2, 0.7, 1.3):
        assert oracle.potts_threshold(b, 1.0) == oracle.threshold(b / 2.0, 1.0)


def test_init_and_value_ranges():
    q, L = 5, 32
    hot = oracle.potts_init(L, 9, q)
    assert hot.min() >= 0 and hot.max() < q and len(np.unique(hot)) == q
    assert np.all(oracle.potts_init(L, 9, q, cold=True) == 0)
    vals = [oracle.potts_spin(3, t, r, q) for t in range(20) for r in range(200)]
    assert min(vals) >= 0 and max(vals) < q


def test_hot_start_site_by_site_and_iid_uniform():
    """Hot start (R14): site s takes floor(w q / 2^32) of word 0 of the
    Philox output for counter {s, 0, 2, 0}, recomputed here with the
    independent Python Philox that the known-answer vectors pin; on a larger
    lattice single values and horizontal neighbour pairs are uniform (chi^2),
    as i.i.d. uniform values must be."""
    for q, L, seed in ((5, 12, 9), (3, 8, 2 ** 40 + 7), (8, 8, 123)):
        key = exact.seed_key(seed)
        want = np.array([(exact.philox4x32_10([s, 0, 2, 0], key)[0] * q) >> 32 for s in range(L * L)])
        assert np.array_equal(oracle.potts_init(L, seed, q), want), (q, L, seed)
    q, L = 5, 192
    hot = oracle.potts_init(L, 31, q).astype(np.int64)
    n = L * L
    chi2, dof, p = exact.chi2_pvalue(np.bincount(hot, minlength=q), np.full(q, n / q))
    assert p > 1e-4, (chi2, dof)
    grid = hot.reshape(L, L)
    pair = (grid * q + np.roll(grid, -1, axis=1)).ravel()
    chi2, dof, p = exact.chi2_pvalue(np.bincount(pair, minlength=q * q), np.full(q * q, n / q ** 2))
    assert p > 1e-4, (chi2, dof)


def test_q2_is_ising_at_half_the_coupling():
    """q = 2 Potts at beta is the Ising model at beta / 2: with e_I = 2 e_P - 2N
    the final states of independent chains follow the exact 4x4 Ising law."""
    L, N, n = 4, 16, 60_000
    e_all, _ = exact.enumerate_torus(L)
    for beta_p in (2 * math.log(1 + math.sqrt(2)) / 2, 0.6):
        w = np.exp(beta_p / 2 * e_all.astype(np.float64))
        ev = np.unique(e_all)
        pe = np.array([w[e_all == v].sum() for v in ev]) / w.sum()
        e_p, _ = oracle.potts_chains(L, 1.0, oracle.potts_threshold(beta_p), 2, 4242, n, 30)
        e_i = 2 * e_p - 2 * N
        obs = np.array([(e_i == v).sum() for v in ev])
        assert obs.sum() == n
        chi2, dof, p = exact.chi2_pvalue(obs, n * pe)
        assert p > 1e-4, (beta_p, chi2, dof)


def test_q3_3x3_exact_energy_law():
    """All 3^9 configurations of the 3x3 torus, Boltzmann weights
    exp(beta * #equal edges): the oracle's chains sample that law."""
    L, q, n = 3, 3, 40_000
    N = L * L
    idx = np.arange(q ** N)
    spins = (idx[:, None] // q ** np.arange(N)[None, :]) % q
    eq = np.zeros(q ** N, dtype=np.int64)
    for a, b in exact.torus_edges(L):
        eq += spins[:, a] == spins[:, b]
    for beta in (potts_beta_c(q), 0.5):
        w = np.exp(beta * eq.astype(np.float64))
        ev = np.unique(eq)
        pe = np.array([w[eq == v].sum() for v in ev]) / w.sum()
        e, n0 = oracle.potts_chains(L, 1.0, oracle.potts_threshold(beta), q, 99, n, 30)
        obs = np.array([(e == v).sum() for v in ev])
        assert obs.sum() == n
        chi2, dof, p = exact.chi2_pvalue(obs, n * pe)
        assert p > 1e-4, (beta, chi2, dof)
        # q-fold symmetry: each site holds value 0 with probability 1/q
        assert abs(n0.mean() - N / q) < 5 * n0.std() / math.sqrt(n), n0.mean()


def test_infinite_temperature_gives_iid_uniform_values():
    """beta = 0: no bonds, every site is its own cluster and draws a fresh
    uniform value each sweep."""
    L, q = 64, 4
    sp = oracle.potts_init(L, 1, q, cold=True)
    counts = np.zeros(q)
    pairs = 0
    for t in range(40):
        rec, lab = oracle.potts_sweep(L, 1.0, 0, q, 1, t, sp)
        assert int(rec["n_clusters"]) == L * L and np.all(lab == np.arange(L * L))
        counts += np.bincount(sp, minlength=q)
        pairs += int(rec["e_sum"])
    total = 40 * L * L
    chi2, dof, p = exact.chi2_pvalue(counts, np.full(q, total / q))
    assert p > 1e-4, (chi2, dof)
    # equal neighbour pairs: 2N edges per sweep, each equal with probability 1/q
    mean, sd = 40 * 2 * L * L / q, math.sqrt(40 * 2 * L * L * (1 / q) * (1 - 1 / q))
    assert abs(pairs - mean) < 5 * sd


def test_clusters_respect_values_and_records():
    """Bonds only join equal values; every cluster gets one new value;
    records are consistent."""
    L, q = 48, 3
    beta = potts_beta_c(q)
    T = oracle.potts_threshold(beta)
    sp = oracle.potts_init(L, 17, q)
    for t in range(6):
        old = sp.copy()
        rec, lab = oracle.potts_sweep(L, 1.0, T, q, 17, t, sp)
        assert np.all(old == old[lab])  # a cluster never spans two values
        assert np.all(sp == sp[lab])  # one new value per cluster
        assert np.all(lab <= np.arange(L * L)) and np.all(lab[lab] == lab)
        N = L * L
        assert 0 <= int(rec["e_sum"]) <= 2 * N and rec["energy"] == -float(rec["e_sum"])
        assert int(rec["m_sum"]) == np.bincount(sp, minlength=q).max()
        assert int(rec["hist_log2"].sum()) == int(rec["n_clusters"])


@pytest.mark.slow
def test_q3_critical_energy():
    """At beta_c the energy per site of the infinite lattice is
    -(1 + 1/sqrt q) J; a 128^2 torus is within its finite-size shift."""
    L, q = 128, 3
    beta = potts_beta_c(q)
    T = oracle.potts_threshold(beta)
    sp = oracle.potts_init(L, 5, q)
    oracle.potts_run(L, 1.0, T, q, 5, 0, 100, sp)
    recs = oracle.potts_run(L, 1.0, T, q, 5, 100, 400, sp)
    u = recs["e_sum"].mean() / (L * L)
    assert abs(u - (1 + 1 / math.sqrt(q))) < 0.03, u
