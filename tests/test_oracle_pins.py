"""Pins of the CPU oracle against facts that do not come from the oracle.

Every check here is independent of the oracle's own code: published
known-answer vectors, closed forms, brute-force enumeration, breadth-first
search, exact transition probabilities and exact thermodynamics of the
finite torus (see exact.py).  All randomness is seeded, so every statistical
test is deterministic; thresholds are set at p > 1e-4 (or |z| < 4.5).
"""
import math
import os
from decimal import Decimal, getcontext

import numpy as np
import pytest

import exact
import oracle

GOLDEN = os.path.join(os.path.dirname(__file__), "golden")
BETA_C = math.log(1.0 + math.sqrt(2.0)) / 2.0


def _kat():
    rows = []
    with open(os.path.join(GOLDEN, "philox_kat.txt")) as f:
        for line in f:
            if line.strip() and not line.startswith("#"):
                v = [int(x, 16) for x in line.split()]
                rows.append((v[0:4], v[4:6], v[6:10]))
    return rows


def test_philox_known_answers():
    rows = _kat()
    assert len(rows) == 3
    for ctr, key, want in rows:
        assert list(oracle.philox4x32_10(ctr, key)) == want
        assert exact.philox4x32_10(ctr, key) == want


def test_threshold_closed_form_at_beta_c():
    # exp(-2 beta_c) = sqrt(2) - 1, so p(beta_c) = 2 - sqrt(2) exactly.
    getcontext().prec = 60
    closed = int(((Decimal(2) - Decimal(2).sqrt()) * Decimal(2 ** 32)).to_integral_value(
        rounding="ROUND_FLOOR"))
    assert closed == exact.threshold_exact(exact.beta_c_decimal())
    assert oracle.threshold(BETA_C, 1.0) == closed


@pytest.mark.parametrize("beta", [0.30, 0.35, 0.40, 0.44, 0.48, 0.55, 0.60, 1.0, 2.5])
def test_threshold_matches_high_precision(beta):
    assert oracle.threshold(beta, 1.0) == exact.threshold_exact(beta)


def test_threshold_grid_and_limits():
    for k in range(32):  # the batched-replica temperature grid
        b = 0.40 + 0.08 * k / 31
        assert oracle.threshold(b, 1.0) == exact.threshold_exact(b)
    rng = np.random.default_rng(5)
    for b in rng.uniform(0.35, 0.55, 64):
        assert oracle.threshold(float(b), 1.0) == exact.threshold_exact(float(b))
    assert oracle.threshold(0.0, 1.0) == 0          # no bonds at infinite T
    assert oracle.threshold(40.0, 1.0) == 0xFFFFFFFF  # p rounds to 1
    assert oracle.threshold(0.2, 2.0) == exact.threshold_exact(0.4)  # only beta*J


def test_init_hot_and_cold():
    L, seed = 8, 0x1234_5678_9ABC
    hot = oracle.init(L, seed, cold=False)
    assert [int(v) for v in hot] == [exact.init_spin(seed, s) for s in range(L * L)]
    assert np.all(oracle.init(L, seed, cold=True) == 1)
    big = oracle.init(256, 7)
    assert abs(int(big.astype(np.int64).sum())) < 5 * 256  # ~N(0, 256)


@pytest.mark.parametrize("L", [2, 5, 6, 9])
def test_bond_keying_and_rule(L):
    """Bond (s,d) <=> equal spins and word 2(s&1)+d of {s>>1,t,0,0} < T."""
    seed, t = (3 << 40) | 77, 11
    T = oracle.threshold(0.5, 1.0)
    rng = np.random.default_rng(L)
    spins = rng.choice(np.array([-1, 1], dtype=np.int8), size=L * L)
    b = oracle.bonds(L, T, seed, t, spins)
    for s in range(L * L):
        x, y = s % L, s // L
        for d, nb in ((0, y * L + (x + 1) % L), (1, ((y + 1) % L) * L + x)):
            want = spins[s] == spins[nb] and exact.bond_word(seed, t, s, d) < T
            assert bool((b[s] >> d) & 1) == want, (s, d)


def test_bond_threshold_is_strict():
    """An edge whose word equals T is not bonded; with T + 1 it is."""
    L, seed, t = 4, 2718, 9
    spins = np.ones(L * L, dtype=np.int8)
    for s_, d in ((5, 0), (6, 1), (11, 0)):
        w = exact.bond_word(seed, t, s_, d)
        assert not (oracle.bonds(L, w, seed, t, spins)[s_] >> d) & 1
        assert (oracle.bonds(L, w + 1, seed, t, spins)[s_] >> d) & 1


def test_cold_start_first_bonds_are_the_uniform_test():
    L, seed = 16, 99
    T = oracle.threshold(BETA_C)
    b = oracle.bonds(L, T, seed, 0, oracle.init(L, seed, cold=True))
    for s in range(L * L):
        for d in (0, 1):
            assert bool((b[s] >> d) & 1) == (exact.bond_word(seed, 0, s, d) < T)
    # fraction of bonded edges is T / 2^32 (binomial z-test)
    p = T / 2 ** 32
    n = 2 * L * L
    k = sum(bin(int(v)).count("1") for v in b)
    assert abs(k - n * p) < 4.5 * math.sqrt(n * p * (1 - p))


@pytest.mark.parametrize("L", [2, 3, 4, 5, 8, 17, 64])
def test_labels_equal_bfs(L):
    rng = np.random.default_rng(100 + L)
    for density in (0.0, 0.3, 0.5, 0.7, 1.0):
        mask = (rng.random(L * L) < density).astype(np.uint8) | \
               ((rng.random(L * L) < density).astype(np.uint8) << 1)
        assert np.array_equal(oracle.label(L, mask), exact.bfs_labels(L, mask))


def test_assignment_uses_root_flip_bit():
    L, seed, t = 12, 2024, 5
    rng = np.random.default_rng(1)
    mask = (rng.random(L * L) < 0.6).astype(np.uint8) | ((rng.random(L * L) < 0.6).astype(np.uint8) << 1)
    lab = oracle.label(L, mask)
    s = oracle.assign(L, seed, t, lab)
    for i in range(L * L):
        assert int(s[i]) == exact.flip_spin(seed, t, int(lab[i]))
        assert oracle.flip_spin(seed, t, i) == exact.flip_spin(seed, t, i)


def test_beta_zero_has_no_bonds():
    L, seed = 16, 8
    sp = oracle.init(L, seed)
    rec, lab, b = oracle.sweep(L, 1.0, oracle.threshold(0.0), seed, 4, sp)
    assert not b.any()
    assert np.array_equal(lab, np.arange(L * L, dtype=np.uint32))
    assert [int(v) for v in sp] == [exact.flip_spin(seed, 4, s) for s in range(L * L)]
    assert rec["n_clusters"] == L * L and rec["max_cluster"] == 1


def test_spin_reversal_symmetry():
    """New spins ignore old spins, and bonds see only equality: sweep(-s) == sweep(s)."""
    L, seed = 10, 31
    T = oracle.threshold(BETA_C)
    rng = np.random.default_rng(3)
    for t in range(8):
        a = rng.choice(np.array([-1, 1], dtype=np.int8), size=L * L)
        b = (-a).astype(np.int8)
        ra, la, ba = oracle.sweep(L, 1.0, T, seed, t, a)
        rb, lb, bb = oracle.sweep(L, 1.0, T, seed, t, b)
        assert np.array_equal(a, b) and np.array_equal(la, lb) and np.array_equal(ba, bb)
        assert ra.tobytes() == rb.tobytes()


def _records_from_definitions(L, spins, labels, J):
    g = spins.reshape(L, L).astype(np.int64)
    e = int((g * np.roll(g, -1, axis=1)).sum() + (g * np.roll(g, -1, axis=0)).sum())
    _, sizes = np.unique(labels, return_counts=True)
    hist = np.zeros(33, dtype=np.uint64)
    for sz in sizes:
        hist[int(sz).bit_length() - 1] += 1
    return e, int(g.sum()), len(sizes), int(sizes.max()), int((sizes.astype(np.int64) ** 2).sum()), hist


def test_records_and_invariants():
    L, seed, J = 16, 12345, 1.0
    T = oracle.threshold(BETA_C, J)
    sp = oracle.init(L, seed)
    N = L * L
    for t in range(60):
        old = sp.copy()
        rec, lab, b, dense = oracle.sweep(L, J, T, seed, t, sp, dense=True)
        e, m, nc, mx, sq, hist = _records_from_definitions(L, sp, lab, J)
        assert rec["sweep"] == t
        assert (rec["e_sum"], rec["m_sum"], rec["n_clusters"], rec["max_cluster"],
                rec["sum_sq_sizes"]) == (e, m, nc, mx, sq)
        assert rec["energy"] == -J * e
        assert np.array_equal(rec["hist_log2"], hist)
        # integer invariants
        assert (rec["e_sum"] - 2 * N) % 4 == 0
        assert (rec["m_sum"] - N) % 2 == 0
        assert int(rec["hist_log2"].sum()) == rec["n_clusters"]
        assert int((dense * np.arange(N + 1, dtype=np.uint64)).sum()) == N
        assert int(dense.sum()) == rec["n_clusters"]
        assert rec["sum_sq_sizes"] >= N and rec["max_cluster"] <= N
        # labels are canonical minimum sites
        idx = np.arange(N, dtype=np.uint32)
        assert np.all(lab <= idx) and np.array_equal(lab[lab], lab)
        # bonds join only equal old spins; bonded ends share a label and a new spin
        g_old = old.reshape(L, L)
        lab2 = lab.reshape(L, L)
        eb = (b.reshape(L, L) & 1).astype(bool)
        nb = (b.reshape(L, L) & 2).astype(bool)
        assert np.all(g_old[eb] == np.roll(g_old, -1, axis=1)[eb])
        assert np.all(g_old[nb] == np.roll(g_old, -1, axis=0)[nb])
        assert np.all(lab2[eb] == np.roll(lab2, -1, axis=1)[eb])
        assert np.all(lab2[nb] == np.roll(lab2, -1, axis=0)[nb])
        assert np.all(sp == sp[lab])


def test_4x4_exact_enumeration_chi2():
    """Final states of independent chains follow the exact Boltzmann law."""
    L = 4
    e_all, m_all = exact.enumerate_torus(L)
    # density of states of the 4x4 torus, by brute force
    vals, g = np.unique(e_all, return_counts=True)
    assert int(g.sum()) == 2 ** 16 and dict(zip(vals.tolist(), g.tolist()))[32] == 2
    for beta in (BETA_C, 0.3):
        w = np.exp(beta * e_all.astype(np.float64))
        Z = w.sum()
        n = 100_000
        e, m = oracle.chains(L, 1.0, oracle.threshold(beta), 777, n, 12)
        ev = np.unique(e_all)
        pe = np.array([w[e_all == v].sum() / Z for v in ev])
        obs = np.array([(e == v).sum() for v in ev])
        assert obs.sum() == n
        chi2, dof, p = exact.chi2_pvalue(obs, n * pe)
        assert p > 1e-4, (beta, chi2, dof)
        mv = np.unique(np.abs(m_all))
        pm = np.array([w[np.abs(m_all) == v].sum() / Z for v in mv])
        obs_m = np.array([(np.abs(m) == v).sum() for v in mv])
        chi2, dof, p = exact.chi2_pvalue(obs_m, n * pm)
        assert p > 1e-4, (beta, chi2, dof)


def test_2x2_exact_transition_matrix_detailed_balance():
    """The enumerated one-sweep kernel is stochastic, satisfies detailed
    balance w.r.t. the Boltzmann weights, and the oracle samples it."""
    L, n = 2, 4
    beta = BETA_C
    T = oracle.threshold(beta)
    P = T / 2 ** 32
    e_all, _ = exact.enumerate_torus(L)
    pi = np.exp(beta * e_all.astype(np.float64))
    pi /= pi.sum()
    M = np.zeros((16, 16))
    for a in range(16):
        for code, pr in exact.transition_row(L, exact.code_to_spins(a, n), P).items():
            M[a, code] += pr
    assert np.allclose(M.sum(axis=1), 1.0, atol=1e-12)
    # detailed balance holds for the exact bond probability 1 - exp(-2 beta)
    Pex = -math.expm1(-2 * beta)
    Mx = np.zeros((16, 16))
    for a in range(16):
        for code, pr in exact.transition_row(L, exact.code_to_spins(a, n), Pex).items():
            Mx[a, code] += pr
    flux = pi[:, None] * Mx
    assert np.allclose(flux, flux.T, atol=1e-14)
    assert np.allclose(pi @ Mx, pi, atol=1e-14)
    # ...and fails for the printed p = 1 - exp(-beta) at the same beta
    Pw = -math.expm1(-beta)
    Mw = np.zeros((16, 16))
    for a in range(16):
        for code, pr in exact.transition_row(L, exact.code_to_spins(a, n), Pw).items():
            Mw[a, code] += pr
    assert not np.allclose(pi @ Mw, pi, atol=1e-6)
    for a in (0, 5, 9):
        start = np.array(exact.code_to_spins(a, n), dtype=np.int8)
        codes = oracle.one_step_codes(L, T, 1000 + a, 60_000, 3, start)
        obs = np.bincount(codes.astype(np.int64), minlength=16)
        chi2, dof, p = exact.chi2_pvalue(obs, 60_000 * M[a])
        assert p > 1e-4, (a, chi2, dof)


def test_3x3_exact_transition_rows():
    L, n = 3, 9
    rng = np.random.default_rng(9)
    for beta in (0.3, BETA_C):
        T = oracle.threshold(beta)
        P = T / 2 ** 32
        for trial in range(2):
            start = rng.choice(np.array([-1, 1], dtype=np.int8), size=n)
            row = exact.transition_row(L, [int(v) for v in start], P)
            assert abs(sum(row.values()) - 1.0) < 1e-12
            nseeds = 60_000
            codes = oracle.one_step_codes(L, T, 5000 + trial, nseeds, 7, start)
            keys = sorted(row)
            index = {k: i for i, k in enumerate(keys)}
            obs = np.zeros(len(keys))
            for c in codes.tolist():
                assert c in index  # never reaches an impossible configuration
                obs[index[c]] += 1
            chi2, dof, p = exact.chi2_pvalue(obs, nseeds * np.array([row[k] for k in keys]))
            assert p > 1e-4, (beta, trial, chi2, dof)


def test_kaufman_formula_pins():
    e_all, _ = exact.enumerate_torus(4)
    for beta in (0.3, BETA_C, 0.6):
        w = np.exp(beta * e_all.astype(np.float64))
        u_enum = -(e_all * w).sum() / w.sum() / 16
        assert abs(exact.kaufman_energy(beta, 4) - u_enum) < 1e-12
    for beta in (0.3, 0.6):  # finite-size corrections vanish exponentially
        assert abs(exact.kaufman_energy(beta, 128) - exact.onsager_energy(beta)) < 1e-12
    assert abs(exact.onsager_energy(BETA_C + 1e-9) + math.sqrt(2)) < 1e-6


def _binned_mean(x, nbins=20):
    x = np.asarray(x, dtype=np.float64)
    b = x[: len(x) // nbins * nbins].reshape(nbins, -1).mean(axis=1)
    return b.mean(), b.std(ddof=1) / math.sqrt(nbins)


def test_energy_at_beta_c_L64_matches_ferdinand_fisher():
    L, seed = 64, 1
    T = oracle.threshold(BETA_C)
    sp = oracle.init(L, seed)
    recs = oracle.run(L, 1.0, T, seed, 0, 4200, sp)
    u = -recs["e_sum"][200:].astype(np.float64) / (L * L)
    mean, err = _binned_mean(u)
    want = exact.kaufman_energy(BETA_C, L)
    assert abs(mean - want) < 4.5 * err, (mean, err, want)
    assert err < 0.005


@pytest.mark.parametrize("beta", [0.3, 0.6])
def test_off_critical_energy_and_magnetisation(beta):
    L, seed = 128, 10
    T = oracle.threshold(beta)
    sp = oracle.init(L, seed)
    recs = oracle.run(L, 1.0, T, seed, 0, 700, sp)
    u = -recs["e_sum"][100:].astype(np.float64) / (L * L)
    mean, err = _binned_mean(u)
    assert abs(mean - exact.onsager_energy(beta)) < 4.5 * err + 1e-9, (mean, err)
    if beta > BETA_C:
        am = np.abs(recs["m_sum"][100:].astype(np.float64)) / (L * L)
        mmean, merr = _binned_mean(am)
        assert abs(mmean - exact.yang_magnetisation(beta)) < 4.5 * merr + 1e-9
