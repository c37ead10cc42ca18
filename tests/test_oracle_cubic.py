"""Pins of the simple cubic (L x L x L, periodic) oracle, Ising and Potts:
the bond rule and its Philox keying, brute-force connected components, the
beta = 0 limit, exact enumeration of the 2x2x2 torus (Ising and q = 3 Potts),
the low- and high-temperature series of the 3D Ising model, spin reversal and
integer invariants; CPU only."""
import math

import numpy as np
import pytest
from scipy.sparse import coo_matrix
from scipy.sparse.csgraph import connected_components

import exact
import oracle


def cube_neighbours(L: int):
    """Index of the +x, +y, +z neighbour of every site s = (z*L + y)*L + x,
    from coordinates."""
    z, y, x = np.meshgrid(np.arange(L), np.arange(L), np.arange(L), indexing="ij")
    idx = lambda zz, yy, xx: ((zz % L) * L + (yy % L)) * L + (xx % L)
    return [idx(z, y, x + 1).ravel(), idx(z, y + 1, x).ravel(), idx(z + 1, y, x).ravel()]


def bond_words(L: int, seed: int, t: int) -> np.ndarray:
    """[N, 3] the word of every (site, direction) from the pinned Philox:
    word d of the output for counter {s, t, 4, 0}."""
    key = [seed & 0xFFFFFFFF, seed >> 32]
    return np.array([oracle.philox4x32_10([s, t, 4, 0], key)[:3] for s in range(L ** 3)])


@pytest.mark.parametrize("q", [0, 3])
def test_bond_keying_and_rule(q):
    """Hot start: bond (s, d) iff the two end spins are equal and word d of
    Philox({s, t, 4, 0}) is below T."""
    L, seed, t = 5, 77, 3
    T = oracle.threshold(0.35) if q == 0 else oracle.potts_threshold(0.8)
    sp = oracle.cubic_init(L, seed, q)
    b = oracle.cubic_bonds(L, T, seed, t, sp)
    w = bond_words(L, seed, t)
    nb = cube_neighbours(L)
    want = np.zeros(L ** 3, dtype=np.uint8)
    for d in range(3):
        want |= ((sp == sp[nb[d]]) & (w[:, d] < T)).astype(np.uint8) << d
    assert np.array_equal(b, want)
    assert b.any() and (b != 7).any()


def test_hot_and_cold_start():
    L = 8
    for q in (0, 4):
        cold = oracle.cubic_init(L, 1, q, cold=True)
        assert np.all(cold == (0 if q else 1))
    key = [5, 0]
    hot = oracle.cubic_init(L, 5, 0)
    want = np.array([-1 if oracle.philox4x32_10([s, 0, 2, 0], key)[0] & 1 else 1 for s in range(L ** 3)])
    assert np.array_equal(hot, want)
    hot3 = oracle.cubic_init(L, 5, 3)
    want3 = np.array([(int(oracle.philox4x32_10([s, 0, 2, 0], key)[0]) * 3) >> 32 for s in range(L ** 3)])
    assert np.array_equal(hot3, want3)


@pytest.mark.parametrize("L,density", [(4, 0.3), (5, 0.25), (6, 0.4)])
def test_labels_are_min_site_components(L, density):
    """Components of random bond masks by a library graph routine; every
    site must carry the smallest site of its component."""
    rng = np.random.default_rng(L)
    n = L ** 3
    mask = np.zeros(n, dtype=np.uint8)
    for d in range(3):
        mask |= (rng.random(n) < density).astype(np.uint8) << d
    lab = oracle.cubic_label(L, mask)
    nb = cube_neighbours(L)
    rows, cols = [], []
    for d in range(3):
        s = np.nonzero(mask & (1 << d))[0]
        rows.append(s)
        cols.append(nb[d][s])
    r, c = np.concatenate(rows), np.concatenate(cols)
    g = coo_matrix((np.ones(len(r)), (r, c)), shape=(n, n))
    ncomp, comp = connected_components(g, directed=False)
    smallest = np.full(ncomp, n)
    np.minimum.at(smallest, comp, np.arange(n))
    assert np.array_equal(lab, smallest[comp])


@pytest.mark.parametrize("q", [0, 5])
def test_beta_zero_every_site_its_own_cluster(q):
    L, seed, t = 6, 12, 4
    sp = oracle.cubic_init(L, seed, q)
    rec, lab, b, dense = oracle.cubic_sweep(L, 1.0, 0, q, seed, t, sp, dense=True)
    n = L ** 3
    assert not b.any()
    assert np.array_equal(lab, np.arange(n))
    want = [oracle.potts_spin(seed, t, s, q) if q else oracle.flip_spin(seed, t, s) for s in range(n)]
    assert np.array_equal(sp, want)
    assert rec["n_clusters"] == n and rec["max_cluster"] == 1 and dense[1] == n


@pytest.mark.parametrize("q", [3, 5])
def test_potts_m_sum_is_the_largest_population(q):
    """Potts records (R14, R15): m_sum is the population of the most
    populated value, recounted here from the returned spins; a high
    temperature keeps every value the largest now and then."""
    L = 6
    T = oracle.potts_threshold(0.2)
    sp = oracle.cubic_init(L, 41, q)
    winners = set()
    for t in range(40):
        rec, lab, b, dense = oracle.cubic_sweep(L, 1.0, T, q, 41, t, sp, dense=True)
        counts = np.bincount(sp, minlength=q)
        assert int(rec["m_sum"]) == counts.max(), (t, counts, int(rec["m_sum"]))
        winners.add(int(counts.argmax()))
    assert len(winners) == q, winners


def cube2_states(q: int):
    """All q^8 configurations of the 2x2x2 torus and their e_sum over the 24
    edges (s, s + d), counted per direction: Ising sum of s_i s_j, Potts
    number of equal pairs."""
    L, N = 2, 8
    idx = np.arange(max(q, 2) ** N)
    if q == 0:
        spins = 1 - 2 * ((idx[:, None] >> np.arange(N)[None, :]) & 1)
    else:
        spins = (idx[:, None] // q ** np.arange(N)[None, :]) % q
    e = np.zeros(len(idx), dtype=np.int64)
    for nb in cube_neighbours(L):
        for s in range(N):
            e += spins[:, s] * spins[:, nb[s]] if q == 0 else spins[:, s] == spins[:, nb[s]]
    return spins, e


def test_2x2x2_ising_exact_enumeration_chi2():
    """The final states of independent chains follow exp(beta e_sum) over
    the 256 states of the 2x2x2 torus, in energy and in |M|."""
    spins, e_all = cube2_states(0)
    m_all = np.abs(spins.sum(axis=1))
    n = 100_000
    for beta in (0.12, 0.2216544):
        w = np.exp(beta * e_all.astype(np.float64))
        e, m = oracle.cubic_chains(2, 1.0, oracle.threshold(beta), 0, 31, n, 16)
        for vals, obs_vals in ((e_all, e), (m_all, np.abs(m))):
            keys = np.unique(vals)
            pk = np.array([w[vals == k].sum() for k in keys]) / w.sum()
            obs = np.array([(obs_vals == k).sum() for k in keys])
            assert obs.sum() == n
            chi2, dof, p = exact.chi2_pvalue(obs, n * pk)
            assert p > 1e-4, (beta, chi2, dof)


def test_2x2x2_potts_q3_exact_enumeration_chi2():
    """q = 3 Potts: chains follow exp(beta * #equal edges) over the 3^8
    states; each site holds value 0 with probability 1/3."""
    spins, e_all = cube2_states(3)
    n = 60_000
    for beta in (0.3, 0.55):
        w = np.exp(beta * e_all.astype(np.float64))
        e, n0 = oracle.cubic_chains(2, 1.0, oracle.potts_threshold(beta), 3, 57, n, 20)
        keys = np.unique(e_all)
        pk = np.array([w[e_all == k].sum() for k in keys]) / w.sum()
        obs = np.array([(e == k).sum() for k in keys])
        assert obs.sum() == n
        chi2, dof, p = exact.chi2_pvalue(obs, n * pk)
        assert p > 1e-4, (beta, chi2, dof)
        assert abs(n0.mean() - 8 / 3) < 5 * n0.std() / math.sqrt(n)


def batch_mean(x: np.ndarray, nb: int = 20):
    b = x[: len(x) // nb * nb].reshape(nb, -1).mean(axis=1)
    return b.mean(), b.std(ddof=1) / math.sqrt(nb)


def test_low_temperature_series():
    """beta = 0.75, L = 8: <e_sum>/N = 3 - 12 x^6 - 60 x^10 + 84 x^12 +
    O(x^14), x = exp(-2 beta) (one flipped site breaks 6 bonds, an adjacent
    pair 10, two separate sites 12)."""
    L, beta, n = 8, 0.75, 60_000
    x = math.exp(-2 * beta)
    want = 3 - 12 * x ** 6 - 60 * x ** 10 + 84 * x ** 12
    sp = oracle.cubic_init(L, 3, 0, cold=True)
    recs = oracle.cubic_run(L, 1.0, oracle.threshold(beta), 0, 3, 0, n + 200, sp)
    mean, err = batch_mean(recs["e_sum"][200:] / L ** 3)
    assert abs(mean - want) < 5 * err + 1e-6, (mean, want, err)
    assert 3 - mean > 10 * err  # the single-flip term is resolved


def test_high_temperature_series():
    """beta = 0.05, L = 8: <e_sum>/N = 3v + 12 v^3 (1 - v^2) + O(v^5),
    v = tanh beta (three edges per site, three plaquettes per site)."""
    L, beta, n = 8, 0.05, 100_000
    v = math.tanh(beta)
    want = 3 * v + 12 * v ** 3 * (1 - v * v)
    sp = oracle.cubic_init(L, 4, 0)
    recs = oracle.cubic_run(L, 1.0, oracle.threshold(beta), 0, 4, 0, n + 50, sp)
    mean, err = batch_mean(recs["e_sum"][50:] / L ** 3)
    assert abs(mean - want) < 4 * err, (mean, want, err)
    assert abs(mean - 3 * v) > 3 * err  # the plaquette term is resolved


def test_spin_reversal_symmetry():
    """Ising: new spins are assigned, not flipped, so -sigma and sigma give
    the same next configuration and record."""
    L, seed = 6, 21
    T = oracle.threshold(0.3)
    a = oracle.cubic_init(L, seed, 0)
    b = (-a).astype(np.int8)
    for t in range(4):
        ra, la, _ = oracle.cubic_sweep(L, 1.0, T, 0, seed, t, a)
        rb, lb, _ = oracle.cubic_sweep(L, 1.0, T, 0, seed, t, b)
        assert np.array_equal(a, b) and np.array_equal(la, lb) and ra.tobytes() == rb.tobytes()
        b = (-b).astype(np.int8)


@pytest.mark.parametrize("L,beta", [(8, 0.2216544), (10, 0.4), (12, 0.1)])
def test_integer_invariants(L, beta):
    """Every line of L sites around the torus holds an even number of domain
    walls, so e_sum = 3N (mod 4); m_sum = N (mod 2); the histograms count
    every cluster and every site once."""
    n = L ** 3
    sp = oracle.cubic_init(L, 8, 0)
    T = oracle.threshold(beta)
    for t in range(5):
        rec, lab, b, dense = oracle.cubic_sweep(L, 1.0, T, 0, 8, t, sp, dense=True)
        assert rec["e_sum"] % 4 == (3 * n) % 4 and rec["m_sum"] % 2 == n % 2
        assert rec["e_sum"] == sum(int((sp * sp[nb]).sum()) for nb in cube_neighbours(L))
        assert rec["hist_log2"].sum() == rec["n_clusters"] == len(np.unique(lab))
        assert int((dense * np.arange(n + 1)).sum()) == n
        assert rec["max_cluster"] == np.bincount(lab).max()
        assert rec["sum_sq_sizes"] == int((np.bincount(lab).astype(np.int64) ** 2).sum())
