"""Pins of the O(4) phi^4 oracle (unit fields, multicluster Wolff-embedding
update: bond probability of eq. 2, reflection of eq. 3; paper Sec. 3),
checked against the exact periodic O(4) ring, the exact two-vector link law,
library exp, uniformity on S^3, library connected components and the
geometric invariants of a reflection; CPU only."""
import math

import numpy as np
import pytest
from scipy import stats
from scipy.sparse import coo_matrix
from scipy.sparse.csgraph import connected_components

import exact
import oracle


def unit_sphere_marginal_cdf(x):
    """CDF of one coordinate of a uniform point on S^3: density
    (2/pi) sqrt(1 - x^2) on [-1, 1]."""
    x = np.clip(x, -1.0, 1.0)
    return 0.5 + (x * np.sqrt(1.0 - x * x) + np.arcsin(x)) / math.pi


def lattice_neighbours(D, L):
    """Index of s + mu-hat for every site s, mu = 0..D-1 (x_0 fastest)."""
    n = L ** D
    coords = np.array(np.unravel_index(np.arange(n), (L,) * D, order="F"))
    out = []
    for mu in range(D):
        c = coords.copy()
        c[mu] = (c[mu] + 1) % L
        out.append(np.ravel_multi_index(tuple(c), (L,) * D, order="F"))
    return out


def test_expm_matches_library_exp():
    """E(a), the evaluation of exp(-a) in the bond test, agrees with the C
    library's exp over the range kappa <= 4 can reach (a <= 16 for unit
    fields): within 1e-15 relative up to a = 1/8 (no squaring), and the
    error at most doubles with each of the k <= 7 squarings above."""
    a = np.concatenate([np.geomspace(1e-12, 16.5, 6000), [0.125, 0.25, 0.5, 1.0, 4.0 * 0.304]])
    got = np.array([oracle.phi4_expm(float(x)) for x in a])
    rel = np.abs(got / np.exp(-a) - 1.0)
    small = a <= 0.125
    assert rel[small].max() < 1e-15, rel[small].max()
    k = np.maximum(0, np.ceil(np.log2(a / 0.125))).astype(int)
    assert np.all(rel <= 2.0 ** k * 2e-16 + 1e-16), (a[rel.argmax()], rel.max())


def test_direction_keying_and_uniformity():
    """Sweep t's direction is the first point of the 4-ball drawn from
    Philox({k, t, 5, 0}) (recomputed with the independent Python Philox);
    over many sweeps n = r / |r| is uniform on S^3: each coordinate follows
    the (2/pi) sqrt(1 - x^2) law and the second moments are delta / 4."""
    seed = 77
    key = exact.seed_key(seed)
    for t in range(40):
        r, rr = oracle.phi4_direction(seed, t)
        for k in range(64):
            w = exact.philox4x32_10([k, t, 5, 0], key)
            v = np.array([(x + 0.5) * 2.0 ** -31 - 1.0 for x in w])
            if np.dot(v, v) < 1.0:
                break
        assert np.array_equal(r, v) and 0.0 < rr < 1.0
    n = []
    for t in range(20000):
        r, rr = oracle.phi4_direction(seed, t)
        n.append(r / math.sqrt(rr))
    n = np.array(n)
    for a in range(4):
        assert stats.kstest(n[:, a], unit_sphere_marginal_cdf).pvalue > 1e-4, a
    m2 = n.T @ n / len(n)
    assert np.abs(m2 - np.eye(4) / 4).max() < 0.01, m2
    assert np.abs(n.mean(axis=0)).max() < 0.02


def test_hot_and_cold_start():
    D, L = 4, 6
    cold = oracle.phi4_init(D, L, 5, cold=True)
    assert np.all(cold == np.array([1.0, 0.0, 0.0, 0.0]))
    hot = oracle.phi4_init(D, L, 5)
    assert np.abs(np.linalg.norm(hot, axis=1) - 1.0).max() < 1e-15
    for a in range(4):
        assert stats.kstest(hot[:, a], unit_sphere_marginal_cdf).pvalue > 1e-4, a
    other = oracle.phi4_init(D, L, 6)
    assert not np.array_equal(hot, other)


@pytest.mark.parametrize("D,L", [(4, 3), (4, 4), (2, 7), (1, 9)])
def test_labels_are_min_site_components(D, L):
    """Components of random D-dimensional bond masks by a library graph
    routine; every site carries the smallest site of its component."""
    rng = np.random.default_rng(D * 100 + L)
    n = L ** D
    mask = np.zeros(n, dtype=np.uint8)
    for mu in range(D):
        mask |= (rng.random(n) < 0.3).astype(np.uint8) << mu
    lab = oracle.phi4_label(D, L, mask)
    rows, cols = [], []
    for mu, nb in enumerate(lattice_neighbours(D, L)):
        on = (mask >> mu) & 1 == 1
        rows.append(np.arange(n)[on])
        cols.append(nb[on])
    r, c = np.concatenate(rows), np.concatenate(cols)
    g = coo_matrix((np.ones(len(r)), (r, c)), shape=(n, n))
    ncomp, comp = connected_components(g, directed=False)
    smallest = np.full(ncomp, n)
    np.minimum.at(smallest, comp, np.arange(n))
    assert np.array_equal(lab, smallest[comp])


def test_bond_rule_keying_and_probability():
    """A link is bonded only when both projections on r have the same sign,
    with the Philox word of the link (independent Python Philox) below
    1 - E(a); over many sweeps the bonded fraction of links in each bin of
    a matches the mean of 1 - exp(-a) (z-test per bin)."""
    D, L, kappa, seed = 4, 4, 0.304, 9
    nbs = lattice_neighbours(D, L)
    phi = oracle.phi4_init(D, L, seed)
    key = exact.seed_key(seed)
    r, rr = oracle.phi4_direction(seed, 3)
    b = oracle.phi4_bonds(D, L, kappa, seed, 3, phi)
    p = phi @ r
    for s in range(0, L ** D, 7):
        w = exact.philox4x32_10([s, 3, 7, 0], key)
        for mu in range(D):
            y = nbs[mu][s]
            a = (p[s] * p[y]) * (4.0 * kappa) / rr
            want = a > 0 and w[mu] * 2.0 ** -32 < 1.0 - oracle.phi4_expm(a)
            assert bool((b[s] >> mu) & 1) == want, (s, mu)
    bins = np.linspace(0.0, 4.0 * kappa, 9)
    hits = np.zeros(len(bins) - 1)
    expect = np.zeros(len(bins) - 1)
    var = np.zeros(len(bins) - 1)
    for t in range(300):
        phi = oracle.phi4_init(D, L, 1000 + t)
        r, rr = oracle.phi4_direction(1000 + t, t)
        b = oracle.phi4_bonds(D, L, kappa, 1000 + t, t, phi)
        p = phi @ r
        for mu in range(D):
            a = p * p[nbs[mu]] * 4.0 * kappa / rr
            bonded = (b >> mu) & 1
            assert np.all(bonded[a <= 0] == 0)
            pos = a > 0
            k = np.clip(np.digitize(a[pos], bins) - 1, 0, len(hits) - 1)
            pr = 1.0 - np.exp(-a[pos])
            np.add.at(hits, k, bonded[pos])
            np.add.at(expect, k, pr)
            np.add.at(var, k, pr * (1 - pr))
    z = (hits - expect) / np.sqrt(np.maximum(var, 1e-9))
    assert np.abs(z).max() < 5, z


def test_reflection_of_whole_clusters():
    """After an update every cluster is either untouched or reflected as a
    whole about the hyperplane orthogonal to r (eq. 3), as its root's
    Philox bit (independent Python Philox) says; lengths are kept."""
    D, L, kappa, seed, t = 4, 5, 0.304, 21, 4
    phi = oracle.phi4_init(D, L, seed)
    old = phi.copy()
    rec, lab, b = oracle.phi4_sweep(D, L, kappa, seed, t, phi)
    r, rr = oracle.phi4_direction(seed, t)
    n = r / math.sqrt(rr)
    refl = old - 2.0 * (old @ n)[:, None] * n[None, :]
    key = exact.seed_key(seed)
    moved = np.any(phi != old, axis=1)
    for root in np.unique(lab):
        w = exact.philox4x32_10([int(root) >> 7, t, 6, 0], key)
        bit = (w[(int(root) >> 5) & 3] >> (int(root) & 31)) & 1
        sites = lab == root
        if bit:
            assert np.abs(phi[sites] - refl[sites]).max() < 1e-14
        else:
            assert not moved[sites].any()
    assert np.abs(np.linalg.norm(phi, axis=1) - 1.0).max() < 1e-14


def test_kappa_zero_single_site_clusters():
    D, L, seed, t = 4, 4, 3, 2
    phi = oracle.phi4_init(D, L, seed)
    rec, lab, b = oracle.phi4_sweep(D, L, 0.0, seed, t, phi)
    assert not b.any() and np.array_equal(lab, np.arange(L ** D))
    assert rec["n_clusters"] == L ** D and rec["max_cluster"] == 1


def test_record_sums():
    """e_fix and m_fix are exact sums of rint(2^32 x) over links and sites;
    action and |M| follow from them."""
    D, L, kappa, seed = 4, 4, 0.304, 8
    phi = oracle.phi4_init(D, L, seed)
    recs = oracle.phi4_run(D, L, kappa, seed, 0, 3, phi)
    rec = recs[-1]
    e = sum(int(np.rint(np.einsum("ij,ij->i", phi, phi[nb]) * 2.0 ** 32).astype(np.int64).sum())
            for nb in lattice_neighbours(D, L))
    m = np.rint(phi * 2.0 ** 32).astype(np.int64).sum(axis=0)
    assert int(rec["e_fix"]) == e and np.array_equal(rec["m_fix"], m)
    assert rec["action"] == -(2.0 * kappa) * (e * 2.0 ** -32)
    assert abs(rec["m_abs"] - np.linalg.norm(m * 2.0 ** -32)) < 1e-12
    assert int(rec["hist_log2"].sum()) == int(rec["n_clusters"])
    assert list(recs["sweep"]) == [0, 1, 2]


def test_two_vector_link_law():
    """D = 1, L = 2: the two links join the same pair, so t = u . v has
    density sqrt(1 - t^2) exp(4 kappa t); the chain's samples follow it (KS
    against the exact CDF by quadrature)."""
    from scipy.integrate import quad

    kappa = 0.5
    b = 4.0 * kappa
    w = lambda x: math.sqrt(max(0.0, 1.0 - x * x)) * math.exp(b * (x - 1.0))
    z = quad(w, -1.0, 1.0)[0]
    grid = np.linspace(-1.0, 1.0, 2001)
    cdf_vals = np.concatenate([[0.0], np.cumsum([quad(w, grid[i], grid[i + 1])[0] for i in range(2000)])]) / z
    cdf = lambda x: np.interp(x, grid, cdf_vals)
    phi = oracle.phi4_init(1, 2, 5)
    oracle.phi4_run(1, 2, kappa, 5, 0, 20, phi)
    ts = []
    for t in range(20, 40020, 4):
        oracle.phi4_run(1, 2, kappa, 5, t, 4, phi)
        ts.append(float(phi[0] @ phi[1]))
    assert stats.kstest(np.array(ts), cdf).pvalue > 1e-4
    assert abs(np.mean(ts) - exact.o4_link_density_mean(b)) < 0.02


@pytest.mark.parametrize("L,kappa", [(3, 0.3), (8, 1.0), (5, 0.152)])
def test_ring_energy_exact(L, kappa):
    """D = 1: the periodic ring of L unit 4-vectors with weight
    exp(2 kappa sum u_i . u_{i+1}) is solved exactly by its transfer matrix
    (Bessel eigenvalues); the chain's mean link energy agrees within 4.5
    standard errors (errors from 50 bins)."""
    seed, burn, n = 31, 100, 60000
    phi = oracle.phi4_init(1, L, seed)
    oracle.phi4_run(1, L, kappa, seed, 0, burn, phi)
    recs = oracle.phi4_run(1, L, kappa, seed, burn, n, phi)
    u = recs["e_fix"].astype(np.float64) * 2.0 ** -32 / L
    bins = u.reshape(50, -1).mean(axis=1)
    err = bins.std(ddof=1) / math.sqrt(len(bins))
    want = exact.o4_ring_link_energy(2.0 * kappa, L)
    assert abs(u.mean() - want) < 4.5 * err, (u.mean(), want, err)
