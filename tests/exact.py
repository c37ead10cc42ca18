"""Exact results that pin the oracle from outside itself.

Nothing here calls the oracle.  Each function is an independent statement of
a mathematical fact about the 2D Ising model or about the random-number
convention:

* ``philox4x32_10`` -- a second, pure-Python Philox4x32-10 (Salmon et al.,
  SC'11), itself pinned by the published known-answer vectors in
  ``golden/philox_kat.txt``;
* ``threshold_exact`` -- the bond threshold floor(p * 2^32) with
  p = 1 - exp(-2 beta J) evaluated in 60-digit decimal arithmetic;
* ``enumerate_torus`` -- brute-force energies / magnetisations of every
  configuration of a small torus (density of states);
* ``transition_row`` -- the exact one-sweep Swendsen-Wang transition
  probabilities from one configuration of a tiny torus, by enumerating every
  subset of bonded edges and every cluster-spin assignment;
* ``kaufman_energy`` -- Kaufman's exact partition function of the finite
  L x L torus (Ferdinand & Fisher 1969) and the energy per site from it;
* ``onsager_energy`` / ``yang_magnetisation`` -- the infinite-lattice results;
* ``bfs_labels`` -- breadth-first connected components with min-site labels.
"""
from __future__ import annotations

import itertools
import math
from collections import deque
from decimal import Decimal, getcontext

import mpmath
import numpy as np

M32 = 0xFFFFFFFF


def philox4x32_10(ctr, key):
    """Pure-Python Philox4x32-10: ten rounds of two 32x32->64 products."""
    c = [int(v) & M32 for v in ctr]
    k = [int(v) & M32 for v in key]
    for _ in range(10):
        pa = 0xD2511F53 * c[0]
        pb = 0xCD9E8D57 * c[2]
        c = [((pb >> 32) ^ c[1] ^ k[0]) & M32, pb & M32,
             ((pa >> 32) ^ c[3] ^ k[1]) & M32, pa & M32]
        k = [(k[0] + 0x9E3779B9) & M32, (k[1] + 0xBB67AE85) & M32]
    return c


def seed_key(seed: int):
    return [seed & M32, (seed >> 32) & M32]


def bond_word(seed: int, t: int, s: int, d: int) -> int:
    """Uniform word of edge (s, d): word 2*(s&1)+d of counter {s>>1, t, 0, 0}."""
    return philox4x32_10([s >> 1, t, 0, 0], seed_key(seed))[2 * (s & 1) + d]


def flip_spin(seed: int, t: int, r: int) -> int:
    """New spin of the cluster whose minimum site is r: bit r mod 128 of the
    128-bit output at counter {r>>7, t, 1, 0}; set -> -1."""
    w = philox4x32_10([r >> 7, t, 1, 0], seed_key(seed))
    return -1 if (w[(r >> 5) & 3] >> (r & 31)) & 1 else 1


def init_spin(seed: int, s: int) -> int:
    w = philox4x32_10([s, 0, 2, 0], seed_key(seed))
    return -1 if w[0] & 1 else 1


def threshold_exact(beta, J=1) -> int:
    """floor((1 - exp(-2 beta J)) * 2^32) in 60-digit decimal arithmetic."""
    getcontext().prec = 60
    b = Decimal(str(beta)) if not isinstance(beta, Decimal) else beta
    p = Decimal(1) - (Decimal(-2) * b * Decimal(str(J))).exp()
    v = int((p * Decimal(2 ** 32)).to_integral_value(rounding="ROUND_FLOOR"))
    return min(v, M32)


def beta_c_decimal() -> Decimal:
    getcontext().prec = 60
    return (Decimal(1) + Decimal(2).sqrt()).ln() / 2


def torus_edges(L: int):
    """All 2N edges (s, E(s)) and (s, N(s)); for L = 2 pairs repeat."""
    out = []
    for s in range(L * L):
        x, y = s % L, s // L
        out.append((s, y * L + (x + 1) % L))
        out.append((s, ((y + 1) % L) * L + x))
    return out


def enumerate_torus(L: int):
    """(e_sum, m_sum) of all 2^N configurations; bit s of the index = spin -1."""
    n = L * L
    idx = np.arange(2 ** n, dtype=np.int64)
    spins = 1 - 2 * ((idx[:, None] >> np.arange(n)[None, :]) & 1)
    e = np.zeros(2 ** n, dtype=np.int64)
    for a, b in torus_edges(L):
        e += spins[:, a] * spins[:, b]
    return e, spins.sum(axis=1)


def components(n: int, edges):
    parent = list(range(n))

    def find(a):
        while parent[a] != a:
            parent[a] = parent[parent[a]]
            a = parent[a]
        return a

    for a, b in edges:
        ra, rb = find(a), find(b)
        if ra != rb:
            parent[max(ra, rb)] = min(ra, rb)
    return [find(a) for a in range(n)]


def transition_row(L: int, start, P):
    """Exact distribution of the configuration after one sweep from `start`.

    Every satisfied edge is bonded independently with probability P; each
    cluster of the resulting bond graph takes +1 or -1 with probability 1/2.
    Returns {code: probability} with code bit s set iff new spin s is -1.
    """
    n = L * L
    start = list(start)
    sat = [e for e in torus_edges(L) if start[e[0]] == start[e[1]]]
    row: dict[int, float] = {}
    for mask in range(2 ** len(sat)):
        chosen = [sat[i] for i in range(len(sat)) if (mask >> i) & 1]
        w = P ** len(chosen) * (1 - P) ** (len(sat) - len(chosen))
        lab = components(n, chosen)
        roots = sorted(set(lab))
        share = w / 2 ** len(roots)
        for bits in range(2 ** len(roots)):
            down = {r for i, r in enumerate(roots) if (bits >> i) & 1}
            code = 0
            for s in range(n):
                if lab[s] in down:
                    code |= 1 << s
            row[code] = row.get(code, 0.0) + share
    return row


def code_to_spins(code: int, n: int):
    return [(-1 if (code >> s) & 1 else 1) for s in range(n)]


def bfs_labels(L: int, bond_mask: np.ndarray) -> np.ndarray:
    """Min-site component labels of the bond graph by breadth-first search."""
    n = L * L
    adj = [[] for _ in range(n)]
    for s in range(n):
        x, y = s % L, s // L
        if bond_mask[s] & 1:
            e = y * L + (x + 1) % L
            adj[s].append(e)
            adj[e].append(s)
        if bond_mask[s] & 2:
            nn = ((y + 1) % L) * L + x
            adj[s].append(nn)
            adj[nn].append(s)
    lab = np.full(n, -1, dtype=np.int64)
    for s in range(n):  # ascending, so the first site reached is the minimum
        if lab[s] >= 0:
            continue
        lab[s] = s
        q = deque([s])
        while q:
            a = q.popleft()
            for b in adj[a]:
                if lab[b] < 0:
                    lab[b] = s
                    q.append(b)
    return lab.astype(np.uint32)


# ---------------------------------------------------------------------------
# Kaufman (1949) exact partition function of the L x L torus, in the form of
# Ferdinand & Fisher (1969):
#   Z = 1/2 (2 sinh 2K)^(N/2) (Z1 + Z2 + Z3 + Z4),
#   Z1 = prod_r 2 cosh(L g_{2r+1}/2), Z2 = prod_r 2 sinh(L g_{2r+1}/2),
#   Z3 = prod_r 2 cosh(L g_{2r}/2),   Z4 = prod_r 2 sinh(L g_{2r}/2),
#   cosh g_l = cosh 2K coth 2K - cos(pi l / L)  (l >= 1),
#   g_0 = 2K + ln tanh K  (signed).
# ---------------------------------------------------------------------------

def _kaufman_lnZ(K, L: int):
    K = mpmath.mpf(K)
    c = mpmath.cosh(2 * K) * mpmath.coth(2 * K)

    def gamma(l):
        if l == 0:
            return 2 * K + mpmath.log(mpmath.tanh(K))
        return mpmath.acosh(c - mpmath.cos(mpmath.pi * l / L))

    z1 = z2 = z3 = z4 = mpmath.mpf(1)
    for r in range(L):
        go, ge = gamma(2 * r + 1), gamma(2 * r)
        z1 *= 2 * mpmath.cosh(L * go / 2)
        z2 *= 2 * mpmath.sinh(L * go / 2)
        z3 *= 2 * mpmath.cosh(L * ge / 2)
        z4 *= 2 * mpmath.sinh(L * ge / 2)
    n = L * L
    return mpmath.log(mpmath.mpf(1) / 2) + (mpmath.mpf(n) / 2) * mpmath.log(
        2 * mpmath.sinh(2 * K)) + mpmath.log(z1 + z2 + z3 + z4)


def kaufman_lnZ(beta, L: int, dps: int = 40):
    with mpmath.workdps(dps):
        return _kaufman_lnZ(mpmath.mpf(beta), L)


def kaufman_energy(beta, L: int, dps: int = 40) -> float:
    """Exact <E>/N per site (J = 1) of the L x L torus: -(1/N) d lnZ / dK."""
    with mpmath.workdps(dps):
        d = mpmath.diff(lambda k: _kaufman_lnZ(k, L), mpmath.mpf(beta))
        return float(-d / (L * L))


def onsager_energy(beta) -> float:
    """Infinite-lattice energy per site (J = 1)."""
    b = mpmath.mpf(beta)
    k = 2 * mpmath.sinh(2 * b) / mpmath.cosh(2 * b) ** 2
    Kk = mpmath.ellipk(k ** 2)
    return float(-mpmath.coth(2 * b) * (1 + (2 / mpmath.pi) * (2 * mpmath.tanh(2 * b) ** 2 - 1) * Kk))


def yang_magnetisation(beta) -> float:
    b = mpmath.mpf(beta)
    return float((1 - mpmath.sinh(2 * b) ** -4) ** (mpmath.mpf(1) / 8))


def chi2_pvalue(observed, expected, min_expected: float = 5.0):
    """Pearson chi-squared with bins of expected count < min_expected pooled."""
    from scipy import stats

    obs = np.asarray(observed, dtype=np.float64)
    exp = np.asarray(expected, dtype=np.float64)
    order = np.argsort(exp)
    obs, exp = obs[order], exp[order]
    po, pe, acc_o, acc_e = [], [], 0.0, 0.0
    for o, e in zip(obs, exp):
        acc_o += o
        acc_e += e
        if acc_e >= min_expected:
            po.append(acc_o)
            pe.append(acc_e)
            acc_o = acc_e = 0.0
    if acc_e > 0:
        if pe:
            po[-1] += acc_o
            pe[-1] += acc_e
        else:
            po.append(acc_o)
            pe.append(acc_e)
    po, pe = np.array(po), np.array(pe)
    chi2 = float(((po - pe) ** 2 / pe).sum())
    dof = max(len(pe) - 1, 1)
    return chi2, dof, float(stats.chi2.sf(chi2, dof))


def all_subsets(n):
    return itertools.product((0, 1), repeat=n)


# ------------------------------------------------------- O(4) ring (exact)
def o4_ring_link_energy(beta: float, L: int, lmax: int = 80) -> float:
    """<u_i . u_{i+1}> on a periodic ring of L unit 4-vectors with weight
    exp(beta sum_i u_i . u_{i+1}) and the uniform measure on S^3.

    Transfer matrix: by the Funk-Hecke theorem the kernel exp(beta u . v)
    acts on the degree-l harmonics of S^3 (multiplicity (l+1)^2) with
    eigenvalue lambda_l = 2 I_{l+1}(beta) / beta (normalised measure), so
    Z = sum_l (l+1)^2 lambda_l^L and <u . v> = (1/L) d ln Z / d beta, with
    I_nu' = (I_{nu-1} + I_{nu+1}) / 2.  Scaled Bessel functions keep the
    terms finite; the common factor e^beta cancels in the ratio."""
    from scipy.special import ive

    lam0 = 2.0 * ive(1, beta) / beta
    num = den = 0.0
    for l in range(lmax):
        nu = l + 1
        i_nu = ive(nu, beta)
        d_nu = 0.5 * (ive(nu - 1, beta) + ive(nu + 1, beta))
        lam = 2.0 * i_nu / beta
        # derivative of the scaled eigenvalue plus the e^beta factor's share
        dlam = 2.0 * d_nu / beta - 2.0 * i_nu / beta ** 2 - lam
        w = (l + 1) ** 2
        ratio = lam / lam0
        den += w * ratio ** L
        num += w * L * ratio ** (L - 1) * dlam / lam0
    # the scaled eigenvalues are e^-beta lambda_l: add back d(beta)/d(beta) = 1 per link
    return num / den / L + 1.0


def o4_link_density_mean(b: float) -> float:
    """Mean of t = u . v for two unit 4-vectors with weight exp(b t): the
    relative angle of uniform vectors has density (2/pi) sqrt(1 - t^2);
    by quadrature."""
    from scipy.integrate import quad

    w = lambda t: math.sqrt(1.0 - t * t) * math.exp(b * (t - 1.0))
    z = quad(w, -1.0, 1.0)[0]
    return quad(lambda t: t * w(t), -1.0, 1.0)[0] / z
