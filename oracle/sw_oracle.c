/*
 * sw_oracle.c -- plain, sequential CPU oracle for one Swendsen-Wang sweep of
 * the 2D Ising model on an L x L periodic square lattice.
 *
 * TEST INFRASTRUCTURE ONLY.  Nothing in the product path may link, load or
 * call this file: only the test-suite, the smoke check and the CPU-baseline
 * leg of the benchmark use it.  It shares no code, header, table or constant
 * generator with the HIP library; it is written to be read against the paper
 * (Protzman & Giedt, "GPU Acceleration of Swendson-Wang Dynamics"), not to be
 * fast.
 *
 * Conventions fixed here (the paper is silent on all of them; the readings
 * are listed in the design notes):
 *   site index        s = y*L + x, x fastest, 0 <= x,y < L, periodic.
 *   E(s)              y*L + (x+1 mod L)          (direction d = 0)
 *   N(s)              ((y+1) mod L)*L + x        (direction d = 1)
 *   Each site owns the two edges to E(s) and N(s), so all 2N torus edges are
 *   visited exactly once (Sec. 2.1: a thread checks two of its four
 *   neighbours; Fig. 2 caption).
 *   Spins are int8 +1 / -1.  Labels are uint32 (min site index of the
 *   cluster, Sec. 2.3 "lowest value label" with initial label = site index).
 *
 * Randomness (the paper names no generator, Sec. 2.1 only says "a random
 * number is generated"): counter-based Philox4x32-10, key = seed, with a
 * domain tag in counter word 2:
 *   bonds  : w(s,d) = word 2*(s&1)+d of Philox({s>>1, t, 0, 0})
 *   flips  : bit (r mod 128) of the 128-bit Philox({r>>7, t, 1, 0}) output,
 *            i.e. word (r>>5)&3, bit r&31;  bit 1 -> spin -1, bit 0 -> +1
 *   init   : bit 0 of word 0 of Philox({s, 0, 2, 0}); 1 -> -1, 0 -> +1
 *
 * Parity pins (all in the CPU test-suite): Philox known-answer vectors,
 * the closed form of the bond threshold at beta_c, brute-force BFS labels,
 * exact enumeration of the 4x4 torus, exact one-sweep transition rows of the
 * 2x2 and 3x3 tori, the Ferdinand-Fisher finite-size energy at beta_c, the
 * Onsager energy off criticality, and integer invariants.
 */
#include <math.h>
#include <stdint.h>
#include <stdlib.h>
#include <string.h>

#include "sw_oracle.h"

/* ------------------------------------------------------------------ */
/* Philox4x32-10 (Salmon, Moraes, Dror, Shaw, SC'11, Sec. 4.1):        */
/* each round multiplies counter words 0 and 2 by two fixed odd        */
/* constants, swaps in the high halves xor-ed with the other counter   */
/* words and the round key; the key is advanced by the Weyl constants  */
/* (golden ratio and sqrt(3)-1) between rounds.                        */
/* ------------------------------------------------------------------ */
void orc_philox4x32_10(const uint32_t ctr[4], const uint32_t key[2],
                       uint32_t out[4])
{
    uint32_t x0 = ctr[0], x1 = ctr[1], x2 = ctr[2], x3 = ctr[3];
    uint32_t k0 = key[0], k1 = key[1];
    for (int round = 0; round < 10; ++round) {
        uint64_t prod_a = (uint64_t)0xD2511F53u * (uint64_t)x0;
        uint64_t prod_b = (uint64_t)0xCD9E8D57u * (uint64_t)x2;
        uint32_t hi_a = (uint32_t)(prod_a >> 32), lo_a = (uint32_t)prod_a;
        uint32_t hi_b = (uint32_t)(prod_b >> 32), lo_b = (uint32_t)prod_b;
        x0 = hi_b ^ x1 ^ k0;
        x1 = lo_b;
        x2 = hi_a ^ x3 ^ k1;
        x3 = lo_a;
        k0 += 0x9E3779B9u;
        k1 += 0xBB67AE85u;
    }
    out[0] = x0; out[1] = x1; out[2] = x2; out[3] = x3;
}

static void philox_seed(uint64_t seed, uint32_t c0, uint32_t c1, uint32_t c2,
                        uint32_t out[4])
{
    uint32_t ctr[4] = {c0, c1, c2, 0u};
    uint32_t key[2] = {(uint32_t)(seed & 0xFFFFFFFFu), (uint32_t)(seed >> 32)};
    orc_philox4x32_10(ctr, key, out);
}

/* ------------------------------------------------------------------ */
/* Bond probability (Sec. 2.1).  The printed p = 1 - exp(-1/kT) puts   */
/* T_c near 1.13, contradicting the paper's own T_c ~ 2.25 (Sec. 4);   */
/* the reading used is p = 1 - exp(-2 beta J), evaluated once in FP64  */
/* and turned into a 32-bit threshold so that P(bond) = T / 2^32.      */
/* ------------------------------------------------------------------ */
uint32_t orc_threshold(double beta, double J)
{
    double p = -expm1(-2.0 * beta * J);
    if (!(p > 0.0)) return 0u;
    double scaled = floor(ldexp(p, 32));
    if (scaled >= 4294967296.0) return 0xFFFFFFFFu;
    return (uint32_t)scaled;
}

/* Initial configuration (Fig. 1): hot = i.i.d. +-1 with probability 1/2,
 * cold = all +1. */
void orc_init(int32_t L, uint64_t seed, int32_t cold, int8_t *spins)
{
    uint32_t n = (uint32_t)L * (uint32_t)L;
    for (uint32_t s = 0; s < n; ++s) {
        if (cold) { spins[s] = 1; continue; }
        uint32_t r[4];
        philox_seed(seed, s, 0u, 2u, r);
        spins[s] = (r[0] & 1u) ? (int8_t)-1 : (int8_t)1;
    }
}

static uint32_t east_of(uint32_t s, uint32_t L)
{
    uint32_t x = s % L, y = s / L;
    return y * L + (x + 1u) % L;
}

static uint32_t north_of(uint32_t s, uint32_t L)
{
    uint32_t x = s % L, y = s / L;
    return ((y + 1u) % L) * L + x;
}

/* Sec. 2.1, Bond formation: an edge is bonded iff both ends carry the same
 * spin and the edge's uniform 32-bit word is below the threshold.
 * bonds[s] bit 0 = bond (s, E(s)), bit 1 = bond (s, N(s)). */
void orc_bonds(int32_t L, uint32_t T, uint64_t seed, uint32_t t,
               const int8_t *spins, uint8_t *bonds)
{
    uint32_t n = (uint32_t)L * (uint32_t)L;
    for (uint32_t s = 0; s < n; ++s) {
        uint32_t r[4];
        philox_seed(seed, s >> 1, t, 0u, r);
        uint32_t wE = r[2u * (s & 1u) + 0u];
        uint32_t wN = r[2u * (s & 1u) + 1u];
        uint8_t b = 0;
        if (spins[s] == spins[east_of(s, (uint32_t)L)] && wE < T) b |= 1u;
        if (spins[s] == spins[north_of(s, (uint32_t)L)] && wN < T) b |= 2u;
        bonds[s] = b;
    }
}

/* Sec. 2.3, Cluster formation: connected components of the bond graph.
 * Textbook sequential union-find; the root of every set is kept at the
 * smallest site index of the set, so after the final find every site
 * carries the lowest label of its cluster. `labels` doubles as the
 * parent array. */
static uint32_t uf_find(uint32_t *parent, uint32_t a)
{
    while (parent[a] != a) {
        parent[a] = parent[parent[a]];
        a = parent[a];
    }
    return a;
}

static void uf_union(uint32_t *parent, uint32_t a, uint32_t b)
{
    uint32_t ra = uf_find(parent, a), rb = uf_find(parent, b);
    if (ra == rb) return;
    if (ra < rb) parent[rb] = ra;
    else parent[ra] = rb;
}

void orc_label(int32_t L, const uint8_t *bonds, uint32_t *labels)
{
    uint32_t n = (uint32_t)L * (uint32_t)L;
    for (uint32_t s = 0; s < n; ++s) labels[s] = s;
    for (uint32_t s = 0; s < n; ++s) {
        if (bonds[s] & 1u) uf_union(labels, s, east_of(s, (uint32_t)L));
        if (bonds[s] & 2u) uf_union(labels, s, north_of(s, (uint32_t)L));
    }
    for (uint32_t s = 0; s < n; ++s) labels[s] = uf_find(labels, s);
}

/* Sec. 2.4, Assignment of new spins: every cluster draws a fresh spin,
 * up or down with probability 1/2, independent of its old spin; the draw is
 * keyed by the cluster's canonical (minimum-site) label. */
int32_t orc_flip_spin(uint64_t seed, uint32_t t, uint32_t root)
{
    uint32_t r[4];
    philox_seed(seed, root >> 7, t, 1u, r);
    uint32_t bit = (r[(root >> 5) & 3u] >> (root & 31u)) & 1u;
    return bit ? -1 : 1;
}

void orc_assign(int32_t L, uint64_t seed, uint32_t t, const uint32_t *labels,
                int8_t *spins)
{
    uint32_t n = (uint32_t)L * (uint32_t)L;
    for (uint32_t s = 0; s < n; ++s)
        spins[s] = (int8_t)orc_flip_spin(seed, t, labels[s]);
}

static void cluster_stats(uint32_t n, const uint32_t *labels, orc_obs *rec, uint64_t *dense);

/* Sec. 2.5 measurement: H = -J sum_<ij> s_i s_j over the 2N torus edges,
 * M = sum_i s_i (the paper divides by N; the exact integer sum is kept and
 * divided at the end).  Cluster statistics come from the labels of the
 * sweep's bonds.  `dense` (may be NULL) receives counts[size] for
 * size = 0..N. */
void orc_observe(int32_t L, double J, uint64_t sweep, const int8_t *spins,
                 const uint32_t *labels, orc_obs *rec, uint64_t *dense)
{
    uint32_t n = (uint32_t)L * (uint32_t)L;
    int64_t e = 0, m = 0;
    for (uint32_t s = 0; s < n; ++s) {
        int32_t si = spins[s];
        e += si * spins[east_of(s, (uint32_t)L)];
        e += si * spins[north_of(s, (uint32_t)L)];
        m += si;
    }
    memset(rec, 0, sizeof(*rec));
    rec->sweep = sweep;
    rec->e_sum = e;
    rec->energy = -J * (double)e;
    rec->m_sum = m;
    cluster_stats(n, labels, rec, dense);
}

/* Cluster statistics of a labelling of n sites (each label the smallest
 * site of its cluster): count, largest size, sum of squared sizes and the
 * log2-binned size histogram; `dense` (may be NULL) receives counts[size]
 * for size = 0..n. */
static void cluster_stats(uint32_t n, const uint32_t *labels, orc_obs *rec, uint64_t *dense)
{
    if (dense) memset(dense, 0, sizeof(uint64_t) * ((size_t)n + 1u));
    if (!labels) return;
    uint32_t *size = (uint32_t *)calloc(n, sizeof(uint32_t));
    if (!size) return;
    for (uint32_t s = 0; s < n; ++s) size[labels[s]] += 1u;
    for (uint32_t r = 0; r < n; ++r) {
        if (size[r] == 0u) continue;
        uint64_t sz = size[r];
        rec->n_clusters += 1u;
        if (sz > rec->max_cluster) rec->max_cluster = sz;
        rec->sum_sq_sizes += sz * sz;
        int k = 0;
        while ((sz >> (k + 1)) != 0u) ++k;
        rec->hist_log2[k] += 1u;
        if (dense) dense[sz] += 1u;
    }
    free(size);
}

/* One full sweep t (Sec. 2, steps 2.1-2.5): bonds, clusters, new spins,
 * measurement of the new configuration.  `spins` is updated in place;
 * `labels` (N words) and `bonds` (N bytes) receive the sweep's clusters and
 * bonds; `rec` the record; `dense` (NULL or N+1 words) the exact cluster
 * size histogram.  Returns 0, or -1 on allocation failure. */
int orc_sweep(int32_t L, double J, uint32_t T, uint64_t seed, uint32_t t,
              int8_t *spins, uint32_t *labels, uint8_t *bonds, orc_obs *rec,
              uint64_t *dense)
{
    uint32_t n = (uint32_t)L * (uint32_t)L;
    uint8_t *b = bonds ? bonds : (uint8_t *)malloc(n);
    uint32_t *lab = labels ? labels : (uint32_t *)malloc(sizeof(uint32_t) * n);
    if (!b || !lab) {
        if (!bonds) free(b);
        if (!labels) free(lab);
        return -1;
    }
    orc_bonds(L, T, seed, t, spins, b);
    orc_label(L, b, lab);
    orc_assign(L, seed, t, lab, spins);
    if (rec) orc_observe(L, J, t, spins, lab, rec, dense);
    if (!bonds) free(b);
    if (!labels) free(lab);
    return 0;
}

/* Runs `count` consecutive sweeps t0, t0+1, ... writing one record each. */
int orc_run(int32_t L, double J, uint32_t T, uint64_t seed, uint32_t t0,
            int64_t count, int8_t *spins, orc_obs *recs)
{
    uint32_t n = (uint32_t)L * (uint32_t)L;
    uint8_t *b = (uint8_t *)malloc(n);
    uint32_t *lab = (uint32_t *)malloc(sizeof(uint32_t) * n);
    if (!b || !lab) { free(b); free(lab); return -1; }
    for (int64_t i = 0; i < count; ++i) {
        uint32_t t = t0 + (uint32_t)i;
        orc_bonds(L, T, seed, t, spins, b);
        orc_label(L, b, lab);
        orc_assign(L, seed, t, lab, spins);
        if (recs) orc_observe(L, J, t, spins, lab, &recs[i], NULL);
    }
    free(b);
    free(lab);
    return 0;
}

/* Ensemble helper for the exact-enumeration pins: runs `nchains`
 * independent chains (seeds seed0, seed0+1, ...) from a hot start for
 * `nsweeps` sweeps each and stores the final e_sum and m_sum of each. */
int orc_chains(int32_t L, double J, uint32_t T, uint64_t seed0, int64_t nchains,
               int32_t nsweeps, int64_t *e_out, int64_t *m_out)
{
    uint32_t n = (uint32_t)L * (uint32_t)L;
    int8_t *sp = (int8_t *)malloc(n);
    if (!sp) return -1;
    for (int64_t c = 0; c < nchains; ++c) {
        uint64_t seed = seed0 + (uint64_t)c;
        orc_init(L, seed, 0, sp);
        if (orc_run(L, J, T, seed, 0u, nsweeps, sp, NULL) != 0) { free(sp); return -1; }
        orc_obs rec;
        orc_observe(L, J, 0, sp, NULL, &rec, NULL);
        e_out[c] = rec.e_sum;
        m_out[c] = rec.m_sum;
    }
    free(sp);
    return 0;
}

/* One sweep from each of `nseeds` seeds, all from the same start state at
 * sweep index t; stores each resulting configuration as an integer code
 * (bit s set iff spin s is -1).  For the tiny-torus transition pins. */
int orc_one_step_codes(int32_t L, uint32_t T, uint64_t seed0, int64_t nseeds,
                       uint32_t t, const int8_t *start, uint64_t *codes)
{
    uint32_t n = (uint32_t)L * (uint32_t)L;
    if (n > 64u) return -1;
    int8_t sp[64];
    for (int64_t c = 0; c < nseeds; ++c) {
        memcpy(sp, start, n);
        if (orc_sweep(L, 1.0, T, seed0 + (uint64_t)c, t, sp, NULL, NULL, NULL, NULL) != 0)
            return -1;
        uint64_t code = 0;
        for (uint32_t s = 0; s < n; ++s)
            if (sp[s] < 0) code |= (uint64_t)1 << s;
        codes[c] = code;
    }
    return 0;
}

/* ================================================================== */
/* q-state Potts model, the paper's other named target of the same     */
/* method (Sec. 1, Sec. 6): H = -J sum_<ij> delta(s_i, s_j) with spins  */
/* 0..q-1.  One sweep is the same three steps: an edge with equal end  */
/* spins is bonded with p = 1 - exp(-beta J) (one coupling per equal   */
/* pair; q = 2 is the Ising model at half the coupling), clusters are  */
/* the components of the bond graph, and every cluster draws a new     */
/* value uniformly from 0..q-1.                                        */
/* ================================================================== */
uint32_t orc_potts_threshold(double beta, double J)
{
    double p = -expm1(-beta * J);
    if (!(p > 0.0)) return 0u;
    double scaled = floor(ldexp(p, 32));
    if (scaled >= 4294967296.0) return 0xFFFFFFFFu;
    return (uint32_t)scaled;
}

/* A value in 0..q-1 from a uniform 32-bit word: floor(w q / 2^32). */
static int8_t potts_value(uint32_t w, uint32_t q)
{
    return (int8_t)(((uint64_t)w * q) >> 32);
}

/* Hot start: value of word 0 for counter {s, 0, 2, 0}; cold: all 0. */
void orc_potts_init(int32_t L, uint64_t seed, int32_t q, int32_t cold, int8_t *spins)
{
    uint32_t n = (uint32_t)L * (uint32_t)L;
    for (uint32_t s = 0; s < n; ++s) {
        if (cold) { spins[s] = 0; continue; }
        uint32_t r[4];
        philox_seed(seed, s, 0u, 2u, r);
        spins[s] = potts_value(r[0], (uint32_t)q);
    }
}

/* New value of the cluster whose smallest site is r in sweep t: word r mod 4
 * of the output for counter {r >> 2, t, 3, 0}. */
int32_t orc_potts_spin(uint64_t seed, uint32_t t, uint32_t root, int32_t q)
{
    uint32_t r[4];
    philox_seed(seed, root >> 2, t, 3u, r);
    return potts_value(r[root & 3u], (uint32_t)q);
}

void orc_potts_assign(int32_t L, uint64_t seed, uint32_t t, int32_t q, const uint32_t *labels,
                      int8_t *spins)
{
    uint32_t n = (uint32_t)L * (uint32_t)L;
    for (uint32_t s = 0; s < n; ++s)
        spins[s] = (int8_t)orc_potts_spin(seed, t, labels[s], q);
}

/* Measurement: e_sum = number of the 2N torus edges whose ends are equal
 * (H = -J e_sum); m_sum = population of the most populated value; cluster
 * statistics as for the Ising model. */
void orc_potts_observe(int32_t L, double J, int32_t q, uint64_t sweep, const int8_t *spins,
                       const uint32_t *labels, orc_obs *rec, uint64_t *dense)
{
    uint32_t n = (uint32_t)L * (uint32_t)L;
    int64_t e = 0;
    int64_t count[256] = {0};
    for (uint32_t s = 0; s < n; ++s) {
        e += spins[s] == spins[east_of(s, (uint32_t)L)];
        e += spins[s] == spins[north_of(s, (uint32_t)L)];
        count[(uint8_t)spins[s]] += 1;
    }
    /* cluster statistics exactly as for the Ising model */
    orc_observe(L, J, sweep, spins, labels, rec, dense);
    int64_t m = 0;
    for (int32_t k = 0; k < q; ++k)
        if (count[k] > m) m = count[k];
    rec->e_sum = e;
    rec->energy = -J * (double)e;
    rec->m_sum = m;
}

int orc_potts_sweep(int32_t L, double J, uint32_t T, int32_t q, uint64_t seed, uint32_t t,
                    int8_t *spins, uint32_t *labels, orc_obs *rec)
{
    uint32_t n = (uint32_t)L * (uint32_t)L;
    uint8_t *b = (uint8_t *)malloc(n);
    uint32_t *lab = labels ? labels : (uint32_t *)malloc(sizeof(uint32_t) * n);
    if (!b || !lab) {
        free(b);
        if (!labels) free(lab);
        return -1;
    }
    orc_bonds(L, T, seed, t, spins, b);
    orc_label(L, b, lab);
    orc_potts_assign(L, seed, t, q, lab, spins);
    if (rec) orc_potts_observe(L, J, q, t, spins, lab, rec, NULL);
    free(b);
    if (!labels) free(lab);
    return 0;
}

int orc_potts_run(int32_t L, double J, uint32_t T, int32_t q, uint64_t seed, uint32_t t0,
                  int64_t count, int8_t *spins, orc_obs *recs)
{
    uint32_t n = (uint32_t)L * (uint32_t)L;
    uint32_t *lab = (uint32_t *)malloc(sizeof(uint32_t) * n);
    if (!lab) return -1;
    for (int64_t i = 0; i < count; ++i) {
        if (orc_potts_sweep(L, J, T, q, seed, t0 + (uint32_t)i, spins, lab, recs ? &recs[i] : NULL) != 0) {
            free(lab);
            return -1;
        }
    }
    free(lab);
    return 0;
}

/* Ensemble helper: independent hot-start chains (seeds seed0, seed0+1, ...),
 * `nsweeps` sweeps each; final e_sum (equal pairs) and the count of value 0. */
int orc_potts_chains(int32_t L, double J, uint32_t T, int32_t q, uint64_t seed0, int64_t nchains,
                     int32_t nsweeps, int64_t *e_out, int64_t *n0_out)
{
    uint32_t n = (uint32_t)L * (uint32_t)L;
    int8_t *sp = (int8_t *)malloc(n);
    if (!sp) return -1;
    for (int64_t c = 0; c < nchains; ++c) {
        uint64_t seed = seed0 + (uint64_t)c;
        orc_potts_init(L, seed, q, 0, sp);
        if (orc_potts_run(L, J, T, q, seed, 0u, nsweeps, sp, NULL) != 0) { free(sp); return -1; }
        int64_t e = 0, z = 0;
        for (uint32_t s = 0; s < n; ++s) {
            e += sp[s] == sp[east_of(s, (uint32_t)L)];
            e += sp[s] == sp[north_of(s, (uint32_t)L)];
            z += sp[s] == 0;
        }
        e_out[c] = e;
        n0_out[c] = z;
    }
    free(sp);
    return 0;
}

/* ================================================================== */
/* Simple cubic lattice, L x L x L, periodic: the other geometry the   */
/* paper names for the same method (Sec. 6).  The sweep is unchanged:  */
/* bond equal neighbours with the model's threshold, take connected    */
/* components, give every cluster a fresh spin (Ising, q = 0) or value  */
/* (Potts, q = 2..8) keyed by its smallest site, measure.              */
/*   site index   s = (z*L + y)*L + x, x fastest                       */
/*   direction d  0: +x, 1: +y, 2: +z; each site owns the three edges  */
/*                to its +x, +y and +z neighbours (all 3N edges once)  */
/*   bond word    word d of Philox({s, t, 4, 0}) (one call per site)   */
/*   hot start    word 0 of Philox({s, 0, 2, 0}), read as in 2D         */
/*   new spins    orc_flip_spin / orc_potts_spin of the root, as in 2D */
/* The caller passes the threshold: orc_threshold(beta, J) for the      */
/* Ising model, orc_potts_threshold(beta, J) for Potts.                 */
/* ================================================================== */
static uint32_t cubic_step(uint32_t s, uint32_t L, int d)
{
    uint32_t x = s % L, y = (s / L) % L, z = s / L / L;
    if (d == 0) x = (x + 1u) % L;
    else if (d == 1) y = (y + 1u) % L;
    else z = (z + 1u) % L;
    return (z * L + y) * L + x;
}

static uint32_t cubic_sites(int32_t L)
{
    return (uint32_t)L * (uint32_t)L * (uint32_t)L;
}

void orc_cubic_init(int32_t L, uint64_t seed, int32_t q, int32_t cold, int8_t *spins)
{
    uint32_t n = cubic_sites(L);
    for (uint32_t s = 0; s < n; ++s) {
        if (cold) { spins[s] = q ? (int8_t)0 : (int8_t)1; continue; }
        uint32_t r[4];
        philox_seed(seed, s, 0u, 2u, r);
        if (q) spins[s] = potts_value(r[0], (uint32_t)q);
        else spins[s] = (int8_t)((r[0] & 1u) ? -1 : 1);
    }
}

/* bonds[s] bit d = bond (s, step d of s). */
void orc_cubic_bonds(int32_t L, uint32_t T, uint64_t seed, uint32_t t,
                     const int8_t *spins, uint8_t *bonds)
{
    uint32_t n = cubic_sites(L);
    for (uint32_t s = 0; s < n; ++s) {
        uint32_t r[4];
        philox_seed(seed, s, t, 4u, r);
        uint8_t b = 0;
        for (int d = 0; d < 3; ++d) {
            uint32_t nb = cubic_step(s, (uint32_t)L, d);
            if (spins[s] == spins[nb] && r[d] < T) b |= (uint8_t)(1u << d);
        }
        bonds[s] = b;
    }
}

void orc_cubic_label(int32_t L, const uint8_t *bonds, uint32_t *labels)
{
    uint32_t n = cubic_sites(L);
    for (uint32_t s = 0; s < n; ++s) labels[s] = s;
    for (uint32_t s = 0; s < n; ++s)
        for (int d = 0; d < 3; ++d)
            if (bonds[s] & (1u << d)) uf_union(labels, s, cubic_step(s, (uint32_t)L, d));
    for (uint32_t s = 0; s < n; ++s) labels[s] = uf_find(labels, s);
}

/* Ising: e_sum = sum over the 3N edges of s_i s_j, m_sum = sum of s_i.
 * Potts: e_sum = number of the 3N edges with equal ends, m_sum = population
 * of the most populated value.  Cluster statistics as in 2D. */
void orc_cubic_observe(int32_t L, double J, int32_t q, uint64_t sweep, const int8_t *spins,
                       const uint32_t *labels, orc_obs *rec, uint64_t *dense)
{
    uint32_t n = cubic_sites(L);
    int64_t e = 0, m = 0;
    int64_t count[256] = {0};
    for (uint32_t s = 0; s < n; ++s) {
        for (int d = 0; d < 3; ++d) {
            int8_t o = spins[cubic_step(s, (uint32_t)L, d)];
            e += q ? (int64_t)(spins[s] == o) : (int64_t)spins[s] * o;
        }
        m += spins[s];
        count[(uint8_t)spins[s]] += 1;
    }
    if (q) {
        m = 0;
        for (int32_t k = 0; k < q; ++k)
            if (count[k] > m) m = count[k];
    }
    memset(rec, 0, sizeof(*rec));
    rec->sweep = sweep;
    rec->e_sum = e;
    rec->energy = -J * (double)e;
    rec->m_sum = m;
    cluster_stats(n, labels, rec, dense);
}

int orc_cubic_sweep(int32_t L, double J, uint32_t T, int32_t q, uint64_t seed, uint32_t t,
                    int8_t *spins, uint32_t *labels, uint8_t *bonds, orc_obs *rec, uint64_t *dense)
{
    uint32_t n = cubic_sites(L);
    uint8_t *b = bonds ? bonds : (uint8_t *)malloc(n);
    uint32_t *lab = labels ? labels : (uint32_t *)malloc(sizeof(uint32_t) * n);
    if (!b || !lab) {
        if (!bonds) free(b);
        if (!labels) free(lab);
        return -1;
    }
    orc_cubic_bonds(L, T, seed, t, spins, b);
    orc_cubic_label(L, b, lab);
    for (uint32_t s = 0; s < n; ++s)
        spins[s] = (int8_t)(q ? orc_potts_spin(seed, t, lab[s], q) : orc_flip_spin(seed, t, lab[s]));
    if (rec) orc_cubic_observe(L, J, q, t, spins, lab, rec, dense);
    if (!bonds) free(b);
    if (!labels) free(lab);
    return 0;
}

int orc_cubic_run(int32_t L, double J, uint32_t T, int32_t q, uint64_t seed, uint32_t t0,
                  int64_t count, int8_t *spins, orc_obs *recs)
{
    uint32_t n = cubic_sites(L);
    uint8_t *b = (uint8_t *)malloc(n);
    uint32_t *lab = (uint32_t *)malloc(sizeof(uint32_t) * n);
    if (!b || !lab) { free(b); free(lab); return -1; }
    for (int64_t i = 0; i < count; ++i) {
        if (orc_cubic_sweep(L, J, T, q, seed, t0 + (uint32_t)i, spins, lab, b,
                            recs ? &recs[i] : NULL, NULL) != 0) {
            free(b);
            free(lab);
            return -1;
        }
    }
    free(b);
    free(lab);
    return 0;
}

/* Ensemble helper: independent hot-start chains (seeds seed0, seed0+1, ...),
 * `nsweeps` sweeps each; final e_sum and m_sum (Ising) or the count of
 * value 0 (Potts). */
int orc_cubic_chains(int32_t L, double J, uint32_t T, int32_t q, uint64_t seed0, int64_t nchains,
                     int32_t nsweeps, int64_t *e_out, int64_t *m_out)
{
    uint32_t n = cubic_sites(L);
    int8_t *sp = (int8_t *)malloc(n);
    if (!sp) return -1;
    for (int64_t c = 0; c < nchains; ++c) {
        uint64_t seed = seed0 + (uint64_t)c;
        orc_cubic_init(L, seed, q, 0, sp);
        if (orc_cubic_run(L, J, T, q, seed, 0u, nsweeps, sp, NULL) != 0) { free(sp); return -1; }
        orc_obs rec;
        orc_cubic_observe(L, J, q, 0, sp, NULL, &rec, NULL);
        int64_t z = 0;
        for (uint32_t s = 0; s < n; ++s) z += sp[s] == 0;
        e_out[c] = rec.e_sum;
        m_out[c] = q ? z : rec.m_sum;
    }
    free(sp);
    return 0;
}

/* ================================================================== */
/* O(4) phi^4 theory: the paper's second workload (Sec. 3), one        */
/* multicluster update of the Wolff embedding (Wolff's algorithm for   */
/* continuous spins, with every cluster reflected independently, as in */
/* Swendsen-Wang).  The paper fixes the bond probability (eq. 2) and   */
/* the reflection (eq. 3) but gives neither the self-coupling lambda   */
/* nor the radial update; the reading used is lambda -> infinity:      */
/* every field phi_x is a unit 4-vector and the weight of a            */
/* configuration is exp(2 kappa sum_<xy> phi_x . phi_y), which the     */
/* cluster update samples on its own.                                  */
/*                                                                     */
/* The lattice is a D-dimensional periodic hypercube of side L         */
/* (D = 4 in the paper; any D here, so that D = 1 can be checked       */
/* against the exact ring), site s = sum_mu x_mu L^mu, x_0 fastest;     */
/* each site owns the D links to s + mu.  Fields are 4 doubles per     */
/* site.  All floating point is IEEE-754 double, evaluated operation   */
/* by operation in the order written (this file is built as ISO C, so  */
/* no multiply-add is contracted):                                     */
/*   uniform of a word w     v = (w + 0.5) 2^-31 - 1, in (-1, 1)       */
/*   random direction of     attempt k = 0..63: Philox({k, t, 5, 0})    */
/*   sweep t                 gives v_0..v_3; accepted iff               */
/*                           rr = ((v0 v0 + v1 v1) + v2 v2) + v3 v3 < 1; */
/*                           r = v, unnormalised (n = r / |r|); after   */
/*                           64 rejections r = (1, 0, 0, 0)             */
/*   projection              p_x = ((f0 r0 + f1 r1) + f2 r2) + f3 r3    */
/*   link (x, mu) bonded iff a = ((p_x p_y) (4 kappa)) / rr > 0 and     */
/*                           u < 1 - E(a), u = w 2^-32, w = word mu of  */
/*                           Philox({x, t, 7, 0}), y = x + mu            */
/*   E(a) ~ exp(-a)          halve b = a while b > 1/8 (k times), then  */
/*                           q = 1; q = 1 - (q b) c_j for j = 13..1     */
/*                           (c_j = 1 / j rounded), then square q k     */
/*                           times (relative error below 1e-14)         */
/*   cluster reflected iff   bit root mod 128 of Philox({root >> 7, t,  */
/*                           6, 0}) is 1 (root = smallest site)         */
/*   reflection (eq. 3)      f = (2 p_x) / rr; phi^a -= f r^a            */
/*   hot start               site x, attempt k = 0..63: Philox({x, k,   */
/*                           8, 0}), v and vv as above, accepted iff    */
/*                           vv < 1: phi^a = v^a / sqrt(vv); after 64   */
/*                           rejections (1, 0, 0, 0); cold start        */
/*                           (1, 0, 0, 0) everywhere                    */
/*   measurement             e_fix = sum over links of                  */
/*                           rint(2^32 phi_x . phi_y), m_fix[a] = sum   */
/*                           of rint(2^32 phi_x^a), exact int64 sums    */
/* ================================================================== */
static uint32_t phi4_sites(int32_t D, int32_t L)
{
    uint32_t n = 1u;
    for (int32_t d = 0; d < D; ++d) n *= (uint32_t)L;
    return n;
}

/* s + mu-hat on the periodic D-dimensional lattice of side L */
static uint32_t phi4_step(uint32_t s, uint32_t L, int32_t mu)
{
    uint32_t stride = 1u;
    for (int32_t d = 0; d < mu; ++d) stride *= L;
    uint32_t x = (s / stride) % L;
    return x + 1u == L ? s - x * stride : s + stride;
}

static double phi4_uniform(uint32_t w)
{
    return ((double)w + 0.5) * 0x1p-31 - 1.0;
}

static double phi4_dot(const double a[4], const double b[4])
{
    return ((a[0] * b[0] + a[1] * b[1]) + a[2] * b[2]) + a[3] * b[3];
}

/* random direction of sweep t: r (unnormalised) and rr = r . r */
void orc_phi4_direction(uint64_t seed, uint32_t t, double r[4], double *rr)
{
    for (uint32_t k = 0; k < 64u; ++k) {
        uint32_t w[4];
        philox_seed(seed, k, t, 5u, w);
        double v[4];
        for (int a = 0; a < 4; ++a) v[a] = phi4_uniform(w[a]);
        double vv = phi4_dot(v, v);
        if (vv < 1.0) {
            for (int a = 0; a < 4; ++a) r[a] = v[a];
            *rr = vv;
            return;
        }
    }
    r[0] = 1.0; r[1] = r[2] = r[3] = 0.0;
    *rr = 1.0;
}

/* E(a), the evaluation of exp(-a) (a > 0) used by the bond test */
double orc_phi4_expm(double a)
{
    double b = a;
    int k = 0;
    while (b > 0.125) {
        b = b * 0.5;
        ++k;
    }
    double q = 1.0;
    for (int j = 13; j >= 1; --j) {
        double c = 1.0 / (double)j;
        q = 1.0 - (q * b) * c;
    }
    for (int i = 0; i < k; ++i) q = q * q;
    return q;
}

void orc_phi4_init(int32_t D, int32_t L, uint64_t seed, int32_t cold, double *phi)
{
    uint32_t n = phi4_sites(D, L);
    for (uint32_t s = 0; s < n; ++s) {
        double *f = phi + 4u * (size_t)s;
        f[0] = 1.0; f[1] = f[2] = f[3] = 0.0;
        if (cold) continue;
        for (uint32_t k = 0; k < 64u; ++k) {
            uint32_t w[4];
            philox_seed(seed, s, k, 8u, w);
            double v[4];
            for (int a = 0; a < 4; ++a) v[a] = phi4_uniform(w[a]);
            double vv = phi4_dot(v, v);
            if (vv < 1.0) {
                double len = sqrt(vv);
                for (int a = 0; a < 4; ++a) f[a] = v[a] / len;
                break;
            }
        }
    }
}

/* Bonds of sweep t (eq. 2): bonds[s] bit mu = link (s, s + mu) bonded. */
void orc_phi4_bonds(int32_t D, int32_t L, double kappa, uint64_t seed, uint32_t t,
                    const double *phi, uint8_t *bonds)
{
    uint32_t n = phi4_sites(D, L);
    double r[4], rr;
    orc_phi4_direction(seed, t, r, &rr);
    double k4 = 4.0 * kappa;
    for (uint32_t s = 0; s < n; ++s) {
        uint32_t w[4];
        philox_seed(seed, s, t, 7u, w);
        double px = phi4_dot(phi + 4u * (size_t)s, r);
        uint8_t b = 0;
        for (int32_t mu = 0; mu < D; ++mu) {
            uint32_t y = phi4_step(s, (uint32_t)L, mu);
            double py = phi4_dot(phi + 4u * (size_t)y, r);
            double a = ((px * py) * k4) / rr;
            if (a > 0.0) {
                double u = (double)w[mu] * 0x1p-32;
                if (u < 1.0 - orc_phi4_expm(a)) b |= (uint8_t)(1u << mu);
            }
        }
        bonds[s] = b;
    }
}

/* Clusters: connected components of the bonds, labelled by their smallest
 * site (the same union-find as the 2D oracle). */
void orc_phi4_label(int32_t D, int32_t L, const uint8_t *bonds, uint32_t *labels)
{
    uint32_t n = phi4_sites(D, L);
    for (uint32_t s = 0; s < n; ++s) labels[s] = s;
    for (uint32_t s = 0; s < n; ++s)
        for (int32_t mu = 0; mu < D; ++mu)
            if (bonds[s] & (1u << mu)) uf_union(labels, s, phi4_step(s, (uint32_t)L, mu));
    for (uint32_t s = 0; s < n; ++s) labels[s] = uf_find(labels, s);
}

/* Each cluster is reflected (eq. 3) with probability 1/2, independently. */
int32_t orc_phi4_flip(uint64_t seed, uint32_t t, uint32_t root)
{
    uint32_t r[4];
    philox_seed(seed, root >> 7, t, 6u, r);
    return (int32_t)((r[(root >> 5) & 3u] >> (root & 31u)) & 1u);
}

void orc_phi4_reflect(int32_t D, int32_t L, uint64_t seed, uint32_t t, const uint32_t *labels,
                      double *phi)
{
    uint32_t n = phi4_sites(D, L);
    double r[4], rr;
    orc_phi4_direction(seed, t, r, &rr);
    for (uint32_t s = 0; s < n; ++s) {
        if (!orc_phi4_flip(seed, t, labels[s])) continue;
        double *f = phi + 4u * (size_t)s;
        double c = (2.0 * phi4_dot(f, r)) / rr;
        for (int a = 0; a < 4; ++a) f[a] = f[a] - c * r[a];
    }
}

/* Measurement of a configuration and statistics of the clusters that made
 * it; the derived doubles are computed from the exact integer sums. */
void orc_phi4_observe(int32_t D, int32_t L, double kappa, uint64_t sweep, const double *phi,
                      const uint32_t *labels, orc_phi4_obs *rec)
{
    uint32_t n = phi4_sites(D, L);
    int64_t e = 0, m[4] = {0, 0, 0, 0};
    for (uint32_t s = 0; s < n; ++s) {
        const double *f = phi + 4u * (size_t)s;
        for (int32_t mu = 0; mu < D; ++mu) {
            const double *g = phi + 4u * (size_t)phi4_step(s, (uint32_t)L, mu);
            e += (int64_t)rint(phi4_dot(f, g) * 0x1p32);
        }
        for (int a = 0; a < 4; ++a) m[a] += (int64_t)rint(f[a] * 0x1p32);
    }
    memset(rec, 0, sizeof(*rec));
    rec->sweep = sweep;
    rec->e_fix = e;
    rec->action = -(2.0 * kappa) * ((double)e * 0x1p-32);
    double ms = 0.0;
    for (int a = 0; a < 4; ++a) {
        rec->m_fix[a] = m[a];
        double ma = (double)m[a] * 0x1p-32;
        ms = ms + ma * ma;
    }
    rec->m_abs = sqrt(ms);
    if (labels) {
        orc_obs c;
        memset(&c, 0, sizeof(c));
        cluster_stats(n, labels, &c, NULL);
        rec->n_clusters = c.n_clusters;
        rec->max_cluster = c.max_cluster;
        rec->sum_sq_sizes = c.sum_sq_sizes;
        memcpy(rec->hist_log2, c.hist_log2, sizeof(rec->hist_log2));
    }
}

/* One multicluster update t: direction, bonds, clusters, reflections, record. */
int orc_phi4_sweep(int32_t D, int32_t L, double kappa, uint64_t seed, uint32_t t, double *phi,
                   uint32_t *labels, uint8_t *bonds, orc_phi4_obs *rec)
{
    uint32_t n = phi4_sites(D, L);
    uint8_t *b = bonds ? bonds : (uint8_t *)malloc(n);
    uint32_t *lab = labels ? labels : (uint32_t *)malloc(sizeof(uint32_t) * n);
    if (!b || !lab) {
        if (!bonds) free(b);
        if (!labels) free(lab);
        return -1;
    }
    orc_phi4_bonds(D, L, kappa, seed, t, phi, b);
    orc_phi4_label(D, L, b, lab);
    orc_phi4_reflect(D, L, seed, t, lab, phi);
    if (rec) orc_phi4_observe(D, L, kappa, t, phi, lab, rec);
    if (!bonds) free(b);
    if (!labels) free(lab);
    return 0;
}

int orc_phi4_run(int32_t D, int32_t L, double kappa, uint64_t seed, uint32_t t0, int64_t count,
                 double *phi, orc_phi4_obs *recs)
{
    uint32_t n = phi4_sites(D, L);
    uint8_t *b = (uint8_t *)malloc(n);
    uint32_t *lab = (uint32_t *)malloc(sizeof(uint32_t) * n);
    if (!b || !lab) { free(b); free(lab); return -1; }
    for (int64_t i = 0; i < count; ++i)
        orc_phi4_sweep(D, L, kappa, seed, t0 + (uint32_t)i, phi, lab, b, recs ? &recs[i] : NULL);
    free(b);
    free(lab);
    return 0;
}
