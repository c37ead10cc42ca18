/*
 * sw_oracle.h -- declarations of the sequential CPU oracle (test
 * infrastructure only; see sw_oracle.c).  Private to oracle/: the HIP
 * library neither includes nor links it.
 */
#ifndef SW_ORACLE_H
#define SW_ORACLE_H

#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

/* One record per sweep: observables of the configuration left by the sweep
 * and statistics of the sweep's clusters. */
typedef struct {
    uint64_t sweep;
    int64_t e_sum;          /* sum over the 2N edges of s_i s_j */
    double energy;          /* -J * e_sum */
    int64_t m_sum;          /* sum of s_i */
    uint64_t n_clusters;
    uint64_t max_cluster;
    uint64_t sum_sq_sizes;
    uint64_t hist_log2[33]; /* clusters with size in [2^k, 2^(k+1)) */
} orc_obs;

void orc_philox4x32_10(const uint32_t ctr[4], const uint32_t key[2],
                       uint32_t out[4]);
uint32_t orc_threshold(double beta, double J);
void orc_init(int32_t L, uint64_t seed, int32_t cold, int8_t *spins);
void orc_bonds(int32_t L, uint32_t T, uint64_t seed, uint32_t t,
               const int8_t *spins, uint8_t *bonds);
void orc_label(int32_t L, const uint8_t *bonds, uint32_t *labels);
int32_t orc_flip_spin(uint64_t seed, uint32_t t, uint32_t root);
void orc_assign(int32_t L, uint64_t seed, uint32_t t, const uint32_t *labels,
                int8_t *spins);
void orc_observe(int32_t L, double J, uint64_t sweep, const int8_t *spins,
                 const uint32_t *labels, orc_obs *rec, uint64_t *dense);
int orc_sweep(int32_t L, double J, uint32_t T, uint64_t seed, uint32_t t,
              int8_t *spins, uint32_t *labels, uint8_t *bonds, orc_obs *rec,
              uint64_t *dense);
int orc_run(int32_t L, double J, uint32_t T, uint64_t seed, uint32_t t0,
            int64_t count, int8_t *spins, orc_obs *recs);
int orc_chains(int32_t L, double J, uint32_t T, uint64_t seed0, int64_t nchains,
               int32_t nsweeps, int64_t *e_out, int64_t *m_out);
int orc_one_step_codes(int32_t L, uint32_t T, uint64_t seed0, int64_t nseeds,
                       uint32_t t, const int8_t *start, uint64_t *codes);

/* q-state Potts model (spins 0..q-1, q <= 127): see sw_oracle.c. */
uint32_t orc_potts_threshold(double beta, double J);
void orc_potts_init(int32_t L, uint64_t seed, int32_t q, int32_t cold, int8_t *spins);
int32_t orc_potts_spin(uint64_t seed, uint32_t t, uint32_t root, int32_t q);
void orc_potts_assign(int32_t L, uint64_t seed, uint32_t t, int32_t q, const uint32_t *labels,
                      int8_t *spins);
void orc_potts_observe(int32_t L, double J, int32_t q, uint64_t sweep, const int8_t *spins,
                       const uint32_t *labels, orc_obs *rec, uint64_t *dense);
int orc_potts_sweep(int32_t L, double J, uint32_t T, int32_t q, uint64_t seed, uint32_t t,
                    int8_t *spins, uint32_t *labels, orc_obs *rec);
int orc_potts_run(int32_t L, double J, uint32_t T, int32_t q, uint64_t seed, uint32_t t0,
                  int64_t count, int8_t *spins, orc_obs *recs);
int orc_potts_chains(int32_t L, double J, uint32_t T, int32_t q, uint64_t seed0, int64_t nchains,
                     int32_t nsweeps, int64_t *e_out, int64_t *n0_out);

/* simple cubic lattice (L x L x L); q = 0 Ising, 2..8 Potts */
void orc_cubic_init(int32_t L, uint64_t seed, int32_t q, int32_t cold, int8_t *spins);
void orc_cubic_bonds(int32_t L, uint32_t T, uint64_t seed, uint32_t t,
                     const int8_t *spins, uint8_t *bonds);
void orc_cubic_label(int32_t L, const uint8_t *bonds, uint32_t *labels);
void orc_cubic_observe(int32_t L, double J, int32_t q, uint64_t sweep, const int8_t *spins,
                       const uint32_t *labels, orc_obs *rec, uint64_t *dense);
int orc_cubic_sweep(int32_t L, double J, uint32_t T, int32_t q, uint64_t seed, uint32_t t,
                    int8_t *spins, uint32_t *labels, uint8_t *bonds, orc_obs *rec, uint64_t *dense);
int orc_cubic_run(int32_t L, double J, uint32_t T, int32_t q, uint64_t seed, uint32_t t0,
                  int64_t count, int8_t *spins, orc_obs *recs);
int orc_cubic_chains(int32_t L, double J, uint32_t T, int32_t q, uint64_t seed0, int64_t nchains,
                     int32_t nsweeps, int64_t *e_out, int64_t *m_out);

/* O(4) model with unit fields (phi^4 at lambda = infinity), D-dimensional
 * periodic hypercube of side L, multicluster Wolff-embedding update. */
typedef struct {
    uint64_t sweep;
    int64_t e_fix;          /* sum over the D N links of rint(2^32 phi_x . phi_y) */
    double action;          /* -2 kappa e_fix 2^-32 (hopping part of the action)  */
    int64_t m_fix[4];       /* sum over sites of rint(2^32 phi_x^a)               */
    double m_abs;           /* |M| from m_fix                                     */
    uint64_t n_clusters;
    uint64_t max_cluster;
    uint64_t sum_sq_sizes;
    uint64_t hist_log2[33];
} orc_phi4_obs;

void orc_phi4_direction(uint64_t seed, uint32_t t, double r[4], double *rr);
double orc_phi4_expm(double a);
void orc_phi4_init(int32_t D, int32_t L, uint64_t seed, int32_t cold, double *phi);
void orc_phi4_bonds(int32_t D, int32_t L, double kappa, uint64_t seed, uint32_t t,
                    const double *phi, uint8_t *bonds);
void orc_phi4_label(int32_t D, int32_t L, const uint8_t *bonds, uint32_t *labels);
int32_t orc_phi4_flip(uint64_t seed, uint32_t t, uint32_t root);
void orc_phi4_reflect(int32_t D, int32_t L, uint64_t seed, uint32_t t, const uint32_t *labels,
                      double *phi);
void orc_phi4_observe(int32_t D, int32_t L, double kappa, uint64_t sweep, const double *phi,
                      const uint32_t *labels, orc_phi4_obs *rec);
int orc_phi4_sweep(int32_t D, int32_t L, double kappa, uint64_t seed, uint32_t t, double *phi,
                   uint32_t *labels, uint8_t *bonds, orc_phi4_obs *rec);
int orc_phi4_run(int32_t D, int32_t L, double kappa, uint64_t seed, uint32_t t0, int64_t count,
                 double *phi, orc_phi4_obs *recs);

#ifdef __cplusplus
}
#endif


#endif
