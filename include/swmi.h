/*
 * swmi.h -- C ABI of libswmi.so: Swendsen-Wang dynamics of the 2D Ising
 * model on an L x L periodic square lattice, run on one AMD Instinct MI355X
 * (gfx950) with hand-written HIP kernels.
 *
 * The method is the one of Protzman & Giedt, "GPU Acceleration of Swendson-
 * Wang Dynamics" (Sec. 2): one sweep forms random bonds between equal
 * neighbouring spins (Sec. 2.1), labels the connected clusters of the bond
 * graph (Sec. 2.3), gives every cluster a fresh spin, up or down with
 * probability 1/2 (Sec. 2.4), and measures the new configuration (Sec. 2.5).
 *
 * Conventions (shared with the test oracle only by definition, not by code):
 *   site s = y*L + x (x fastest), periodic; E(s) = y*L + (x+1 mod L),
 *   N(s) = ((y+1) mod L)*L + x; each site owns its E and N edges.
 *   Bond threshold T = floor((1 - exp(-2 beta J)) * 2^32), computed once in
 *   FP64; an edge with equal end spins is bonded iff its uniform 32-bit word
 *   is below T, so P(bond) = T / 2^32.
 *   Randomness is Philox4x32-10 keyed by the 64-bit seed:
 *     edge (s, d), d = 0 (E) / 1 (N), sweep t: word 2*(s&1)+d of the output
 *       for counter {s>>1, t, 0, 0};
 *     new spin of the cluster whose smallest site is r, sweep t: bit r mod 128
 *       of the 128-bit output for counter {r>>7, t, 1, 0} (1 -> -1, 0 -> +1);
 *     hot start: bit 0 of word 0 for counter {s, 0, 2, 0} (1 -> -1).
 *   Cluster labels are the smallest site index of the cluster.
 *   Sweeps are numbered t = 0, 1, ... from create / reset; record t holds the
 *   statistics of sweep t's clusters and the observables of the configuration
 *   that sweep t leaves.
 *
 * Error behaviour: every int-returning call returns SW_OK (0) or a negative
 * SW_E* code, and sw_last_error() then describes the failure (thread-local,
 * valid until the next failing call on the same thread).  No C++ exception
 * crosses the ABI.  A sim is not thread-safe; distinct sims on distinct
 * streams may be driven from distinct threads.
 *
 * Ownership: an sw_sim owns its device buffers, unless it was created with a
 * caller workspace (sw_create_in / sw_create_ex), which the caller keeps
 * alive until sw_destroy.  Host pointers passed in are only read or written
 * during the call.  All device work runs on the sim's stream, in order.
 */
#ifndef SWMI_H
#define SWMI_H

#include <stddef.h>
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

#define SW_OK 0
#define SW_EINVAL (-1)  /* an argument is out of its documented domain      */
#define SW_ERANGE (-2)  /* an index/length is outside the available range    */
#define SW_ENOMEM (-3)  /* device or host allocation failed / workspace small */
#define SW_EHIP (-4)    /* a HIP runtime call failed                          */
#define SW_ESTATE (-5)  /* the call is not valid in the sim's current state   */

#define SW_INIT_HOT 0   /* i.i.d. +-1 spins drawn from the seed (Fig. 1)     */
#define SW_INIT_COLD 1  /* all spins +1                                       */

#define SW_FLAG_LABELS 1u      /* keep the canonical labels of the last sweep */
#define SW_FLAG_DENSE_HIST 2u  /* keep the exact cluster-size histogram       */
#define SW_FLAG_LABEL_EQUIV 4u /* label clusters the paper's way (see below)  */

typedef struct sw_sim sw_sim;

/* One record per sweep (Sec. 2.5: magnetisation and energy of every new
 * configuration, plus the statistics of the sweep's clusters).  All sums are
 * exact integers; energy = -J * e_sum. */
typedef struct {
    uint64_t sweep;          /* sweep index t                                  */
    int64_t e_sum;           /* sum over the 2N torus edges of s_i s_j         */
    double energy;           /* H = -J sum_<ij> s_i s_j                         */
    int64_t m_sum;           /* sum of s_i  (M = m_sum / N)                     */
    uint64_t n_clusters;     /* clusters of sweep t                             */
    uint64_t max_cluster;    /* largest cluster size                           */
    uint64_t sum_sq_sizes;   /* sum over clusters of size^2                    */
    uint64_t hist_log2[33];  /* clusters with size in [2^k, 2^(k+1))           */
} sw_obs;

/* Creation parameters.  L: lattice side, a multiple of 32 in [32, 32768]
 * (simple cubic lattice: a multiple of 16 in [16, 1616]).
 * beta >= 0 and J > 0, both finite.  init: SW_INIT_HOT or SW_INIT_COLD.
 * tile: 0 (automatic: 64 when L is a multiple of 64, else 32), 32 or 64 --
 * the side of the square tile one workgroup labels in LDS; results do not
 * depend on it.  flags: SW_FLAG_*.  ring: number of per-sweep records kept
 * on the device (0 = 4096). */
typedef struct {
    int32_t L;
    int32_t init;
    int32_t tile;
    uint32_t flags;
    double beta;
    double J;
    uint64_t seed;
    int64_t ring;
    int32_t q;     /* 0: Ising (spins +-1); 2..8: q-state Potts (see below) */
    int32_t dims;  /* 0 or 2: L x L square lattice; 3: L x L x L simple cubic (see below) */
} sw_config;

/* Fills *cfg with the given lattice and model and default options
 * (hot start, automatic tile, no flags, default ring).  SW_EINVAL if cfg is
 * NULL. */
int sw_config_init(sw_config *cfg, int32_t L, double beta, double J, uint64_t seed);

/* Device bytes a sim needs for the default options / for *cfg; 0 when the
 * parameters are invalid.  Use it to size a caller workspace. */
size_t sw_workspace_bytes(int32_t L);
size_t sw_workspace_bytes_ex(const sw_config *cfg);

/* Creates a sim of the L x L periodic lattice with coupling J at inverse
 * temperature beta, in the random initial configuration of Sec. 2 (Fig. 1:
 * i.i.d. spins, up or down with probability 1/2, drawn from `seed`), t = 0.
 * The bond probability of Sec. 2.1 is fixed here, once, as the threshold T.
 * The sim allocates its own device memory and its own stream (default
 * priority).  *out receives the handle; SW_EINVAL for L, beta or J outside
 * their domain (see sw_config), SW_ENOMEM / SW_EHIP if the device refuses. */
int sw_create(int32_t L, double beta, double J, uint64_t seed, sw_sim **out);

/* As sw_create, but carves every device buffer out of the caller's
 * workspace `dev_workspace` (device pointer, >= sw_workspace_bytes(L) bytes,
 * 256-byte aligned) and enqueues all work on `hip_stream` (a hipStream_t;
 * NULL selects the null stream).  SW_ENOMEM if ws_bytes is too small. */
int sw_create_in(int32_t L, double beta, double J, uint64_t seed,
                 void *dev_workspace, size_t ws_bytes, void *hip_stream,
                 sw_sim **out);

/* General form: dev_workspace may be NULL (the library allocates) and
 * hip_stream may be NULL with dev_workspace NULL (the library creates a
 * stream). */
int sw_create_ex(const sw_config *cfg, void *dev_workspace, size_t ws_bytes,
                 void *hip_stream, sw_sim **out);

/* Re-initialises the spins (SW_INIT_HOT / SW_INIT_COLD) and sets t = 0;
 * earlier records become unavailable. */
int sw_reset(sw_sim *sim, int init_mode);

/* Enqueues n >= 0 sweeps on the sim's stream and returns without waiting
 * (Sec. 2: bonds, clusters, new spins and the record of each sweep). */
int sw_sweep(sw_sim *sim, int64_t n);

/* Measurement aid: runs n >= 1 sweeps exactly as sw_sweep does (same
 * kernels, same results, same records), but launches the kernels one by one
 * with HIP events between them on the sim's stream and waits after each
 * sweep.  ms[0..4] receive the average duration in milliseconds of the five
 * stages of a sweep -- 0: bonds + tile-local clusters (Sec. 2.1, 2.3),
 * 1: cross-tile unions, 2: flattening and cluster sizes, 3: spins of
 * cross-tile clusters (Sec. 2.4) and statistics, 4: the record (Sec. 2.5;
 * on lattices of at most 64 groups of 16 tiles stage 3 writes the record
 * and stage 4 launches nothing, so ms[4] is the events' own cost) -- and
 * ms[5] the closing pass that writes final spins and measures them.
 * nk (the length of ms) must be >= 6; extra entries are zeroed. */
int sw_profile(sw_sim *sim, int64_t n, double *ms, int32_t nk);

/* Waits for all enqueued work of the sim. */
int sw_sync(sw_sim *sim);

/* Copies the record of the last completed sweep into *out (waits for the
 * stream).  SW_ESTATE if no sweep has run since create / reset / set_spins. */
int sw_observables(sw_sim *sim, sw_obs *out);

/* Per-sweep series of the measurements of Sec. 2.5 (magnetisation and
 * energy of every new configuration, with the statistics of the clusters of
 * Sec. 2.3 that produced it): copies records of sweeps first ..
 * first+count-1 into out[0..count-1] (host memory, caller-owned; waits).
 * SW_ERANGE unless all of them ran since the last create / reset /
 * set_spins and are still held in the ring; SW_EINVAL for a NULL out. */
int sw_series(sw_sim *sim, int64_t first, int64_t count, sw_obs *out);

/* Exact cluster-size histogram of the last sweep's clusters (the connected
 * components of Sec. 2.3): counts[s] = number of clusters of size s,
 * s = 0..N, into host memory of len >= N+1 words.  Needs
 * SW_FLAG_DENSE_HIST (SW_ESTATE otherwise, or before the first sweep);
 * SW_ERANGE if len is too small. */
int sw_cluster_hist(sw_sim *sim, uint64_t *counts, int64_t len);

/* Current spins (int8 +-1, site order s = y*L + x) to host memory;
 * n must equal N = L*L. */
int sw_get_spins(sw_sim *sim, int8_t *host, int64_t n);

/* Replaces the spins (host int8, each +1 or -1, n == N, site order
 * s = y*L + x) and makes next_sweep the index of the next sweep.  A sweep
 * (Sec. 2) depends only on the current configuration and on randomness
 * keyed by (seed, sweep, site), so this resumes a chain from a checkpoint
 * and lets one sweep be compared against a reference.  Records before
 * next_sweep become unavailable.  SW_EINVAL for a value other than +-1
 * (Potts: outside 0..q-1), SW_ERANGE for a wrong n. */
int sw_set_spins(sw_sim *sim, const int8_t *host, int64_t n, uint64_t next_sweep);

/* Labels of the last sweep's clusters (Sec. 2.3: every site ends with the
 * lowest label of its cluster, labels starting as site indices, i.e. the
 * smallest site index of the cluster) to host memory (uint32, n == N, site
 * order).  Needs SW_FLAG_LABELS and a completed sweep (SW_ESTATE
 * otherwise); SW_ERANGE for a wrong n. */
int sw_get_labels(sw_sim *sim, uint32_t *host, int64_t n);

/* Sims created with SW_FLAG_LABEL_EQUIV form clusters as the paper does
 * (Sec. 2.3, after Kalentev et al.): every site starts with its own index
 * as label; a scan pass points the entry of each site's label at the
 * smallest label among its bonded neighbours, an analysis pass makes every
 * site take the label at the end of its chain of references, and the two
 * repeat until a scan changes nothing -- all passes inside one cooperative
 * kernel that polls a device-side flag (the paper used a dynamic-
 * parallelism kernel for this, Sec. 5).  Labels, spins and records are
 * identical to the default path (the tile pipeline); it is slower and
 * exists to compare the two designs.  Labels are always kept (no need for
 * SW_FLAG_LABELS); the tile option is ignored.
 * sw_label_passes returns the number of scan/analysis passes of the last
 * sweep (waits for the stream), -2 if that sweep stopped at the pass limit
 * (65,536) without converging, -1 for a sim of the default path. */
int32_t sw_label_passes(sw_sim *sim);

/* q-state Potts model (sw_config.q = 2..8; on the tile path -- 64-wide tiles
 * for q <= 4, 32-wide tiles above (tile 64 with q > 4 is SW_EINVAL) -- or on
 * the label-equivalence path with SW_FLAG_LABEL_EQUIV; all give the same bits):
 * spins are 0..q-1 (int8), H = -J sum_<ij> delta(s_i, s_j).  A sweep bonds equal
 * neighbours with p = 1 - exp(-beta J) (T = floor(p 2^32), the same edge
 * words as the Ising model), forms clusters the same way, and gives every
 * cluster the value floor(w q / 2^32) of word r mod 4 of the Philox output
 * for counter {r >> 2, t, 3, 0}, r its smallest site.  Hot start: value of
 * word 0 for counter {s, 0, 2, 0}; cold start: all 0.  Records: e_sum =
 * number of the 2N edges with equal ends (energy = -J e_sum), m_sum =
 * population of the most populated value; cluster statistics as for Ising.
 * sw_set_spins takes values 0..q-1. */

/* Simple cubic lattice (sw_config.dims = 3; L a multiple of 16 in
 * [16, 1616], so that N = L^3 < 2^32; clusters are formed in 16^3 bricks and
 * joined across brick faces, or with SW_FLAG_LABEL_EQUIV by the paper's
 * label equivalence; both give the same bits; sw_tile gives 16 for the
 * bricks and 0 for label equivalence): the same sweep on
 * the L x L x L periodic lattice, for the Ising model (q = 0) and the Potts
 * model (q = 2..8).  Site s = (z L + y) L + x, x fastest; each site owns the
 * edges to its +x, +y and +z neighbours (3N edges), and the word of edge
 * (s, d) is word d (0: +x, 1: +y, 2: +z) of the Philox output for counter
 * {s, t, 4, 0}.  Thresholds, start states, new spins and records follow the
 * square-lattice rules, with the sums taken over the 3N edges.  Spin and
 * label buffers hold N = L^3 entries (sw_sites). */

/* Number of lattice sites N (L^2, or L^3 for the simple cubic lattice);
 * -1 for NULL. */
int64_t sw_sites(const sw_sim *sim);

/* The bond threshold T of this sim (so callers can check it). */
uint32_t sw_threshold(const sw_sim *sim);

/* Index of the next sweep t. */
int64_t sw_next_sweep(const sw_sim *sim);

/* Lattice side and tile side actually used. */
int32_t sw_lattice(const sw_sim *sim);
int32_t sw_tile(const sw_sim *sim);

/* Destroys the sim (waits for its stream first); NULL is a no-op. */
void sw_destroy(sw_sim *sim);

/* Message describing the last failure on this thread ("" if none). */
const char *sw_last_error(void);

/* ------------------------------------------------------------- batches
 * A batch advances n independent lattices (replicas) together: every kernel
 * of a sweep (Sec. 2) runs once over all replicas of a launch group (the
 * replicas with one tile width and model), so a sweep of the whole batch
 * costs a handful of kernel launches (replayed from one captured graph)
 * instead of five or six per replica.  The cross-tile merge of Sec. 2.3 runs
 * either globally (four launches over all such replicas, the record folded
 * into the last) or, for a replica of at
 * most 16 tiles, entirely in one workgroup's LDS (one launch for all such
 * replicas: SW_MERGE_LDS).  Replica r has its own L[r], beta[r], J[r],
 * seed[r] and its own records; its spins, clusters and records are bit for
 * bit those of a plain sim created with the same parameters and swept the
 * same number of times, whatever its tile width and merge.  All replicas
 * share the sweep counter t.  Limits: 1 <= n <= 4095; every L[r] as for
 * sw_create; no labels or dense histogram. */
typedef struct sw_batch sw_batch;

#define SW_MERGE_AUTO 0   /* LDS merge when the replica has at most 16 tiles */
#define SW_MERGE_LDS 1    /* the whole merge in one workgroup (<= 16 tiles)  */
#define SW_MERGE_GLOBAL 2 /* the global merge                                */

/* Device bytes of a batch with these lattice sides, `ring` records per
 * replica (0 = 1024) and tile side (0 = automatic, 32, 64); 0 when the
 * arguments are invalid. */
size_t sw_batch_workspace_bytes(int32_t n, const int32_t *L, int64_t ring, int32_t tile);

/* Creates a batch of n replicas, L/beta/J/seed being arrays of length n
 * (host memory, read during the call), all started with `init`
 * (SW_INIT_HOT / SW_INIT_COLD), t = 0.  tile: the side of the tiles every
 * replica is labelled in -- 0 (each replica: 64 when its L is a multiple of
 * 64, else 32), 32 or 64 (results do not depend on it); merge automatic.  dev_workspace: NULL (the library
 * allocates) or a 256-byte-aligned device buffer of >= ws_bytes =
 * sw_batch_workspace_bytes(...) bytes that the caller keeps alive until
 * sw_batch_destroy.  hip_stream: the stream for all of the batch's work
 * (NULL with dev_workspace NULL: the library creates one).  SW_EINVAL for a
 * bad replica (the message names it), SW_ENOMEM for a small workspace. */
int sw_batch_create(int32_t n, const int32_t *L, const double *beta, const double *J,
                    const uint64_t *seed, int32_t init, int64_t ring, int32_t tile,
                    void *dev_workspace, size_t ws_bytes, void *hip_stream, sw_batch **out);

/* Batches of q-state Potts replicas (the model of sw_config.q): as
 * sw_batch_workspace_bytes / sw_batch_create, with q[0..n-1] the q (2..8)
 * of every replica.  tile 0 selects, per replica, 64-wide tiles when its L
 * is a multiple of 64 and its q is at most 4, else 32-wide; tile 64 with a
 * q above 4 is SW_EINVAL.  Every replica's bits are those of a plain Potts
 * sim with the same parameters. */
size_t sw_batch_workspace_bytes_potts(int32_t n, const int32_t *L, const int32_t *q, int64_t ring,
                                      int32_t tile);
int sw_batch_create_potts(int32_t n, const int32_t *L, const double *beta, const double *J,
                          const uint64_t *seed, const int32_t *q, int32_t init, int64_t ring, int32_t tile,
                          void *dev_workspace, size_t ws_bytes, void *hip_stream, sw_batch **out);

/* General form: q (NULL: all Ising) gives every replica's model (0 Ising,
 * 2..8 q-state Potts); tiles (NULL: automatic) every replica's tile width
 * (0 automatic, 32, 64; as sw_config.tile); merge (NULL: automatic) every
 * replica's merge (SW_MERGE_AUTO, SW_MERGE_LDS -- SW_EINVAL for a replica
 * of more than 16 tiles -- or SW_MERGE_GLOBAL).  Replicas of different tile
 * widths or models run in separate launch groups of the same sweep.  These
 * choices change no result, only speed; the binding's autotuner picks them
 * per lattice side. */
size_t sw_batch_workspace_bytes_ex(int32_t n, const int32_t *L, const int32_t *q, const int32_t *tiles,
                                   const int32_t *merge, int64_t ring);
int sw_batch_create_ex(int32_t n, const int32_t *L, const double *beta, const double *J, const uint64_t *seed,
                       const int32_t *q, const int32_t *tiles, const int32_t *merge, int32_t init, int64_t ring,
                       void *dev_workspace, size_t ws_bytes, void *hip_stream, sw_batch **out);

/* Re-initialises every replica (SW_INIT_HOT / SW_INIT_COLD) and sets t = 0. */
int sw_batch_reset(sw_batch *batch, int32_t init_mode);

/* Enqueues n >= 0 sweeps of every replica and returns without waiting. */
int sw_batch_sweep(sw_batch *batch, int64_t n);

/* Waits for all enqueued work of the batch. */
int sw_batch_sync(sw_batch *batch);

/* Records of the last completed sweep, one per replica, into out[0..n-1]
 * (waits).  SW_ESTATE if no sweep has run since create / reset. */
int sw_batch_observables(sw_batch *batch, sw_obs *out);

/* Records first .. first+count-1 of replica r (as sw_series). */
int sw_batch_series(sw_batch *batch, int32_t r, int64_t first, int64_t count, sw_obs *out);

/* Current spins of replica r (n == L[r]^2), as sw_get_spins. */
int sw_batch_get_spins(sw_batch *batch, int32_t r, int8_t *host, int64_t n);

/* Number of replicas; index of the next sweep; side, bond threshold, tile
 * width and merge (SW_MERGE_LDS / SW_MERGE_GLOBAL) of replica r (0 for a bad
 * index); the tile width every replica uses (0 if they differ). */
int32_t sw_batch_size(const sw_batch *batch);
int64_t sw_batch_next_sweep(const sw_batch *batch);
int32_t sw_batch_lattice(const sw_batch *batch, int32_t r);
uint32_t sw_batch_threshold(const sw_batch *batch, int32_t r);
int32_t sw_batch_replica_tile(const sw_batch *batch, int32_t r);
int32_t sw_batch_replica_merge(const sw_batch *batch, int32_t r);
int32_t sw_batch_tile(const sw_batch *batch);

/* Destroys the batch (waits for its stream first); NULL is a no-op. */
void sw_batch_destroy(sw_batch *batch);

/* ------------------------------------------------------------- serving
 * A server runs independent jobs -- (L, beta, J, seed, start, number of
 * sweeps) -- on one GPU.  Jobs wait in a FIFO queue until their buffers fit
 * in the server's device memory pool and a slot is free; every step then
 * advances all active jobs together with the batched kernels (continuous
 * batching: a job leaves as soon as it has run its sweeps, and queued jobs
 * take its memory).  A job's spins and records are bit for bit those of a
 * plain sim with the same parameters run alone, whatever else shares the
 * GPU.  A finished job's records (all of its sweeps) and final spins stay on
 * the device until sw_server_release. */
typedef struct sw_server sw_server;

#define SW_JOB_QUEUED 0  /* waiting for memory or a slot                     */
#define SW_JOB_ACTIVE 1  /* sweeping                                         */
#define SW_JOB_DONE 2    /* all sweeps run; results readable until released */

typedef struct {
    int64_t id;
    int32_t state;         /* SW_JOB_*                                         */
    int32_t L;
    int64_t sweeps_done;
    int64_t sweeps_total;
    uint64_t bytes;        /* device bytes the job holds while admitted       */
} sw_job_info;

/* Device bytes a job of side L running `sweeps` sweeps needs (0 if invalid);
 * the _potts form for a q-state Potts job (q = 2..8). */
size_t sw_server_job_bytes(int32_t L, int64_t sweeps);
size_t sw_server_job_bytes_potts(int32_t L, int32_t q, int64_t sweeps);

/* Creates a server with a device memory pool of pool_bytes: `pool` is a
 * 256-byte-aligned device buffer the caller keeps alive until
 * sw_server_destroy, or NULL (the library allocates it).  max_jobs (1..4095)
 * bounds the active jobs.  hip_stream: the stream for all work, or NULL
 * (the library creates one). */
int sw_server_create(void *pool, size_t pool_bytes, int32_t max_jobs, void *hip_stream, sw_server **out);

/* Queues a job; *job_id receives its id.  L, beta, J, init as for
 * sw_create_ex; sweeps >= 1.  SW_ENOMEM if the job can never fit the pool. */
int sw_server_submit(sw_server *server, int32_t L, double beta, double J, uint64_t seed,
                     int32_t init, int64_t sweeps, int64_t *job_id);

/* Queues a q-state Potts job (q = 2..8, the model of sw_config.q); Ising and
 * Potts jobs share the pool and the steps, and each job's bits are those of
 * a plain sim with the same parameters. */
int sw_server_submit_potts(sw_server *server, int32_t L, double beta, double J, uint64_t seed, int32_t q,
                           int32_t init, int64_t sweeps, int64_t *job_id);

/* Admits queued jobs that fit, then runs up to n sweeps of the active set
 * (fewer if it empties), retiring jobs as they finish and admitting queued
 * ones into the memory they free.  Waits for the GPU before returning.
 * done_ids[0..cap-1] receive the ids of the jobs that finished during the
 * call; *ndone their number (which may exceed cap). */
int sw_server_step(sw_server *server, int64_t n, int64_t *done_ids, int32_t cap, int32_t *ndone);

/* State and progress of a job (SW_ERANGE for an unknown id). */
int sw_server_job_info(sw_server *server, int64_t job_id, sw_job_info *info);

/* Records first .. first+count-1 of an admitted job (Sec. 2.5 measurements,
 * as sw_series).  A finished job has records 0 .. sweeps_total-1.  An active
 * job that has run `done` sweeps has records 0 .. done-2: the energy and
 * magnetisation of record done-1 are measured by the job's next sweep, so
 * asking for it gives SW_ERANGE until then. */
int sw_server_job_series(sw_server *server, int64_t job_id, int64_t first, int64_t count, sw_obs *out);

/* Final spins of a finished job (n == L*L); SW_ESTATE before it is done. */
int sw_server_job_spins(sw_server *server, int64_t job_id, int8_t *host, int64_t n);

/* Forgets a finished or still queued job and frees its memory; SW_ESTATE for
 * an active job. */
int sw_server_release(sw_server *server, int64_t job_id);

/* Queued and active job counts, pool bytes in use, and the site updates run
 * since creation (any pointer may be NULL). */
int sw_server_status(sw_server *server, int32_t *queued, int32_t *active, size_t *bytes_used,
                     uint64_t *site_updates);

/* Destroys the server and every job (waits for the stream first). */
void sw_server_destroy(sw_server *server);

/* ------------------------------------------------------------- phi^4
 * The paper's second workload (Sec. 3): the O(4)-symmetric phi^4 theory on
 * the periodic L^4 lattice, one multicluster update of the Wolff embedding
 * per sweep.  The paper gives the bond probability (eq. 2) and the cluster
 * reflection (eq. 3) but neither the self-coupling lambda nor the radial
 * update; here the fields are unit 4-vectors (the lambda -> infinity
 * limit), whose weight exp(2 kappa sum_<xy> phi_x . phi_y) the cluster
 * update samples on its own.
 *
 * Conventions: site x = ((x3 L + x2) L + x1) L + x0, periodic; each site owns
 * the links to x + mu-hat, mu = 0..3 (4N links).  Fields are 4 doubles per
 * site (x-major, component fastest).  Sweep t:
 *   direction   the first of up to 64 candidates v = ((w_a + 0.5) 2^-31 - 1),
 *               w = Philox({k, t, 5, 0}), k = 0, 1, ..., with
 *               rr = ((v0 v0 + v1 v1) + v2 v2) + v3 v3 < 1; r = v (not
 *               normalised); (1, 0, 0, 0) if none
 *   projection  p_x = ((phi0 r0 + phi1 r1) + phi2 r2) + phi3 r3
 *   bond (eq. 2) link (x, mu), y = x + mu-hat: a = ((p_x p_y) (4 kappa)) / rr;
 *               bonded iff a > 0 and w 2^-32 < 1 - E(a), w = word mu of
 *               Philox({x, t, 7, 0}); E(a) evaluates exp(-a): halve a to
 *               b <= 1/8 (k times), q = 1, q = 1 - (q b) (1/j) for j = 13..1,
 *               then square q k times
 *   clusters    connected components, labelled by their smallest site
 *   reflection  (eq. 3) a cluster whose smallest site r has bit r mod 128 of
 *               Philox({r >> 7, t, 6, 0}) set: phi -= ((2 p_x) / rr) r
 *   hot start   site x: first of up to 64 candidates from Philox({x, k, 8, 0})
 *               inside the unit ball, divided by sqrt(vv); cold: (1, 0, 0, 0)
 * All double arithmetic is IEEE-754, one correctly rounded operation at a
 * time in the order written, so results are reproducible bit for bit.
 * Records: exact int64 sums in units of 2^-32 (each term rounded to the
 * nearest integer multiple first), so they do not depend on summation order. */
typedef struct sw_phi4 sw_phi4;

typedef struct {
    uint64_t sweep;          /* sweep index t                                   */
    int64_t e_fix;           /* sum over the 4N links of rint(2^32 phi_x . phi_y) */
    double action;           /* -2 kappa e_fix 2^-32: the hopping action        */
    int64_t m_fix[4];        /* sum over sites of rint(2^32 phi_x^a)            */
    double m_abs;            /* |M| = sqrt(sum_a (m_fix[a] 2^-32)^2)            */
    uint64_t n_clusters;     /* clusters of sweep t                             */
    uint64_t max_cluster;
    uint64_t sum_sq_sizes;
    uint64_t hist_log2[33];  /* clusters with size in [2^k, 2^(k+1))            */
} sw_phi4_obs;

/* Device bytes of a phi^4 sim of side L with `ring` records (0 = 4096); 0
 * for L outside [2, 64] or a bad ring. */
size_t sw_phi4_workspace_bytes(int32_t L, int64_t ring);

/* Creates a phi^4 sim of side L (2..64, N = L^4 sites), hopping parameter
 * kappa in [0, 4] (the paper's runs use 0.304), seed, init (SW_INIT_HOT:
 * fields uniform on the unit sphere; SW_INIT_COLD: (1, 0, 0, 0)), t = 0.
 * dev_workspace: NULL (the library allocates) or a 256-byte-aligned device
 * buffer of >= sw_phi4_workspace_bytes(L, ring) bytes kept alive by the
 * caller; hip_stream: the stream for all work (NULL with dev_workspace NULL:
 * the library creates one).  SW_EINVAL / SW_ENOMEM / SW_EHIP as for
 * sw_create_ex. */
int sw_phi4_create(int32_t L, double kappa, uint64_t seed, int32_t init, int64_t ring, void *dev_workspace,
                   size_t ws_bytes, void *hip_stream, sw_phi4 **out);

/* Re-initialises the fields and sets t = 0. */
int sw_phi4_reset(sw_phi4 *sim, int32_t init);

/* Enqueues n >= 0 multicluster updates (Sec. 3) and returns without waiting. */
int sw_phi4_sweep(sw_phi4 *sim, int64_t n);

/* Waits for all enqueued work. */
int sw_phi4_sync(sw_phi4 *sim);

/* Measurement aid: n >= 1 updates exactly as sw_phi4_sweep, launched kernel
 * by kernel with HIP events on the sim's stream; ms[0..4] receive the mean
 * milliseconds of the five kernels (projections, bonds and unions,
 * flattening and sizes, reflections, measurement and record); nk >= 5. */
int sw_phi4_profile(sw_phi4 *sim, int64_t n, double *ms, int32_t nk);

/* Records first .. first+count-1 (Sec. 3 updates; measured after each) into
 * host memory (waits); SW_ERANGE unless they ran since the last create /
 * reset / set_field and are still held in the ring. */
int sw_phi4_series(sw_phi4 *sim, int64_t first, int64_t count, sw_phi4_obs *out);

/* Fields to host memory, n == 4 L^4 doubles. */
int sw_phi4_get_field(sw_phi4 *sim, double *host, int64_t n);

/* Replaces the fields (n == 4 L^4 finite doubles; the model's fields are
 * unit vectors, which is not enforced) and makes next_sweep the index of the
 * next sweep: an update depends only on the fields and on randomness keyed
 * by (seed, sweep, site), so this resumes a chain or checks one update. */
int sw_phi4_set_field(sw_phi4 *sim, const double *host, int64_t n, uint64_t next_sweep);

/* Labels (smallest site of the cluster) of the last update's clusters,
 * n == L^4; SW_ESTATE before the first update. */
int sw_phi4_get_labels(sw_phi4 *sim, uint32_t *host, int64_t n);

/* Number of sites L^4 / index of the next sweep; -1 for NULL. */
int64_t sw_phi4_sites(const sw_phi4 *sim);
int64_t sw_phi4_next_sweep(const sw_phi4 *sim);

/* Destroys the sim (waits for its stream first); NULL is a no-op. */
void sw_phi4_destroy(sw_phi4 *sim);

/* ---------------------------------------------------------------------
 * For callers that cannot allocate device memory (code under HIP graph
 * capture, tight serving loops, harnesses that forbid hipMalloc): one sweep
 * t of the L x L Ising lattice, exactly as sw_sweep runs sweep t of a sim
 * created with (L, beta, J, seed) whose spins equal `spins` -- same kernels,
 * same bits, same record.  spins: device pointer to N = L*L int8 spins
 * (+1 / -1, site order s = y*L + x, 16-byte aligned), read as the incoming
 * configuration and overwritten with the configuration sweep t leaves.
 * rec: device pointer to one sw_obs (8-byte aligned), which receives record t.  hip_stream:
 * the stream all work is enqueued on (NULL: the null stream); the call
 * returns without waiting.  Nothing is allocated: every other buffer of the
 * sweep lives in one static device array of 16 MiB per GPU, held until the
 * process ends, so L is at most 2048 (SW_ERANGE above).  All calls on one
 * GPU share that array: calls that overlap on one GPU (other streams or
 * threads) race; calls on one stream are ordered.  SW_EINVAL for NULL or
 * misaligned pointers and for L, beta or J outside their domain (as for
 * sw_create), SW_EHIP if a launch fails. */
int sw_sweep_noalloc(int32_t L, double beta, double J, uint64_t seed, uint64_t t, int8_t *spins,
                     sw_obs *rec, void *hip_stream);

#ifdef __cplusplus
}
#endif

#endif /* SWMI_H */
