// sw_internal.h -- device-state layout and kernel entry points of libswmi.
//
// One sweep (paper Sec. 2) runs as these kernels on the sim's stream:
//   k_tile    bond formation (Sec. 2.1) and cluster formation (Sec. 2.3)
//             inside one 64x64 (or 32x32) tile per workgroup, in LDS; new
//             spins (Sec. 2.4) of clusters that stay inside the tile; the
//             tile's boundary clusters become "nodes" of a global graph;
//             the spins of the previous sweep are resolved on the fly and
//             measured (Sec. 2.5).
//   k_union   union of nodes joined by bonds that cross tile edges: first
//             (k_ulocal) inside each 4x4 group of tiles in LDS, then, for
//             the edges between groups, by lock-free union-find in global
//             memory (the root is the node with the smaller index).
//   k_flatten point every node at its root; add node sizes into the roots
//             and reduce node keys to the cluster's smallest site.
//   k_roots   new spin of each cross-tile cluster, cluster statistics.
//   k_record  fold partial statistics into the per-sweep record ring (on
//             lattices of at most 64 groups the last k_roots workgroup
//             folds them, and the sweep is four launches).
// Spins are double-buffered by sweep parity.  A written spin byte is either
// the final spin (0x01 = +1, 0xFF = -1) or 2 + k, a reference to node k of
// the tile, resolved through the node tables of that sweep when the byte is
// read next (by the next sweep's k_tile, or by k_resolve at the end of
// every sw_sweep call).  The q-state Potts model runs the same kernels with
// values 0..q-1 as final bytes and node codes from 4 (64-wide tiles, q <= 4)
// or 8 (32-wide tiles).
//
// The simple cubic lattice, and the paper's label equivalence on either
// lattice, keep 32-bit labels per site in global memory instead (sw_le.hip).
#pragma once

#include <hip/hip_runtime.h>
#include <stdint.h>

#include "swmi.h"

namespace swmi {

constexpr uint32_t kNodeSlots = 256;  // node slots per tile (64x64 tile: <= 252 nodes)
constexpr int kTilePart = 32;         // int32 words of a per-tile partial
constexpr int kGroupPart = 48;        // uint64 words of a per-group partial
constexpr int kMaxQ = 8;              // largest q of the Potts model
constexpr int kAccWords = 64;         // record accumulator + completion counter
constexpr int kGroupTiles = 16;       // tiles per workgroup in k_flatten / k_roots
constexpr uint32_t kUG = 4;           // side, in tiles, of a k_ulocal group

// tile partial (int32 words)
// hist: 12 bins; TP_CNT..: population of each Potts value
enum { TP_E = 0, TP_M = 1, TP_N = 2, TP_MAX = 3, TP_SQ = 4, TP_HIST = 5, TP_CNT = 17 };
// group partial / accumulator (uint64 words)
// GP_CNT..: population of each Potts value
enum { GP_N = 0, GP_MAX = 1, GP_SQ = 2, GP_E = 3, GP_M = 4, GP_HIST = 5, GP_CNT = 38, GP_END = 46 };
enum { ACC_COUNT = 48 };

struct Dev {
    int8_t *spins[2];     // [N] by sweep parity
    uint32_t *parent[2];  // [ntiles * kNodeSlots] by sweep parity
    uint32_t *nk[2];      // [ntiles] number of nodes per tile, by parity
    uint32_t *key;        // [ntiles * kNodeSlots] smallest site of the node
    uint32_t *nsize;      // [ntiles * kNodeSlots] node size; cluster size at roots
    int8_t *rspin;        // [ntiles * kNodeSlots] new spin of each node's cluster
    uint8_t *edge;        // [ntiles][4][tw] node index of W, E, S, N edge sites
    uint64_t *xb;         // [ntiles][2] bonds leaving the tile: E (bit y), N (bit x)
    int32_t *tpart;       // [ntiles][kTilePart]
    uint64_t *gpart;      // [ngroups][kGroupPart]
    uint64_t *acc;        // [kAccWords]
    uint64_t *tdev;       // [0] = index of the next sweep
    sw_obs *ring;         // [ring_cap]
    uint32_t *labels;     // [N] or nullptr
    uint64_t *dense;      // [N + 1] or nullptr
    // label-equivalence path (SW_FLAG_LABEL_EQUIV); nullptr otherwise
    uint8_t *le_mask;     // [N] bonds of each site: bit 0 to E, bit 1 to N
    uint32_t *le_cnt;     // [N] cluster size at each root
    int8_t *le_rsp;       // [N] new spin, valid at roots
    uint32_t *le_ctl;     // [8] pass flags (3), passes of the last sweep, status
    uint32_t *bface;      // cubic bricks: [nbricks][2][256] labels of the x = 15 sites
                          // (kMapNone unless bonded to +x) and of the x = 0 sites
    uint32_t L, tw, ntx, ntiles, ngroups;
    uint32_t T, seed_lo, seed_hi;
    uint32_t ring_cap;
    uint32_t le_grid;     // workgroups of the cooperative labelling kernel (0: tile path)
    uint32_t q;           // 0: Ising; 2..kMaxQ: q-state Potts (label-equivalence path)
    uint32_t dims;        // 2: L x L; 3: L x L x L (labels in global memory)
    uint32_t brick;       // 1: simple cubic lattice on kBrick^3 bricks (else label equivalence)
    uint64_t nsite;       // N = L^dims
    double J;
};

constexpr int kStages = 5;  // kernels of one sweep, in stream order

hipError_t launch_init(const Dev &d, int cold, hipStream_t s);
hipError_t launch_stage(const Dev &d, int stage, hipStream_t s);
hipError_t launch_sweep(const Dev &d, hipStream_t s);
hipError_t launch_resolve(const Dev &d, hipStream_t s);

// Batched sweeps: each kernel of a sweep runs once over a table of
// independent lattices (replicas), each with its own Dev, so the launches
// per sweep do not grow with the batch (five per launch group under the
// global merge, the record folded by k_roots_b).  The maps list the work units
// of every replica: entry = replica << kMapShift | unit.
constexpr uint32_t kMapShift = 20;
constexpr uint32_t kMapMask = (1u << kMapShift) - 1u;
constexpr uint32_t kMapNone = 0xFFFFFFFFu;
// 4095 so that no entry (replica <= 4094) can equal kMapNone, whatever the unit
constexpr int32_t kMaxReplicas = 4095;
static_assert(((uint32_t)(kMaxReplicas - 1) << kMapShift | kMapMask) != kMapNone, "map entry collides with kMapNone");

// Replicas of at most kSmallTiles tiles may run their whole merge in one
// workgroup, in LDS (k_smerge_b); the others run the global merge.
constexpr uint32_t kSmallTiles = 16;

struct BatchDev {
    const Dev *devs;       // the replicas' Dev, in device memory
    const uint32_t *tmap;  // [ntiles] one entry per tile of every replica (k_tile, k_resolve)
    const uint32_t *wmap;  // [nwmap] tiles with an E (first nwE) or N group edge (k_union), kMapNone-padded to 4
    const uint32_t *gmap;  // [ngroups] one per group of kGroupTiles tiles (k_flatten, k_roots)
    const uint32_t *umap;  // [nugroups] one per kUG x kUG group of tiles (k_ulocal)
    const uint32_t *rmap;  // [n] the replicas (indices into devs) of the global merge
    const uint32_t *smap;  // [nsmall] the replicas merged in LDS
    const uint32_t *amap;  // [nall] every replica of the launch (records after k_resolve)
    uint32_t n, ntiles, nwmap, ngroups, nugroups, tw;
    uint32_t nwE, nsmall, nall;
    uint32_t potts;        // 1: every replica is a Potts model (q in its Dev)
};


// Paths with labels in global memory: stages 0..4 of a sweep (bonds and, for
// cubic bricks, brick-local clusters; global labelling by iterated label
// equivalence or by union-find across brick faces; new spins and sizes;
// statistics; record), and the cooperative grid size of label equivalence.
hipError_t launch_le_stage(const Dev &d, int stage, hipStream_t s);
uint32_t le_grid_size(uint32_t dims);
constexpr uint32_t kLeChunk = 4096;  // sites per workgroup in the per-site passes
constexpr uint32_t kBrick = 16;      // side of a brick of the simple cubic lattice
enum { LE_PASSES = 3, LE_STATUS = 4 };

// Stage 0 is the tile kernel of every replica; stages 1..4 the global merge;
// launch_batch_smerge the LDS merge of the small replicas, which may run
// beside stages 1..4 once stage 0 is done.  launch_batch_sweep runs them
// all in order on one stream.
hipError_t launch_batch_stage(const BatchDev &b, int stage, hipStream_t s);
hipError_t launch_batch_smerge(const BatchDev &b, hipStream_t s);
hipError_t launch_batch_sweep(const BatchDev &b, hipStream_t s);
hipError_t launch_batch_resolve(const BatchDev &b, hipStream_t s);

}  // namespace swmi
