// sw_kernels.hip -- gfx950 kernels of one Swendsen-Wang sweep (see
// sw_internal.h for the pipeline).  Written for 64-wide wavefronts: a tile
// row of 64 sites is one 64-bit mask, so row runs of horizontal bonds come
// from bit arithmetic on ballot-sized masks, and only vertical bonds go
// through the LDS union-find.
#include "sw_internal.h"
#include "sw_philox.h"
#include "sw_uf.h"

namespace swmi {
namespace {

constexpr uint32_t kEmpty = 0xFFFFFFFFu;

template <int TW> struct RowOf;
template <> struct RowOf<64> { using T = uint64_t; };
template <> struct RowOf<32> { using T = uint32_t; };

// Highest set bit of B at a position <= x (bit 0 of B is always set).
__device__ __forceinline__ uint32_t hsb_le(uint64_t B, uint32_t x) {
    const uint64_t m = B & (~0ull >> (63u - x));
    return 63u - (uint32_t)__clzll((long long)m);
}
__device__ __forceinline__ uint32_t hsb_le(uint32_t B, uint32_t x) {
    const uint32_t m = B & (~0u >> (31u - x));
    return 31u - (uint32_t)__clz((int)m);
}

// The TW-bit row mask whose 16-bit pieces (piece k at bit 16 k) are held by
// the RPT = TW / 16 consecutive lanes of a tile row (a quad for TW = 64, a
// pair for TW = 32): data-parallel moves within quads, no LDS.
template <int K, int RPT>
__device__ __forceinline__ uint32_t row_piece(uint32_t v) {
    constexpr int ctrl = RPT == 4 ? K * 0x55 : (K | (K << 2) | ((2 + K) << 4) | ((2 + K) << 6));
    return (uint32_t)__builtin_amdgcn_mov_dpp((int)v, ctrl, 0xF, 0xF, false);
}
template <int TW>
__device__ __forceinline__ typename RowOf<TW>::T row_gather(uint32_t piece) {
    if constexpr (TW == 64) {
        const uint64_t lo = row_piece<0, 4>(piece) | (row_piece<1, 4>(piece) << 16);
        const uint64_t hi = row_piece<2, 4>(piece) | (row_piece<3, 4>(piece) << 16);
        return lo | (hi << 32);
    } else {
        return row_piece<0, 2>(piece) | (row_piece<1, 2>(piece) << 16);
    }
}

// Workgroup b runs on XCD b % 8; give each XCD a contiguous band of tiles so
// that neighbouring tiles (which share halo rows and cache lines) meet in
// the same L2 (the last n mod 8 blocks keep their own index).
__device__ __forceinline__ uint32_t tile_of_block(uint32_t b, uint32_t n) {
    const uint32_t n8 = n & ~7u;
    if (b < n8) return (b & 7u) * (n8 >> 3) + (b >> 3);
    return b;
}

// ---------------------------------------------------------------- LDS union-find
// (the plain-index helpers are in sw_uf.h)
// The tile kernel's parent words hold byte offsets into the LDS array (so a
// parent is directly a load address) and carry other data in their high
// halves (a work list while the unions run).
__device__ __forceinline__ uint32_t *word_at(uint32_t *base, uint32_t off) {
    return reinterpret_cast<uint32_t *>(reinterpret_cast<char *>(base) + off);
}

// Union of the sets of the words at byte offsets a and b: parents are the
// low 16 bits, and the compare-and-swap that links the larger root under the
// smaller keeps the high half it read.  A failed swap (another lane linked
// the root, or the high half changed) resumes from what it found.
__device__ __forceinline__ void lds_union_lo(uint32_t *par, uint32_t a, uint32_t b) {
    while (true) {
        uint32_t wa = lds_load(word_at(par, a)), wb = lds_load(word_at(par, b));
        uint32_t pa = wa & 0xFFFFu, pb = wb & 0xFFFFu;
        while (pa != a || pb != b) {
            a = pa;
            b = pb;
            wa = lds_load(word_at(par, a));
            wb = lds_load(word_at(par, b));
            pa = wa & 0xFFFFu;
            pb = wb & 0xFFFFu;
        }
        if (a == b) return;
        const bool ahi = a > b;
        const uint32_t hi = ahi ? a : b, lo = ahi ? b : a;
        uint32_t expected = ahi ? wa : wb;
        const uint32_t desired = (expected & 0xFFFF0000u) | lo;
        if (__hip_atomic_compare_exchange_strong(word_at(par, hi), &expected, desired, __ATOMIC_RELAXED,
                                                 __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_WORKGROUP))
            return;
        a = lo;
        b = expected & 0xFFFFu;
    }
}

// Low half (the parent) and high half of the word at byte offset off, each
// read on its own (16-bit loads; the halves are little-endian).
__device__ __forceinline__ uint32_t lo16_at(uint32_t *base, uint32_t off) {
    return *reinterpret_cast<const uint16_t *>(reinterpret_cast<const char *>(base) + off);
}
__device__ __forceinline__ uint32_t hi16_at(uint32_t *base, uint32_t off) {
    return *reinterpret_cast<const uint16_t *>(reinterpret_cast<const char *>(base) + off + 2u);
}

// Root (byte offset) of the word at byte offset a once the unions are done.
__device__ __forceinline__ uint32_t lds_root_b(uint32_t *par, uint32_t a) {
    while (true) {
        const uint32_t p = lds_load(word_at(par, a)) & 0xFFFFu;
        if (p == a) return a;
        a = p;
    }
}



// Spin (+1/-1) encoded by a byte of the previous sweep's output that belongs
// to tile `tile`: final spins are 0x01 / 0xFF, a code 2 + k refers to node k
// of that tile, whose cluster's new spin k_roots stored at the node.
__device__ __forceinline__ int8_t resolve_byte(uint32_t b, uint32_t tile, const int8_t *nspin) {
    const uint32_t k = b - 2u;
    if (k < 252u) return nspin[tile * kNodeSlots + k];
    return (int8_t)b;
}

__device__ __forceinline__ uint32_t byte_at(const uint4 &v, int q) {
    const uint32_t w = q < 4 ? v.x : q < 8 ? v.y : q < 12 ? v.z : v.w;
    return (w >> (8 * (q & 3))) & 0xFFu;
}

// Shared front end of k_tile and k_resolve: the table that maps every byte
// of this tile's previous output to its spin as an up bit (1 for +1): final
// spins 0x01 / 0xFF map to themselves, node code 2 + k to the spin of node
// k's root.
// Output bytes of the Potts model on the tile path: a byte below
// potts_code<TW>() is a final value, potts_code<TW>() + k refers to node k of
// its tile.  A 32-wide tile has at most 124 nodes, so all values 0..7 fit
// below 8; a 64-wide tile has up to 252 nodes, which leaves bytes 0..3 for
// the values of q <= 4.
template <int TW> constexpr uint32_t potts_code() { return TW == 64 ? 4u : 8u; }

// The node spins are loaded whether or not the node exists (every slot is
// in bounds), so that this load does not wait for the node count.
template <int TW, bool POTTS>
__device__ __forceinline__ void load_table(const Dev &d, uint32_t tile, uint32_t pp, uint8_t *s_tab,
                                           uint32_t tid) {
    constexpr int NT = TW * TW / 16;
    const uint32_t kprev = min(d.nk[pp][tile], 252u);
    for (uint32_t b = tid; b < 256u; b += NT) {
        uint8_t val;
        uint32_t k;
        if constexpr (POTTS) {
            val = (uint8_t)(b & 7u);
            k = b - potts_code<TW>();
        } else {
            val = b == 0xFFu ? 0u : 1u;
            k = b - 2u;
        }
        const int8_t ns = k < 252u ? d.rspin[tile * kNodeSlots + k] : (int8_t)0;
        if (k < kprev) val = POTTS ? (uint8_t)((uint32_t)ns & 7u) : (ns > 0 ? 1u : 0u);
        s_tab[b] = val;
    }
}

template <int TW>
__device__ __forceinline__ uint32_t decode16(const uint4 &v, const uint8_t *s_tab) {
    uint32_t up = 0;
#pragma unroll
    for (int q = 0; q < 16; ++q) up |= (uint32_t)s_tab[byte_at(v, q)] << q;
    return up;
}

__device__ __forceinline__ uint32_t decode16_remote(const uint4 &v, uint32_t tile, const int8_t *nspin) {
    uint32_t up = 0;
#pragma unroll
    for (int q = 0; q < 16; ++q) up |= (uint32_t)(resolve_byte(byte_at(v, q), tile, nspin) > 0) << q;
    return up;
}

// Potts value (0..7) of a byte of tile `tile`'s previous output.
template <int TW>
__device__ __forceinline__ uint32_t potts_byte(uint32_t b, uint32_t tile, const int8_t *nspin) {
    const uint32_t k = b - potts_code<TW>();
    if (k < 252u) return (uint32_t)nspin[tile * kNodeSlots + k] & 7u;
    return b & 7u;
}

// Values of 16 sites as three bit planes (bit q of pl[i] = bit i of site q).
__device__ __forceinline__ void decode16_potts(const uint4 &v, const uint8_t *s_tab, uint32_t pl[3]) {
    pl[0] = pl[1] = pl[2] = 0u;
#pragma unroll
    for (int q = 0; q < 16; ++q) {
        const uint32_t x = s_tab[byte_at(v, q)];
        pl[0] |= (x & 1u) << q;
        pl[1] |= ((x >> 1) & 1u) << q;
        pl[2] |= (x >> 2) << q;
    }
}

template <int TW>
__device__ __forceinline__ void decode16_potts_remote(const uint4 &v, uint32_t tile, const int8_t *nspin,
                                                      uint32_t pl[3]) {
    pl[0] = pl[1] = pl[2] = 0u;
#pragma unroll
    for (int q = 0; q < 16; ++q) {
        const uint32_t x = potts_byte<TW>(byte_at(v, q), tile, nspin);
        pl[0] |= (x & 1u) << q;
        pl[1] |= ((x >> 1) & 1u) << q;
        pl[2] |= (x >> 2) << q;
    }
}

// Equal-neighbour masks of 16 sites from their bit planes and those of the
// E and N neighbours; equal pairs and the population of every value 0..7
// (two 16-bit counts per word).
__device__ __forceinline__ void potts_counts(const uint32_t pl[3], uint32_t cpk[4]) {
#pragma unroll
    for (int k = 0; k < 8; k += 2) {
        uint32_t c[2];
#pragma unroll
        for (int h = 0; h < 2; ++h) {
            const int v = k + h;
            const uint32_t m = ~((pl[0] ^ ((v & 1) ? 0xFFFFu : 0u)) | (pl[1] ^ ((v & 2) ? 0xFFFFu : 0u)) |
                                 (pl[2] ^ ((v & 4) ? 0xFFFFu : 0u))) & 0xFFFFu;
            c[h] = (uint32_t)__popc(m);
        }
        cpk[k >> 1] = c[0] | (c[1] << 16);
    }
}

// =====================================================================
// k_tile: bonds (Sec. 2.1), tile-local clusters (Sec. 2.3), new spins of
// tile-interior clusters (Sec. 2.4), measurement of the incoming
// configuration (Sec. 2.5).  One workgroup per TW x TW tile, 16 sites per
// thread (one 16-site segment of a row), so per-row bond and run data are
// bit masks and most per-site work is one bit operation per 16 sites.
// Cluster formation: every site's LDS word first points at the start of its
// row run; vertical bonds (one per group that joins the same two runs) are
// unions of run starts; each run start is then pointed at its root, which
// collects the cluster size and, after numbering, the output byte.
// =====================================================================
// POTTS: the q-state Potts model (64-wide tiles for q <= 4, else 32-wide):
// spins are values held as three bit planes, bonds join equal values, an
// interior cluster takes the Potts value of its root site, node codes start
// at potts_code<TW>(), and the tile measures equal pairs and the population
// of every value.
template <int TW, bool POTTS = false>
__device__ __forceinline__ void tile_body(const Dev &d, const uint32_t tile) {
    using Row = typename RowOf<TW>::T;
    constexpr int NT = TW * TW / 16;
    constexpr uint32_t RPT = TW / 16;
    constexpr int NS = TW * TW;
    constexpr int NW = NS / 32;
    constexpr int NWAVE = (NT + 63) / 64;
    constexpr int NPL = POTTS ? 3 : 1;  // bit planes of a spin
    constexpr uint32_t EW = (TW + 31) / 32;
    constexpr uint32_t CB = POTTS ? potts_code<TW>() : 2u;  // output byte of node 0

    // One word per site, rows padded to PS = TW + 1 words so that the 16
    // sites a lane gathers at equal offsets fall in distinct banks.  Low 16
    // bits: parent, as the byte offset of its word.  High 16 bits: the union
    // work list while the unions run, then the cluster size (roots), then
    // the root's output byte.
    constexpr uint32_t PS = TW + 1;
    __shared__ __align__(16) uint32_t s_par[TW * PS];
    // spin masks (Potts: bit planes); they are dead before s_par is first
    // written, so the 64-wide Potts tile keeps its three planes in s_par
    constexpr bool UP_IN_PAR = POTTS && TW == 64;
    static_assert(!UP_IN_PAR || 3 * (TW + 1) * sizeof(Row) <= TW * PS * 4, "planes must fit in s_par");
    __shared__ Row s_up_own[POTTS && !UP_IN_PAR ? NPL * (TW + 1) : 1];
    Row *const s_up = UP_IN_PAR ? reinterpret_cast<Row *>(s_par) : s_up_own;
    __shared__ Row s_ebnb[2 * TW];  // bond masks to E of every row (rows 0..TW-1)
    Row *const s_eb = s_ebnb;
    __shared__ Row s_fb[TW];
    __shared__ Row s_xn;
    __shared__ uint32_t s_eup[NPL * EW];
    __shared__ uint32_t s_xe[EW];
    __shared__ uint32_t s_bf[NW];
    __shared__ uint8_t s_tab[256];
    __shared__ uint32_t s_hist[12];
    // root | size << 16 of each node; for 64-wide tiles it reuses the bond
    // masks, which are dead once the unions are done
    __shared__ uint32_t s_node_own[TW == 64 ? 1 : 4 * TW];
    uint32_t *const s_node = TW == 64 ? reinterpret_cast<uint32_t *>(s_ebnb) : s_node_own;
    __shared__ int32_t s_red[NWAVE][POTTS ? 8 : 4];

    const uint32_t tid = threadIdx.x;
    const uint32_t L = d.L, ntx = d.ntx;
    const uint32_t tx = tile % ntx, ty = tile / ntx;
    const uint64_t tsw = *d.tdev;
    const uint32_t t = (uint32_t)tsw;
    const uint32_t pc = (uint32_t)(tsw & 1u), pp = pc ^ 1u;
    const int8_t *__restrict__ sin = d.spins[pc];
    int8_t *__restrict__ sout = d.spins[pp];
    uint32_t *__restrict__ par_cur = d.parent[pc];

    const uint32_t ly = tid / RPT, seg = tid % RPT, x0 = seg * 16u;
    const uint32_t gy = ty * TW + ly, gx0 = tx * TW + x0;
    const uint32_t east = ty * ntx + (tx + 1u == ntx ? 0u : tx + 1u);
    const uint32_t north = (ty + 1u == ntx ? 0u : ty + 1u) * ntx + tx;
    const uint32_t rowbase = ly * PS;  // padded index of the row's first site
    const uint32_t rowoff = 4u * rowbase;  // its byte offset
    const uint32_t srow = ly * TW;     // site index of the row's first site

    // rows of the tile a wavefront holds; lanes of a wavefront's last row
    // (Ising) decode the next row's spins themselves, the others take them
    // from the lanes RPT above
    constexpr uint32_t RPW = 64u / RPT;
    const bool wlast = (ly % RPW) == RPW - 1u;

    // ---- issue the spin loads first, then build the node table
    const uint4 v = *reinterpret_cast<const uint4 *>(sin + (size_t)gy * L + gx0);
    uint4 vn = make_uint4(0u, 0u, 0u, 0u);
    if (POTTS ? ly == TW - 1 : wlast) {
        const uint32_t gyn = (gy + 1u == L) ? 0u : gy + 1u;
        vn = *reinterpret_cast<const uint4 *>(sin + (size_t)gyn * L + gx0);
    }
    uint32_t ve = 0;
    if (seg == RPT - 1) {
        const uint32_t gxe = (gx0 + 16u == L) ? 0u : gx0 + 16u;
        ve = (uint8_t)sin[(size_t)gy * L + gxe];
    }
    // the bond words of this lane's 16 sites (Sec. 2.1), drawn while the
    // loads are in flight: bit 2j (2j+1) of rE / rN is the E / N edge of
    // site 2j (2j+1) past the lane's first site, set iff its word is below T
    uint32_t rE = 0u, rN = 0u;
    {
        const uint32_t c0 = (gy * L + gx0) >> 1;
        const uint32_t T = d.T;
#pragma unroll
        for (int j = 0; j < 8; ++j) {
            uint32_t w0 = c0 + (uint32_t)j, w1 = t, w2 = 0u, w3 = 0u;
            philox10(w0, w1, w2, w3, d.seed_lo, d.seed_hi);
            rE |= ((uint32_t)(w0 < T) << (2 * j)) | ((uint32_t)(w2 < T) << (2 * j + 1));
            rN |= ((uint32_t)(w1 < T) << (2 * j)) | ((uint32_t)(w3 < T) << (2 * j + 1));
        }
    }
    load_table<TW, POTTS>(d, tile, pp, s_tab, tid);

    // Potts: the value each of this lane's 16 sites would give its cluster
    // as its root (4 bits per site): word i of the output for counter
    // {s >> 2, t, 3, 0} for site s = 4j + i past the lane's first site
    uint64_t pv = 0;
    if constexpr (POTTS) {
        const uint32_t r0 = gy * L + gx0, q = d.q;
#pragma unroll
        for (uint32_t j = 0; j < 4u; ++j) {
            uint32_t w0 = (r0 >> 2) + j, w1 = t, w2 = 3u, w3 = 0u;
            philox10(w0, w1, w2, w3, d.seed_lo, d.seed_hi);
            const uint64_t v4 = (uint64_t)(((uint64_t)w0 * q) >> 32) | ((((uint64_t)w1 * q) >> 32) << 4) |
                                ((((uint64_t)w2 * q) >> 32) << 8) | ((((uint64_t)w3 * q) >> 32) << 12);
            pv |= v4 << (16u * j);
        }
    }
    // Ising: flip bits of every tile row, one Philox call per row of TW sites
    if (!POTTS && tid < (uint32_t)TW) {
        const uint32_t r0 = (ty * TW + tid) * L + tx * TW;
        uint32_t w0 = r0 >> 7, w1 = t, w2 = 1u, w3 = 0u;
        philox10(w0, w1, w2, w3, d.seed_lo, d.seed_hi);
        const uint32_t off = r0 & 127u;
        if constexpr (TW == 64) {
            s_fb[tid] = off == 0u ? (((uint64_t)w1 << 32) | w0) : (((uint64_t)w3 << 32) | w2);
        } else {
            const uint32_t q = off >> 5;
            s_fb[tid] = q == 0 ? w0 : q == 1 ? w1 : q == 2 ? w2 : w3;
        }
    }
    for (uint32_t i = tid; i < (uint32_t)NW; i += NT) s_bf[i] = 0u;
    if (tid < EW) s_xe[tid] = 0u;
    if (tid < NPL * EW) s_eup[tid] = 0u;
    if (tid < 12u) s_hist[tid] = 0u;
    if (tid == 0) s_xn = 0;
    __syncthreads();

    // ---- decode the incoming configuration (Sec. 2.5 measures it; Sec. 2.1
    // bonds it).  Ising: the up-spin mask of the lane's 16 sites, of the 16
    // sites above (lanes RPT further on, or decoded here by a wavefront's
    // last row) and the east neighbour of its last site (the next lane, or
    // the east tile).  Potts: three bit planes per row, through LDS.
    uint32_t up = 0u, pl[3] = {0u, 0u, 0u};
    uint32_t upN = 0u, ebit = 0u;
    if constexpr (POTTS) {
        decode16_potts(v, s_tab, pl);
#pragma unroll
        for (int b = 0; b < 3; ++b) reinterpret_cast<uint16_t *>(s_up + b * (TW + 1))[ly * RPT + seg] = (uint16_t)pl[b];
        if (ly == TW - 1) {
            uint32_t pn[3];
            decode16_potts_remote<TW>(vn, north, d.rspin, pn);
#pragma unroll
            for (int b = 0; b < 3; ++b)
                reinterpret_cast<uint16_t *>(s_up + b * (TW + 1))[TW * RPT + seg] = (uint16_t)pn[b];
        }
        if (seg == RPT - 1) {
            const uint32_t ev = potts_byte<TW>(ve, east, d.rspin);
#pragma unroll
            for (uint32_t b = 0; b < 3u; ++b)
                if ((ev >> b) & 1u) atomicOr(&s_eup[b * EW + (ly >> 5)], 1u << (ly & 31u));
        }
        __syncthreads();
    } else {
        up = decode16<TW>(v, s_tab);
        const uint32_t upA = (uint32_t)__shfl_down((int)up, (int)RPT, 64);
        const uint32_t upR = (uint32_t)__shfl_down((int)up, 1, 64);
        if (wlast)
            upN = ly == TW - 1 ? decode16_remote(vn, north, d.rspin) : decode16<TW>(vn, s_tab);
        else
            upN = upA;
        ebit = seg == RPT - 1 ? (uint32_t)(resolve_byte(ve, east, d.rspin) > 0) : (upR & 1u);
    }

    // ---- bonds (Sec. 2.1) and energy / magnetisation of the incoming spins
    // (Potts: equal pairs and value populations); then every site points at
    // the start of its row run (the row's E bonds are gathered from its RPT
    // lanes), and the bond masks go to LDS for the vertical unions
    int32_t e_part, m_part;
    uint32_t cpk[4] = {0u, 0u, 0u, 0u};
    uint32_t bE, bN;
    {
        uint32_t eqE, eqN;
        if constexpr (POTTS) {
            uint32_t dE = 0u, dN = 0u;
#pragma unroll
            for (int b = 0; b < 3; ++b) {
                const Row rowv = s_up[b * (TW + 1) + ly];
                const uint32_t pN = (uint32_t)(s_up[b * (TW + 1) + ly + 1] >> x0) & 0xFFFFu;
                const uint32_t eb = (s_eup[b * EW + (ly >> 5)] >> (ly & 31u)) & 1u;
                const uint32_t nxt = (x0 + 16u < (uint32_t)TW) ? ((uint32_t)(rowv >> (x0 + 16u)) & 1u) : eb;
                const uint32_t pE = (pl[b] >> 1) | (nxt << 15);
                dE |= pl[b] ^ pE;
                dN |= pl[b] ^ pN;
            }
            eqE = ~dE & 0xFFFFu;
            eqN = ~dN & 0xFFFFu;
            e_part = __popc(eqE) + __popc(eqN);
            m_part = 0;
            potts_counts(pl, cpk);
        } else {
            const uint32_t upE = (up >> 1) | (ebit << 15);
            eqE = ~(up ^ upE) & 0xFFFFu;
            eqN = ~(up ^ upN) & 0xFFFFu;
            e_part = 2 * (__popc(eqE) + __popc(eqN)) - 32;
            m_part = 2 * __popc(up) - 16;
        }
        bE = eqE & rE;
        bN = eqN & rN;
        if (seg == RPT - 1) {
            if (bE >> 15) atomicOr(&s_xe[ly >> 5], 1u << (ly & 31u));
            bE &= 0x7FFFu;
        }
        if (ly == TW - 1) {
            reinterpret_cast<uint16_t *>(&s_xn)[seg] = (uint16_t)bN;
            bN = 0u;
        }
        reinterpret_cast<uint16_t *>(s_eb)[ly * RPT + seg] = (uint16_t)bE;
    }
    const Row E0 = row_gather<TW>(bE);  // this row's E bonds inside the tile
    const Row V = row_gather<TW>(bN);   // this row's N bonds inside the tile
    const Row B0 = (Row)~(Row)(E0 << 1);
    const uint32_t st = (uint32_t)(B0 >> x0) & 0xFFFFu;
    const uint32_t rs0 = rowoff + 4u * hsb_le(B0, x0);  // byte offset of the run start at x0
    // the 64-wide Potts tile keeps its planes in s_par: wait until every
    // lane has read them
    if constexpr (UP_IN_PAR) __syncthreads();
    {
        uint32_t cur = rs0;
#pragma unroll
        for (int q = 0; q < 16; ++q) {
            if ((st >> q) & 1u) cur = rowoff + 4u * (x0 + (uint32_t)q);
            s_par[rowbase + x0 + q] = cur;
        }
        if (seg == RPT - 1u) s_par[rowbase + TW] = 0u;  // pad word: list slot only
    }
    __syncthreads();

    // ---- vertical bonds join runs of adjacent rows.  One union per group of
    // vertical bonds that connect the same pair of runs; each wavefront lists
    // its unions in the high halves of its own rows' words and then works
    // through the list 64 at a time, so that lanes with many bonds do not
    // hold up the rest.  The list is private to the wavefront; the compare-
    // and-swap of a union keeps a word's high half and retries if it
    // changed, so other wavefronts may build or clear their lists meanwhile.
    uint32_t r = 0u;  // representative vertical bonds of this segment
    if (ly + 1u < (uint32_t)TW) {
        const Row E1 = s_eb[ly + 1];
        const Row R = V & (Row)~(Row)((V << 1) & (E0 << 1) & (E1 << 1));
        r = (uint32_t)(R >> x0) & 0xFFFFu;
    }
    const uint32_t lane = tid & 63u;
    const uint32_t wbase = (tid >> 6) * (64u / RPT) * PS;
    uint32_t nlist;
    {
        const uint32_t c = __popc(r);
        uint32_t pre = 0u;
        nlist = 0u;
#pragma unroll
        for (int j = 0; j < 5; ++j) {
            const uint64_t bal = __ballot((c >> j) & 1u);
            pre += (uint32_t)__builtin_amdgcn_mbcnt_hi((uint32_t)(bal >> 32),
                                                      __builtin_amdgcn_mbcnt_lo((uint32_t)bal, 0u))
                   << j;
            nlist += (uint32_t)__popcll(bal) << j;
        }
        uint32_t w = wbase + pre, rr = r;
        while (rr) {
            const uint32_t i = (uint32_t)__ffs((int)rr) - 1u;
            rr &= rr - 1u;
            __hip_atomic_fetch_or(&s_par[w], (rowoff + 4u * (x0 + i)) << 16, __ATOMIC_RELAXED,
                                  __HIP_MEMORY_SCOPE_WORKGROUP);
            ++w;
        }
    }
    __builtin_amdgcn_fence(__ATOMIC_ACQ_REL, "wavefront");
    __builtin_amdgcn_wave_barrier();
    for (uint32_t k = lane; k < nlist; k += 64u) {
        const uint32_t n = lds_load(&s_par[wbase + k]) >> 16;
        __hip_atomic_fetch_and(&s_par[wbase + k], 0xFFFFu, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_WORKGROUP);
        lds_union_lo(s_par, n, n + 4u * PS);
    }
    __syncthreads();

    // ---- cluster sizes.  Every run start in this lane's 16 sites is pointed
    // at its root and adds the whole run's length (read off the row's
    // run-start mask; the run may go on into the next lanes' sites).  Runs
    // that touch the tile edge mark their root: the S and N rows, the first
    // run of every row (x = 0) and the run holding x = TW - 1.
    uint32_t rootmask = 0u;
    {
        const bool edge_row = ly == 0u || ly == TW - 1u;
        // where the run holding the lane's last site ends: the first run
        // start past the lane's 16 sites, or the row's end
        uint32_t end_out = (uint32_t)TW;
        if (x0 + 16u < (uint32_t)TW) {
            const Row past = (Row)(B0 >> (x0 + 16u));
            if (past) end_out = x0 + 16u + (uint32_t)__builtin_ctzll((unsigned long long)past);
        }
        // lengths of consecutive runs with the same root are summed in a
        // register (at most TW per lane) and added with one atomic
        uint32_t acc_root = 0u, acc_len = 0u;
        uint32_t m = st;
        while (m) {
            const uint32_t i = (uint32_t)__ffs((int)m) - 1u;
            m &= m - 1u;
            const uint32_t n = rowoff + 4u * (x0 + i);
            const uint32_t root = lds_root_b(s_par, n);
            if (root != n)
                __hip_atomic_store(word_at(s_par, n), root, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_WORKGROUP);
            else
                rootmask |= 1u << i;
            if (edge_row || (seg == 0u && i == 0u) || (seg == RPT - 1u && m == 0u)) {
                const uint32_t rsite = root / 4u - root / (4u * PS);
                atomicOr(&s_bf[rsite >> 5], 1u << (rsite & 31u));
            }
            // the run goes on to the lane's next run start, or past the lane
            const uint32_t len = (m ? (uint32_t)__ffs((int)m) - 1u + x0 : end_out) - (x0 + i);
            if (root != acc_root && acc_len != 0u)
                __hip_atomic_fetch_add(word_at(s_par, acc_root), acc_len << 16, __ATOMIC_RELAXED,
                                       __HIP_MEMORY_SCOPE_WORKGROUP);
            acc_len = root != acc_root ? len : acc_len + len;
            acc_root = root;
        }
        if (acc_len != 0u)
            __hip_atomic_fetch_add(word_at(s_par, acc_root), acc_len << 16, __ATOMIC_RELAXED,
                                   __HIP_MEMORY_SCOPE_WORKGROUP);
        // a segment that starts inside a run which reaches the S or N edge,
        // or (last segment of a row) holds no run start of its own
        if (!(st & 1u) && (edge_row || (seg == RPT - 1u && st == 0u))) {
            const uint32_t root = lds_root_b(s_par, rs0);
            const uint32_t rsite = root / 4u - root / (4u * PS);
            atomicOr(&s_bf[rsite >> 5], 1u << (rsite & 31u));
        }
    }
    __syncthreads();

    // ---- number the boundary clusters (nodes) in site order: every
    // wavefront scans the marks itself, lane l holding the prefix of mark
    // words (NW / 64) l .. (NW / 64) (l + 1) - 1
    uint32_t pf_a, pf_b, n_nodes;
    {
        uint32_t wa = 0u, wb = 0u, c;
        if constexpr (NW == 128) {
            wa = s_bf[2 * lane];
            wb = s_bf[2 * lane + 1];
            c = __popc(wa) + __popc(wb);
        } else {
            wa = lane < (uint32_t)NW ? s_bf[lane] : 0u;
            c = __popc(wa);
        }
        uint32_t incl = c;
#pragma unroll
        for (int o = 1; o < 64; o <<= 1) {
            const uint32_t n = __shfl_up(incl, o, 64);
            if (lane >= (uint32_t)o) incl += n;
        }
        pf_a = incl - c;
        pf_b = pf_a + __popc(wa);
        // at most 4 (TW - 1) boundary clusters; the bound keeps the node
        // tables in their slots whatever the marks
        n_nodes = min((uint32_t)__shfl((int)incl, 63, 64), 4u * ((uint32_t)TW - 1u));
    }

    // ---- roots: output byte into the root's word; node entries staged in
    // LDS; interior-cluster statistics (size classes 0-2 packed in one
    // register, 10 bits each)
    uint32_t max_int = 0u, sq_int = 0u, hpk = 0u;
    {
        const uint32_t sbase = srow + x0;  // site index of this lane's first site
        const uint32_t bfw = s_bf[sbase >> 5];
        const uint32_t bsh = sbase & 31u;
        const uint32_t bmask = (bfw >> bsh) & 0xFFFFu;
        // prefix of mark word sbase >> 5, held by lane (sbase >> 5) / (NW / 64)
        uint32_t pf;
        if constexpr (NW == 128) {
            const uint32_t qa = (uint32_t)__shfl((int)pf_a, (int)((sbase >> 5) >> 1), 64);
            const uint32_t qb = (uint32_t)__shfl((int)pf_b, (int)((sbase >> 5) >> 1), 64);
            pf = ((sbase >> 5) & 1u) ? qb : qa;
        } else {
            pf = (uint32_t)__shfl((int)pf_a, (int)(sbase >> 5), 64);
        }
        const uint32_t kbase = pf + __popc(bfw & ((1u << bsh) - 1u));
        const uint32_t fl = POTTS ? 0u : (uint32_t)(s_fb[ly] >> x0) & 0xFFFFu;
        while (rootmask) {
            const uint32_t q = (uint32_t)__ffs((int)rootmask) - 1u;
            rootmask &= rootmask - 1u;
            const uint32_t root = rowbase + x0 + q;
            const uint32_t S = hi16_at(s_par, 4u * root);
            uint32_t code;
            if ((bmask >> q) & 1u) {
                const uint32_t k = kbase + __popc(bmask & ((1u << q) - 1u));
                s_node[k] = (sbase + q) | (S << 16);
                code = CB + k;
            } else {
                if constexpr (POTTS)
                    code = (uint32_t)(pv >> (4u * q)) & 0xFu;
                else
                    code = ((fl >> q) & 1u) ? 0xFFu : 0x01u;
                max_int = max(max_int, S);
                sq_int += S * S;
                const uint32_t bin = 31u - (uint32_t)__clz((int)S);
                if (bin < 3u)
                    hpk += 1u << (10u * bin);
                else
                    atomicAdd(&s_hist[bin], 1u);
                if (d.dense) atomicAdd(reinterpret_cast<unsigned long long *>(&d.dense[S]), 1ull);
            }
            s_par[root] = (4u * root) | (code << 16);
        }
    }
    __syncthreads();
    // node tables of this tile, written in node order
    for (uint32_t k = tid; k < n_nodes; k += NT) {
        const uint32_t e = s_node[k], site = e & 0xFFFFu, node = tile * kNodeSlots + k;
        d.key[node] = (ty * TW + site / TW) * L + tx * TW + site % TW;
        d.nsize[node] = e >> 16;
        par_cur[node] = node;
    }

    // ---- outputs: one byte per site (final spin or node code)
    uint32_t out[4] = {0u, 0u, 0u, 0u};
    {
        uint32_t cur = rs0;
#pragma unroll
        for (int q = 0; q < 16; ++q) {
            if ((st >> q) & 1u) cur = rowoff + 4u * (x0 + (uint32_t)q);
            const uint32_t root = lo16_at(s_par, cur);
            const uint32_t code = hi16_at(s_par, root);
            out[q >> 2] |= code << (8 * (q & 3));
        }
    }
    *reinterpret_cast<uint4 *>(sout + (size_t)gy * L + gx0) = make_uint4(out[0], out[1], out[2], out[3]);
    if (d.labels) {
        uint32_t lab[16];
        uint32_t cur = rs0;
#pragma unroll
        for (int q = 0; q < 16; ++q) {
            if ((st >> q) & 1u) cur = rowoff + 4u * (x0 + (uint32_t)q);
            const uint32_t root = lo16_at(s_par, cur);
            const uint32_t rsite = root / 4u - root / (4u * PS);
            const uint32_t code = (out[q >> 2] >> (8 * (q & 3))) & 0xFFu;
            lab[q] = (code >= CB && code < CB + 252u) ? (0x80000000u | (tile * kNodeSlots + code - CB))
                                                      : (ty * TW + rsite / TW) * L + tx * TW + rsite % TW;
        }
        uint4 *lp = reinterpret_cast<uint4 *>(d.labels + (size_t)gy * L + gx0);
        lp[0] = make_uint4(lab[0], lab[1], lab[2], lab[3]);
        lp[1] = make_uint4(lab[4], lab[5], lab[6], lab[7]);
        lp[2] = make_uint4(lab[8], lab[9], lab[10], lab[11]);
        lp[3] = make_uint4(lab[12], lab[13], lab[14], lab[15]);
    }
    {
        // node index of every edge site (all of them belong to nodes)
        uint8_t *eg = d.edge + (size_t)tile * 4u * TW;
        // (every edge byte is a node code, so the bytewise subtraction never borrows)
        constexpr uint32_t CB4 = CB * 0x01010101u;
        if (seg == 0u) eg[0 * TW + ly] = (uint8_t)((out[0] & 0xFFu) - CB);
        if (seg == RPT - 1u) eg[1 * TW + ly] = (uint8_t)((out[3] >> 24) - CB);
        if (ly == 0u)
            *reinterpret_cast<uint4 *>(eg + 2 * TW + x0) = make_uint4(out[0] - CB4, out[1] - CB4, out[2] - CB4, out[3] - CB4);
        if (ly == (uint32_t)TW - 1u)
            *reinterpret_cast<uint4 *>(eg + 3 * TW + x0) = make_uint4(out[0] - CB4, out[1] - CB4, out[2] - CB4, out[3] - CB4);
    }
    // energy and magnetisation packed as (e + 32) | (m + 16) << 16 per lane:
    // the wavefront sums stay below 2^13 and 2^12
    // (Potts: the equal pairs alone, at most 32 per lane)
    uint32_t em = POTTS ? (uint32_t)e_part : (uint32_t)(e_part + 32) | ((uint32_t)(m_part + 16) << 16);

    // ---- workgroup reductions -> tile partial
#pragma unroll
    for (int o = 32; o > 0; o >>= 1) {
        em += __shfl_xor(em, o, 64);
        hpk += __shfl_xor(hpk, o, 64);
        max_int = max(max_int, (uint32_t)__shfl_xor((int)max_int, o, 64));
        sq_int += __shfl_xor(sq_int, o, 64);
        if constexpr (POTTS) {
#pragma unroll
            for (int i = 0; i < 4; ++i) cpk[i] += __shfl_xor(cpk[i], o, 64);
        }
    }
    if ((tid & 63u) == 0u) {
        s_red[tid >> 6][0] = (int32_t)em;
        s_red[tid >> 6][1] = (int32_t)hpk;
        s_red[tid >> 6][2] = (int32_t)max_int;
        s_red[tid >> 6][3] = (int32_t)sq_int;
        if constexpr (POTTS) {
#pragma unroll
            for (int i = 0; i < 4; ++i) s_red[tid >> 6][4 + i] = (int32_t)cpk[i];
        }
    }
    __syncthreads();
    if (tid == 0u) {
        int32_t e = 0, m = 0, mx = 0, sq = 0, b0 = 0, b1 = 0, b2 = 0;
        for (int w = 0; w < NWAVE; ++w) {
            const uint32_t ew = (uint32_t)s_red[w][0], hw = (uint32_t)s_red[w][1];
            if constexpr (POTTS) {
                e += (int32_t)ew;
            } else {
                e += (int32_t)(ew & 0xFFFFu) - 32 * 64;
                m += (int32_t)(ew >> 16) - 16 * 64;
            }
            b0 += (int32_t)(hw & 0x3FFu);
            b1 += (int32_t)((hw >> 10) & 0x3FFu);
            b2 += (int32_t)(hw >> 20);
            mx = max(mx, s_red[w][2]);
            sq += s_red[w][3];
        }
        int32_t n = b0 + b1 + b2;
        for (int b = 3; b < 12; ++b) n += (int32_t)s_hist[b];
        int32_t *tp = d.tpart + (size_t)tile * kTilePart;
        tp[TP_E] = e;
        tp[TP_M] = m;
        tp[TP_N] = n;
        tp[TP_MAX] = mx;
        tp[TP_SQ] = sq;
        tp[TP_HIST + 0] = b0;
        tp[TP_HIST + 1] = b1;
        tp[TP_HIST + 2] = b2;
        for (int b = 3; b < 12; ++b) tp[TP_HIST + b] = (int32_t)s_hist[b];
        if constexpr (POTTS) {
            for (int k = 0; k < 8; ++k) {
                int32_t c = 0;
                for (int w = 0; w < NWAVE; ++w) c += (int32_t)(((uint32_t)s_red[w][4 + k / 2] >> (16 * (k & 1))) & 0xFFFFu);
                tp[TP_CNT + k] = c;
            }
        }
        d.nk[pc][tile] = n_nodes;
        uint64_t xe = s_xe[0];
        if constexpr (TW == 64) xe |= (uint64_t)s_xe[1] << 32;
        d.xb[2u * tile] = xe;
        d.xb[2u * tile + 1u] = (uint64_t)s_xn;
    }
}

// 64-wide tiles: at most 64 VGPRs, so that the 8 workgroups per CU that the
// LDS allows (8 wavefronts per SIMD) all fit.
constexpr int kTileWavesPerEU = 8;

template <int TW, bool POTTS = false>
__global__ __launch_bounds__(TW *TW / 16, TW == 64 ? kTileWavesPerEU : 1) void k_tile(Dev d) {
    tile_body<TW, POTTS>(d, tile_of_block(blockIdx.x, d.ntiles));
}

// Batched launches run the same bodies over a table of replicas (map
// entries replica << kMapShift | unit index), so every replica's bits are
// those of its own plain sweep.
template <int TW, bool POTTS = false>
__global__ __launch_bounds__(TW *TW / 16, TW == 64 ? kTileWavesPerEU : 1) void k_tile_b(const Dev *devs, const uint32_t *map) {
    const uint32_t e = map[tile_of_block(blockIdx.x, gridDim.x)];
    tile_body<TW, POTTS>(devs[e >> kMapShift], e & kMapMask);
}

// =====================================================================
// k_union: bonds that leave a tile through its E or N edge join the nodes
// on both sides (Sec. 2.3, global part).  One wavefront per tile.
// =====================================================================
// The global union-find links nodes by index (sw_uf.h); the cluster's
// smallest site is gathered separately (k_flatten takes the minimum of the
// nodes' keys into the root's key), so finds never read keys.
template <int TW>
__device__ __forceinline__ void union_body(const Dev &d, const uint32_t tile, const uint32_t dir) {
    const uint32_t lane = threadIdx.x & 63u;
    const uint32_t ntx = d.ntx, tx = tile % ntx, ty = tile / ntx;
    // edges to a tile of the same kUG x kUG group were joined by k_ulocal
    const bool glob = dir == 0u ? ((tx % kUG) == kUG - 1u || tx + 1u == ntx)
                                : ((ty % kUG) == kUG - 1u || ty + 1u == ntx);
    if (!glob) return;
    static_assert(TW <= 64, "one lane per edge position");
    const uint32_t nb = dir == 0u ? ty * ntx + (tx + 1u == ntx ? 0u : tx + 1u)
                                  : (ty + 1u == ntx ? 0u : ty + 1u) * ntx + tx;
    const uint8_t *eg = d.edge + (size_t)tile * 4u * TW;
    const uint8_t *egb = d.edge + (size_t)nb * 4u * TW;
    // one lane per edge position; the bond bits, both sides' node bytes and
    // the sweep parity are all loaded before any of them is waited on
    const bool in = lane < (uint32_t)TW;
    const uint32_t i = in ? lane : 0u;
    const uint32_t an = dir == 0u ? eg[1 * TW + i] : eg[3 * TW + i];
    const uint32_t bn = dir == 0u ? egb[0 * TW + i] : egb[2 * TW + i];
    const uint64_t bits = d.xb[2u * tile + dir];
    // (volatile: keeps the compiler from sinking the load to its first use)
    const uint32_t pc = (uint32_t)(*(volatile const uint64_t *)d.tdev & 1u);
    uint32_t *par = pc ? d.parent[1] : d.parent[0];
    const bool has = in && ((bits >> i) & 1u);
    const uint32_t a = tile * kNodeSlots + an, b = nb * kNodeSlots + bn;
    // every union starts from the two nodes' parents (their group roots, or
    // nearer the root); a bond whose parents equal those of the previous
    // bond along the edge adds nothing, so only the first of such a run
    // links (fewer lanes compete for the same roots' compare-and-swap)
    uint32_t ra = 0u, rb = 0u;
    if (has) {
        ra = g_load(&par[a]);
        rb = g_load(&par[b]);
    }
    const uint64_t below = __ballot(has) & ((1ull << lane) - 1ull);
    const int prev = below ? 63 - __clzll((long long)below) : (int)lane;
    const uint32_t pra = (uint32_t)__shfl((int)ra, prev, 64), prb = (uint32_t)__shfl((int)rb, prev, 64);
    const bool dup = below != 0ull && pra == ra && prb == rb;
    if (has && !dup) g_union(par, ra, rb);
}

// =====================================================================
// k_ulocal: the bonds between tiles of one kUG x kUG group join their nodes
// in LDS (local index = tile-in-group * kNodeSlots + node, which orders
// nodes as their global indices do, so the smaller index is the root in
// both); every node then points at its group-local root in global memory,
// and k_union only has the edges between groups left.
// =====================================================================
template <int TW>
__device__ __forceinline__ void ulocal_body(const Dev &d, const uint32_t ugroup) {
    constexpr uint32_t NG = kUG * kUG;
    __shared__ uint32_t s_p[NG * kNodeSlots];
    const uint32_t tid = threadIdx.x, lane = tid & 63u;
    const uint32_t pc = (uint32_t)(*d.tdev & 1u);
    const uint32_t ntx = d.ntx, ngx = (ntx + kUG - 1u) / kUG;
    const uint32_t gx = ugroup % ngx, gy = ugroup / ngx;
    auto tile_of = [&](uint32_t t) { return (gy * kUG + t / kUG) * ntx + gx * kUG + t % kUG; };
    auto valid = [&](uint32_t t) { return gx * kUG + t % kUG < ntx && gy * kUG + t / kUG < ntx; };
    // tile-edges inside the group: E edges (lx < kUG-1), then N edges (ly <
    // kUG-1), one position per thread and iteration; all of a thread's loads
    // are issued first (they do not depend on the sweep parity), then the
    // node counts, then the unions
    constexpr uint32_t NE = (kUG - 1u) * kUG;
    constexpr uint32_t NIT = 2u * NE * TW / 256u;
    static_assert(2u * NE * TW % 256u == 0u, "edge positions must fill the workgroup");
    uint32_t ua[NIT], ub[NIT];
    bool uh[NIT];
#pragma unroll
    for (uint32_t it = 0; it < NIT; ++it) {
        const uint32_t f = tid + 256u * it, e = f / TW, i = f % TW;
        const bool isn = e >= NE;
        const uint32_t e2 = isn ? e - NE : e;
        const uint32_t lx = isn ? e2 % kUG : e2 % (kUG - 1u), ly = isn ? e2 / kUG : e2 / (kUG - 1u);
        const uint32_t ta = ly * kUG + lx, tb = isn ? ta + kUG : ta + 1u;
        const bool ok = valid(ta) && valid(tb);
        const uint32_t A = ok ? tile_of(ta) : 0u, B = ok ? tile_of(tb) : 0u;  // tile 0: read and ignored
        const uint8_t *ea = d.edge + (size_t)A * 4u * TW, *eb = d.edge + (size_t)B * 4u * TW;
        uh[it] = ok && ((d.xb[2u * A + (isn ? 1u : 0u)] >> i) & 1u);
        ua[it] = ta * kNodeSlots + (isn ? ea[3 * TW + i] : ea[1 * TW + i]);
        ub[it] = tb * kNodeSlots + (isn ? eb[2 * TW + i] : eb[0 * TW + i]);
    }
    // 16 threads per tile of the group (thread tid: tile tid / 16, node
    // slots tid % 16 + 16 m), so that the slots of every tile's nodes, and
    // only those, are set up and later resolved in about nk / 16 steps
    static_assert(NG * 16u == 256u, "16 threads per tile");
    const uint32_t mt = tid >> 4, mk = tid & 15u;
    const uint32_t nkt = valid(mt) ? min(d.nk[pc][tile_of(mt)], 252u) : 0u;
    for (uint32_t k = mk; k < nkt; k += 16u) s_p[mt * kNodeSlots + k] = mt * kNodeSlots + k;
    __syncthreads();
#pragma unroll
    for (uint32_t it = 0; it < NIT; ++it) {
        const uint32_t i = (tid + 256u * it) % TW, a = ua[it], b = ub[it];
        const bool has = uh[it];
        // a run of bonds along the edge between the same two nodes needs one union
        const uint32_t pa = __shfl_up(a, 1, 64), pb = __shfl_up(b, 1, 64);
        const int ph = __shfl_up((int)has, 1, 64);
        const bool dup = i > 0u && lane > 0u && ph && pa == a && pb == b;
        if (has && !dup) lds_union(s_p, a, b);
    }
    __syncthreads();

    uint32_t *par = d.parent[pc];
    const uint32_t gt = tile_of(mt);
    for (uint32_t k = mk; k < nkt; k += 16u) {
        const uint32_t li = mt * kNodeSlots + k;
        const uint32_t r = lds_root(s_p, li);
        if (r != li) par[gt * kNodeSlots + k] = tile_of(r / kNodeSlots) * kNodeSlots + r % kNodeSlots;
    }
}

template <int TW>
__global__ __launch_bounds__(256) void k_ulocal(Dev d) {
    ulocal_body<TW>(d, blockIdx.x);
}

template <int TW>
__global__ __launch_bounds__(256) void k_ulocal_b(const Dev *devs, const uint32_t *map) {
    const uint32_t e = map[blockIdx.x];
    ulocal_body<TW>(devs[e >> kMapShift], e & kMapMask);
}

// One wavefront per (tile, direction): wave w of the launch takes tile w / 2
// and its E (w even) or N (w odd) edge.
// Plain lattices launch only the edges between kUG x kUG groups: wave w <
// ngx * ntx takes the E edge of the last tile column of a group in tile row
// w / ngx; the next ngx * ntx waves the N edges of the groups' last tile rows.
template <int TW>
__global__ __launch_bounds__(256) void k_union(Dev d) {
    const uint32_t ntx = d.ntx, ngx = (ntx + kUG - 1u) / kUG, nE = ngx * ntx;
    uint32_t w = blockIdx.x * 4u + (threadIdx.x >> 6);
    if (w < nE) {
        const uint32_t ty = w / ngx, tx = min((w % ngx) * kUG + kUG - 1u, ntx - 1u);
        union_body<TW>(d, ty * ntx + tx, 0u);
    } else if ((w -= nE) < nE) {
        const uint32_t tx = w % ntx, ty = min((w / ntx) * kUG + kUG - 1u, ntx - 1u);
        union_body<TW>(d, ty * ntx + tx, 1u);
    }
}

// One wavefront per map entry: the first nE entries are tiles whose E edge
// is a group edge, the rest tiles whose N edge is (kMapNone pads the map to
// whole workgroups).
template <int TW>
__global__ __launch_bounds__(256) void k_union_b(const Dev *devs, const uint32_t *map, uint32_t nE) {
    const uint32_t w = blockIdx.x * 4u + (threadIdx.x >> 6);
    const uint32_t e = map[w];
    if (e != kMapNone) union_body<TW>(devs[e >> kMapShift], e & kMapMask, w < nE ? 0u : 1u);
}

// =====================================================================
// k_flatten: every node points at its root; node sizes are summed into the
// root's size and node keys (smallest sites) reduced to their minimum in the
// root's key, first per workgroup in an LDS hash, then with one global
// atomic of each kind per (workgroup, root).  The structure is final here,
// so finds only read and the only stores are roots.
// =====================================================================
constexpr int kHashSlots = 2048;

// Node count of tile i in the sweep of parity pc: both parities are loaded,
// so that the loads need not wait for the sweep index.
__device__ __forceinline__ uint32_t nk_either(const Dev &d, uint32_t pc, uint32_t i) {
    const uint32_t a = d.nk[0][i], b = d.nk[1][i];
    return pc ? b : a;
}

__device__ __forceinline__ void hash_add(uint32_t *hk, uint32_t *hv, uint32_t *hm, uint32_t root, uint32_t size,
                                         uint32_t key, const Dev &d) {
    uint32_t h = (root * 2654435761u) >> 21;  // 11 bits
    for (int probe = 0; probe < 64; ++probe) {
        const uint32_t cur = lds_load(&hk[h]);
        bool mine = cur == root;
        if (cur == kEmpty) {
            const uint32_t old = atomicCAS(&hk[h], kEmpty, root);
            mine = old == kEmpty || old == root;
        }
        if (mine) {
            atomicAdd(&hv[h], size);
            atomicMin(&hm[h], key);
            return;
        }
        h = (h + 1u) & (kHashSlots - 1);
    }
    atomicAdd(&d.nsize[root], size);
    if (key < g_load(&d.key[root])) atomicMin(&d.key[root], key);
}

// FT tiles per workgroup (16: the tile groups): a root gets one atomic of
// each kind per workgroup that holds some of its nodes, so a cluster that
// spans the lattice receives ntiles / FT of them, one after the other.  A key
// minimum is skipped when a plain read already shows a key no larger (keys
// only decrease).
template <uint32_t FT>
__device__ __forceinline__ void flatten_body(const Dev &d, const uint32_t group) {
    __shared__ uint32_t hk[kHashSlots];
    __shared__ uint32_t hv[kHashSlots];
    __shared__ uint32_t hm[kHashSlots];
    for (uint32_t i = threadIdx.x; i < (uint32_t)kHashSlots; i += 256u) {
        hk[i] = kEmpty;
        hv[i] = 0u;
        hm[i] = kEmpty;
    }
    __syncthreads();
    const uint32_t pc = (uint32_t)(*d.tdev & 1u);
    uint32_t *par = d.parent[pc];
    const uint32_t lane = threadIdx.x & 63u, wv = threadIdx.x >> 6;
    const uint32_t g0 = group * FT;
    static_assert(FT % 16u == 0u, "four tiles per wavefront and quad");
    // wavefront wv owns tiles g0 + wv + 4q, taken four at a time (a quad);
    // the nodes of a quad are numbered one after the other (about 80 per
    // tile at beta_c, so mostly one batch), and each lane chases the roots
    // of up to 8 nodes at once, one level per round, so their loads overlap
    for (uint32_t quad = 0; quad < FT / 16u; ++quad) {
    uint32_t nkq[4];
#pragma unroll
    for (uint32_t q = 0; q < 4u; ++q) {
        const uint32_t tile = g0 + wv + 4u * (4u * quad + q);
        const uint32_t v = nk_either(d, pc, min(tile, d.ntiles - 1u));  // issued unconditionally
        nkq[q] = tile < d.ntiles ? min(v, 252u) : 0u;
    }
    const uint32_t pre1 = nkq[0], pre2 = pre1 + nkq[1], pre3 = pre2 + nkq[2], tot = pre3 + nkq[3];
    constexpr uint32_t kChase = 8;
#pragma unroll
    for (uint32_t m0 = 0; m0 < 4u * 252u / 64u + 1u; m0 += kChase) {
        if (64u * m0 >= tot) break;
        uint32_t nd[kChase], r[kChase];
#pragma unroll
        for (uint32_t j = 0; j < kChase; ++j) {
            const uint32_t i = lane + 64u * (m0 + j);
            const uint32_t q = (uint32_t)(i >= pre1) + (uint32_t)(i >= pre2) + (uint32_t)(i >= pre3);
            const uint32_t base = q == 0u ? 0u : q == 1u ? pre1 : q == 2u ? pre2 : pre3;
            nd[j] = i < tot ? (g0 + wv + 4u * (4u * quad + q)) * kNodeSlots + (i - base) : kEmpty;
            r[j] = nd[j];
        }
        bool more = true;
        while (more) {
            // all loads first (an empty slot reads node 0 and ignores it)
            uint32_t p[kChase];
#pragma unroll
            for (uint32_t j = 0; j < kChase; ++j)
                p[j] = __hip_atomic_load(&par[r[j] == kEmpty ? 0u : r[j]], __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
            more = false;
#pragma unroll
            for (uint32_t j = 0; j < kChase; ++j) {
                const uint32_t q = r[j] == kEmpty ? kEmpty : p[j];
                more |= q != r[j];
                r[j] = q;
            }
        }
#pragma unroll
        for (uint32_t j = 0; j < kChase; ++j) {
            if (nd[j] == kEmpty || r[j] == nd[j]) continue;
            g_store(&par[nd[j]], r[j]);
            hash_add(hk, hv, hm, r[j], d.nsize[nd[j]], d.key[nd[j]], d);
        }
    }
    }
    __syncthreads();
    // each thread flushes kHashSlots / 256 slots; the current keys of all its
    // roots are read before any atomic so that those loads overlap
    constexpr uint32_t kPer = (uint32_t)kHashSlots / 256u;
    uint32_t fk[kPer], fm[kPer];
#pragma unroll
    for (uint32_t j = 0; j < kPer; ++j) fk[j] = hk[threadIdx.x + 256u * j];
#pragma unroll
    for (uint32_t j = 0; j < kPer; ++j) fm[j] = fk[j] != kEmpty ? g_load(&d.key[fk[j]]) : 0u;
#pragma unroll
    for (uint32_t j = 0; j < kPer; ++j) {
        if (fk[j] == kEmpty) continue;
        const uint32_t i = threadIdx.x + 256u * j;
        atomicAdd(&d.nsize[fk[j]], hv[i]);
        if (hm[i] < fm[j]) atomicMin(&d.key[fk[j]], hm[i]);
    }
}

template <uint32_t FT>
__global__ __launch_bounds__(256) void k_flatten(Dev d) { flatten_body<FT>(d, blockIdx.x); }

__global__ __launch_bounds__(256) void k_flatten_b(const Dev *devs, const uint32_t *map) {
    const uint32_t e = map[blockIdx.x];
    flatten_body<kGroupTiles>(devs[e >> kMapShift], e & kMapMask);
}

// Canonical labels of sites of cross-tile clusters (only with SW_FLAG_LABELS).
__global__ __launch_bounds__(256) void k_relabel(Dev d) {
    const size_t n = (size_t)d.L * d.L;
    const uint32_t pc = (uint32_t)(*d.tdev & 1u);
    const uint32_t *par = d.parent[pc];
    const uint32_t nnodes = d.ntiles * kNodeSlots;
    for (size_t i = blockIdx.x * (size_t)256 + threadIdx.x; i < n; i += (size_t)gridDim.x * 256) {
        const uint32_t l = d.labels[i];
        if (l & 0x80000000u) {
            uint32_t node = l & 0x7FFFFFFFu;
            node = node < nnodes ? node : 0u;
            uint32_t r = par[node];
            r = r < nnodes ? r : 0u;
            d.labels[i] = d.key[r];
        }
    }
}

// =====================================================================
// k_roots: new spin of every cross-tile cluster (Sec. 2.4) and the cluster
// statistics of the workgroup's tiles -> group partial.
// =====================================================================
// RB: nodes a lane takes at once (see below).  AG: the group partial is
// written with agent-scope stores, for a fold in the same launch.
template <uint32_t RB, bool AG = false>
__device__ __forceinline__ void roots_body(const Dev &d, const uint32_t group) {
    __shared__ uint32_t s_hist[33];
    __shared__ uint32_t s_cnt[kMaxQ];  // Potts value populations of the group's tiles
    __shared__ uint64_t s_red[4][5];
    if (threadIdx.x < 33u) s_hist[threadIdx.x] = 0u;
    if (threadIdx.x < (uint32_t)kMaxQ) s_cnt[threadIdx.x] = 0u;
    const uint64_t tsw = *d.tdev;
    const uint32_t t = (uint32_t)tsw, pc = (uint32_t)(tsw & 1u);
    const uint32_t *par = d.parent[pc];
    const uint32_t lane = threadIdx.x & 63u, wv = threadIdx.x >> 6;
    const uint32_t g0 = group * (uint32_t)kGroupTiles;
    uint64_t n = 0, mx = 0, sq = 0;
    int64_t e = 0, m = 0;
    // the nodes of the wavefront's four tiles g0 + wv + 4q, one after the other
    uint32_t nkq[4];
#pragma unroll
    for (uint32_t q = 0; q < 4u; ++q) {
        const uint32_t tile = g0 + wv + 4u * q;
        const uint32_t v = nk_either(d, pc, min(tile, d.ntiles - 1u));
        nkq[q] = tile < d.ntiles ? min(v, 252u) : 0u;
    }
    const uint32_t pre1 = nkq[0], pre2 = pre1 + nkq[1], pre3 = pre2 + nkq[2], tot = pre3 + nkq[3];
    __syncthreads();  // s_hist and s_cnt cleared
    // every node (flattened: its parent is its root) stores its cluster's
    // new spin, drawn from the cluster's smallest site (the root's key).  A
    // lane takes up to RB nodes at once and issues all their parent loads,
    // then all their key and size loads, so that the wavefront waits on two
    // rounds of loads per batch rather than on two for every node: launches
    // of a few workgroups per CU wait on those rounds; full ones hide them
    // behind other wavefronts and run faster with RB = 1 (fewer registers).
    constexpr uint32_t kRootBatch = RB;
    for (uint32_t m0 = 0; 64u * m0 < tot; m0 += kRootBatch) {
        uint32_t nd[kRootBatch], rt[kRootBatch], rk[kRootBatch], sz[kRootBatch];
#pragma unroll
        for (uint32_t j = 0; j < kRootBatch; ++j) {
            const uint32_t i = lane + 64u * (m0 + j);
            const uint32_t q = (uint32_t)(i >= pre1) + (uint32_t)(i >= pre2) + (uint32_t)(i >= pre3);
            const uint32_t base = q == 0u ? 0u : q == 1u ? pre1 : q == 2u ? pre2 : pre3;
            nd[j] = i < tot ? (g0 + wv + 4u * q) * kNodeSlots + (i - base) : kEmpty;
        }
#pragma unroll
        for (uint32_t j = 0; j < kRootBatch; ++j) rt[j] = nd[j] != kEmpty ? par[nd[j]] : 0u;
#pragma unroll
        for (uint32_t j = 0; j < kRootBatch; ++j) {
            rk[j] = nd[j] != kEmpty ? d.key[rt[j]] : 0u;
            sz[j] = nd[j] != kEmpty && rt[j] == nd[j] ? d.nsize[nd[j]] : 0u;
        }
#pragma unroll
        for (uint32_t j = 0; j < kRootBatch; ++j) {
            if (64u * (m0 + j) >= tot) break;  // wavefront-uniform
            if (nd[j] == kEmpty) continue;
            d.rspin[nd[j]] = d.q ? potts_spin(rk[j], t, d.q, d.seed_lo, d.seed_hi)
                                 : cluster_spin(rk[j], t, d.seed_lo, d.seed_hi);
            if (rt[j] == nd[j]) {
                const uint32_t S = sz[j];
                ++n;
                mx = max(mx, (uint64_t)S);
                sq += (uint64_t)S * S;
                atomicAdd(&s_hist[31 - __clz((int)max(S, 1u))], 1u);
                if (d.dense) atomicAdd(reinterpret_cast<unsigned long long *>(&d.dense[S]), 1ull);
            }
        }
    }
    if (threadIdx.x < (uint32_t)kGroupTiles) {
        const uint32_t tile = g0 + threadIdx.x;
        if (tile < d.ntiles) {
            const int32_t *tp = d.tpart + (size_t)tile * kTilePart;
            e += tp[TP_E];
            m += tp[TP_M];
            n += (uint32_t)tp[TP_N];
            mx = max(mx, (uint64_t)(uint32_t)tp[TP_MAX]);
            sq += (uint32_t)tp[TP_SQ];
            for (int b = 0; b < 12; ++b)
                if (tp[TP_HIST + b]) atomicAdd(&s_hist[b], (uint32_t)tp[TP_HIST + b]);
            if (d.q)
                for (int k = 0; k < kMaxQ; ++k)
                    if (tp[TP_CNT + k]) atomicAdd(&s_cnt[k], (uint32_t)tp[TP_CNT + k]);
        }
    }
#pragma unroll
    for (int o = 32; o > 0; o >>= 1) {
        n += __shfl_xor(n, o, 64);
        mx = max(mx, (uint64_t)__shfl_xor((unsigned long long)mx, o, 64));
        sq += __shfl_xor(sq, o, 64);
        e += __shfl_xor(e, o, 64);
        m += __shfl_xor(m, o, 64);
    }
    if (lane == 0u) {
        s_red[wv][0] = n;
        s_red[wv][1] = mx;
        s_red[wv][2] = sq;
        s_red[wv][3] = (uint64_t)e;
        s_red[wv][4] = (uint64_t)m;
    }
    __syncthreads();
    uint64_t *gp = d.gpart + (size_t)group * kGroupPart;
    auto put = [&](int f, uint64_t v) {
        if constexpr (AG)
            __hip_atomic_store(&gp[f], v, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
        else
            gp[f] = v;
    };
    if (threadIdx.x == 0u) {
        uint64_t a0 = 0, a1 = 0, a2 = 0, a3 = 0, a4 = 0;
        for (int w = 0; w < 4; ++w) {
            a0 += s_red[w][0];
            a1 = max(a1, s_red[w][1]);
            a2 += s_red[w][2];
            a3 += s_red[w][3];
            a4 += s_red[w][4];
        }
        put(GP_N, a0);
        put(GP_MAX, a1);
        put(GP_SQ, a2);
        put(GP_E, a3);
        put(GP_M, a4);
    }
    if (threadIdx.x < 33u) put(GP_HIST + (int)threadIdx.x, s_hist[threadIdx.x]);
    if (threadIdx.x < (uint32_t)kMaxQ) put(GP_CNT + (int)threadIdx.x, s_cnt[threadIdx.x]);
}


// =====================================================================
// k_record: fold group partials (mode 0, end of a sweep) or tile partials
// (mode 1, end of k_resolve) into the record ring; the last workgroup to
// finish writes the record and clears the accumulator.
// =====================================================================
// Folds partials [begin, end) into the workgroup's LDS accumulator.  Group
// partials (mode 0): thread t sums field t % 64 over every fourth partial,
// so each accumulator word takes four LDS atomics.  Tile partials (mode 1,
// energy and magnetisation only): per-thread sums, reduced per wavefront.
constexpr uint32_t kRecordGroups = 64;   // group partials per k_record workgroup
constexpr uint32_t kRecordTiles = 2048;  // tile partials per k_record workgroup

// AG: the group partials were written in the same launch (agent-scope
// stores), so they are read with agent-scope loads.
template <bool AG = false>
__device__ __forceinline__ void record_fold(const Dev &d, uint32_t begin, uint32_t end, int mode, uint64_t *s_acc) {
    const uint32_t tid = threadIdx.x;
    unsigned long long *a = reinterpret_cast<unsigned long long *>(s_acc);
    if (mode != 1) {
        const uint32_t f = tid & 63u, sub = tid >> 6;
        if (f < (uint32_t)GP_END) {
            // four partials per round, their loads issued together (0 is
            // the identity of both the sums and the maximum)
            uint64_t v = 0;
            for (uint32_t item = begin + sub; item < end; item += 16u) {
                uint64_t x[4];
#pragma unroll
                for (uint32_t u = 0; u < 4u; ++u) {
                    const uint32_t it = item + 4u * u;
                    const uint64_t *src = &d.gpart[(size_t)min(it, end - 1u) * kGroupPart + f];
                    const uint64_t y = AG ? __hip_atomic_load(src, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT) : *src;
                    x[u] = it < end ? y : 0u;
                }
#pragma unroll
                for (uint32_t u = 0; u < 4u; ++u) v = f == (uint32_t)GP_MAX ? max(v, x[u]) : v + x[u];
            }
            if (f == (uint32_t)GP_MAX)
                atomicMax(&a[f], (unsigned long long)v);
            else if (v)
                atomicAdd(&a[f], (unsigned long long)v);
        }
    } else {
        int64_t e = 0, m = 0;
        uint32_t c[kMaxQ] = {0u, 0u, 0u, 0u, 0u, 0u, 0u, 0u};
        for (uint32_t item = begin + tid; item < end; item += 256u) {
            const int32_t *tp = d.tpart + (size_t)item * kTilePart;
            e += tp[TP_E];
            m += tp[TP_M];
            if (d.q)
                for (int k = 0; k < kMaxQ; ++k) c[k] += (uint32_t)tp[TP_CNT + k];
        }
#pragma unroll
        for (int o = 32; o > 0; o >>= 1) {
            e += __shfl_xor(e, o, 64);
            m += __shfl_xor(m, o, 64);
        }
        if ((tid & 63u) == 0u) {
            atomicAdd(&a[GP_E], (unsigned long long)e);
            atomicAdd(&a[GP_M], (unsigned long long)m);
        }
        if (d.q)
            for (int k = 0; k < kMaxQ; ++k)
                if (c[k]) atomicAdd(&a[GP_CNT + k], (unsigned long long)c[k]);
    }
}

// Writes the totals in s_acc.  Mode 0 (end of a tile-pipeline sweep): the
// record of sweep t = *tdev gets the cluster statistics and t advances; the
// energy and magnetisation are those of the configuration sweep t-1 left
// (measured by this sweep's tile kernel), written into record t-1.  Mode 1
// (end of k_resolve): only that energy and magnetisation.  Mode 2 (end of a
// label-equivalence sweep): every field of record t, and t advances.
__device__ __forceinline__ void record_write(const Dev &d, const uint64_t *s_acc, int mode) {
    const uint32_t tid = threadIdx.x;
    const uint64_t tsw = *d.tdev;
    if (mode != 1) {
        sw_obs *rec = &d.ring[tsw % d.ring_cap];
        if (tid == 0u) {
            rec->sweep = tsw;
            rec->n_clusters = s_acc[GP_N];
            rec->max_cluster = s_acc[GP_MAX];
            rec->sum_sq_sizes = s_acc[GP_SQ];
        }
        if (tid < 33u) rec->hist_log2[tid] = s_acc[GP_HIST + tid];
    }
    const bool own = mode == 2;
    if (tid == 0u && (own || tsw >= 1u)) {
        sw_obs *rec = &d.ring[(own ? tsw : tsw - 1u) % d.ring_cap];
        const int64_t e = (int64_t)s_acc[GP_E];
        rec->e_sum = e;
        rec->energy = -d.J * (double)e;
        int64_t m = (int64_t)s_acc[GP_M];
        if (d.q) {  // Potts: population of the most populated value
            m = 0;
            for (uint32_t k = 0; k < d.q; ++k) m = max(m, (int64_t)s_acc[GP_CNT + k]);
        }
        rec->m_sum = m;
    }
    __syncthreads();  // every thread has read the sweep index
    if (tid == 0u) {
        if (mode != 1) *d.tdev = tsw + 1u;
        __threadfence();
    }
}

__global__ __launch_bounds__(256) void k_record(Dev d, uint32_t nitems, int mode) {
    __shared__ uint64_t s_acc[GP_END];
    __shared__ int s_last;
    const uint32_t tid = threadIdx.x;
    if (tid < (uint32_t)GP_END) s_acc[tid] = 0u;
    __syncthreads();
    const uint32_t per = mode != 1 ? kRecordGroups : kRecordTiles;
    const uint32_t begin = blockIdx.x * per;
    record_fold(d, begin, min(begin + per, nitems), mode, s_acc);
    __syncthreads();
    unsigned long long *acc = reinterpret_cast<unsigned long long *>(d.acc);
    if (tid < (uint32_t)GP_END && s_acc[tid] != 0u) {
        if (tid == (uint32_t)GP_MAX)
            atomicMax(&acc[tid], (unsigned long long)s_acc[tid]);
        else
            atomicAdd(&acc[tid], (unsigned long long)s_acc[tid]);
    }
    // device-scope atomics are performed where every XCD sees them: once each
    // wavefront has seen its own complete, the count may go up, and the last
    // workgroup reads the totals with device-scope loads (no cache fences)
    __builtin_amdgcn_s_waitcnt(0);
    __syncthreads();
    if (tid == 0u) {
        const unsigned long long old = atomicAdd(&acc[ACC_COUNT], 1ull);
        s_last = (old == (unsigned long long)gridDim.x - 1ull) ? 1 : 0;
    }
    __syncthreads();
    if (!s_last) return;
    // the last workgroup: take the totals (one field per thread) and clear
    // the accumulator for the next fold
    if (tid < (uint32_t)GP_END) {
        s_acc[tid] = __hip_atomic_load(&acc[tid], __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
        __hip_atomic_store(&acc[tid], 0ull, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
    }
    if (tid == (uint32_t)GP_END)
        __hip_atomic_store(&acc[ACC_COUNT], 0ull, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
    __syncthreads();
    record_write(d, s_acc, mode);
}

// Batched record of the tile partials at the end of a resolve (mode 1): one
// workgroup per replica folds all of that replica's partials itself, so no
// cross-workgroup accumulator is needed (the group partials of a sweep are
// folded by k_roots_b).
__global__ __launch_bounds__(256) void k_record_b(const Dev *devs, const uint32_t *rmap, int mode) {
    __shared__ uint64_t s_acc[GP_END];
    const Dev &d = devs[rmap[blockIdx.x]];
    const uint32_t tid = threadIdx.x;
    if (tid < (uint32_t)GP_END) s_acc[tid] = 0u;
    __syncthreads();
    record_fold(d, 0u, mode != 1 ? d.ngroups : d.ntiles, mode, s_acc);
    __syncthreads();
    record_write(d, s_acc, mode);
}

// k_roots, and the record folded into the same launch: the last workgroup of
// a lattice to write its group partial folds them all and writes the record
// (one launch less per sweep).  The partials go out as agent-scope stores
// and every wavefront waits for its own to complete before its workgroup
// counts itself in, so the last one reads them all with agent-scope loads
// (no cache fences).  Used where a lattice has few groups (the fold is one
// workgroup's work) and for every replica of a batch.
template <uint32_t RB>
__device__ __forceinline__ void roots_fold_body(const Dev &d, const uint32_t group) {
    __shared__ uint64_t s_acc[GP_END];
    __shared__ int s_last;
    roots_body<RB, true>(d, group);
    __builtin_amdgcn_s_waitcnt(0);
    __syncthreads();
    unsigned long long *acc = reinterpret_cast<unsigned long long *>(d.acc);
    if (threadIdx.x == 0u) {
        const unsigned long long old = atomicAdd(&acc[ACC_COUNT], 1ull);
        s_last = old == (unsigned long long)d.ngroups - 1ull ? 1 : 0;
    }
    if (threadIdx.x < (uint32_t)GP_END) s_acc[threadIdx.x] = 0u;
    __syncthreads();
    if (!s_last) return;
    if (threadIdx.x == 0u) __hip_atomic_store(&acc[ACC_COUNT], 0ull, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
    record_fold<true>(d, 0u, d.ngroups, 0, s_acc);
    __syncthreads();
    record_write(d, s_acc, 0);
}

// Plain lattices: up to kRootsFold groups the record is folded by k_roots;
// from kRootsWide groups (32768 tiles) on, a lane takes one node at a time.
constexpr uint32_t kRootsFold = 64;
constexpr uint32_t kRootsWide = 2048;

template <uint32_t RB>
__global__ __launch_bounds__(256) void k_roots(Dev d) { roots_body<RB>(d, blockIdx.x); }

__global__ __launch_bounds__(256) void k_roots_fold(Dev d) { roots_fold_body<4>(d, blockIdx.x); }

__global__ __launch_bounds__(256) void k_roots_b(const Dev *devs, const uint32_t *map) {
    const uint32_t e = map[blockIdx.x];
    roots_fold_body<4>(devs[e >> kMapShift], e & kMapMask);
}

// =====================================================================
// k_smerge_b: the whole cross-tile part of a sweep of one small replica
// (at most kSmallTiles tiles) in one workgroup, in LDS: unions across every
// tile edge (Sec. 2.3), every node to its root with the cluster's size and
// smallest site, the new spin of every node's cluster (Sec. 2.4), the
// cluster statistics and the record (Sec. 2.5) -- the work of k_ulocal,
// k_union, k_flatten, k_roots and k_record for that replica, same results.
// Nodes are numbered locally in global-index order (tile by tile), so the
// root of a set is its node with the smallest global index, as in the
// global merge.
// =====================================================================
constexpr uint32_t kSmallNodes = kSmallTiles * 252u;

__device__ __forceinline__ void smerge_body(const Dev &d) {
    __shared__ uint32_t s_par[kSmallNodes];
    __shared__ uint32_t s_key[kSmallNodes];
    __shared__ uint32_t s_sz[kSmallNodes];
    __shared__ uint32_t s_off[kSmallTiles + 1];
    __shared__ unsigned long long s_acc[GP_END];
    const uint32_t tid = threadIdx.x, lane = tid & 63u;
    const uint64_t tsw = *d.tdev;
    const uint32_t t = (uint32_t)tsw, pc = (uint32_t)(tsw & 1u);
    const uint32_t nt = d.ntiles, tw = d.tw, ntx = d.ntx;
    uint32_t *par = d.parent[pc];
    if (tid == 0u) {
        uint32_t o = 0u;
        for (uint32_t T = 0; T < nt; ++T) {
            s_off[T] = o;
            o += min(d.nk[pc][T], tw == 64u ? 252u : 124u);
        }
        s_off[nt] = o;
    }
    if (tid < (uint32_t)GP_END) s_acc[tid] = 0ull;
    __syncthreads();
    const uint32_t n = s_off[nt];
    // local node i: tile T (s_off[T] <= i < s_off[T + 1]), slot i - s_off[T]
    auto tile_of = [&](uint32_t i) {
        uint32_t T = 0u;
        while (T + 1u < nt && s_off[T + 1u] <= i) ++T;
        return T;
    };
    for (uint32_t i = tid; i < n; i += 256u) {
        const uint32_t T = tile_of(i), node = T * kNodeSlots + (i - s_off[T]);
        s_par[i] = i;
        s_key[i] = d.key[node];
        s_sz[i] = d.nsize[node];
    }
    __syncthreads();
    // bonds across every tile edge, E and N, periodic; a run of bonds along
    // an edge between the same two nodes needs one union
    for (uint32_t f0 = 0; f0 < nt * 2u * tw; f0 += 256u) {
        const uint32_t f = f0 + tid;
        const bool in = f < nt * 2u * tw;
        const uint32_t T = in ? f / (2u * tw) : 0u, dir = (f / tw) & 1u, i = f % tw;
        const uint32_t tx = T % ntx, ty = T / ntx;
        const uint32_t nb = dir == 0u ? ty * ntx + (tx + 1u == ntx ? 0u : tx + 1u)
                                      : (ty + 1u == ntx ? 0u : ty + 1u) * ntx + tx;
        const uint8_t *ea = d.edge + (size_t)T * 4u * tw, *eb = d.edge + (size_t)nb * 4u * tw;
        const bool has = in && ((d.xb[2u * T + dir] >> i) & 1u);
        const uint32_t a = s_off[T] + (dir == 0u ? ea[1u * tw + i] : ea[3u * tw + i]);
        const uint32_t b = s_off[nb] + (dir == 0u ? eb[0u * tw + i] : eb[2u * tw + i]);
        const uint32_t pa = __shfl_up(a, 1, 64), pb = __shfl_up(b, 1, 64);
        const int ph = __shfl_up((int)has, 1, 64);
        const bool dup = i > 0u && lane > 0u && ph && pa == a && pb == b;
        if (has && !dup) lds_union(s_par, a, b);
    }
    __syncthreads();
    // every node to its root; sizes and smallest sites into the roots
    for (uint32_t i = tid; i < n; i += 256u) {
        const uint32_t r = lds_root(s_par, i);
        if (r != i) {
            atomicMin(&s_key[r], s_key[i]);
            atomicAdd(&s_sz[r], s_sz[i]);
            const uint32_t T = tile_of(i), Tr = tile_of(r);
            par[T * kNodeSlots + (i - s_off[T])] = Tr * kNodeSlots + (r - s_off[Tr]);
        }
    }
    __syncthreads();
    // the new spin of every node's cluster, drawn from its smallest site;
    // statistics of the cross-tile clusters
    uint64_t cn = 0, cmx = 0, csq = 0;
    for (uint32_t i = tid; i < n; i += 256u) {
        const uint32_t r = lds_root(s_par, i), T = tile_of(i);
        const uint32_t rkey = s_key[r];
        d.rspin[T * kNodeSlots + (i - s_off[T])] =
            d.q ? potts_spin(rkey, t, d.q, d.seed_lo, d.seed_hi) : cluster_spin(rkey, t, d.seed_lo, d.seed_hi);
        if (r == i) {
            const uint32_t S = s_sz[i];
            ++cn;
            cmx = max(cmx, (uint64_t)S);
            csq += (uint64_t)S * S;
            atomicAdd(&s_acc[GP_HIST + 31 - __clz((int)max(S, 1u))], 1ull);
            if (d.dense) atomicAdd(reinterpret_cast<unsigned long long *>(&d.dense[S]), 1ull);
        }
    }
    // the tile partials (interior clusters, energy and magnetisation of the
    // incoming configuration, Potts populations)
    int64_t ce = 0, cm = 0;
    for (uint32_t T = tid; T < nt; T += 256u) {
        const int32_t *tp = d.tpart + (size_t)T * kTilePart;
        ce += tp[TP_E];
        cm += tp[TP_M];
        cn += (uint32_t)tp[TP_N];
        cmx = max(cmx, (uint64_t)(uint32_t)tp[TP_MAX]);
        csq += (uint32_t)tp[TP_SQ];
        for (int b = 0; b < 12; ++b)
            if (tp[TP_HIST + b]) atomicAdd(&s_acc[GP_HIST + b], (unsigned long long)(uint32_t)tp[TP_HIST + b]);
        if (d.q)
            for (int k = 0; k < kMaxQ; ++k)
                if (tp[TP_CNT + k]) atomicAdd(&s_acc[GP_CNT + k], (unsigned long long)(uint32_t)tp[TP_CNT + k]);
    }
#pragma unroll
    for (int o = 32; o > 0; o >>= 1) {
        cn += __shfl_xor(cn, o, 64);
        cmx = max(cmx, (uint64_t)__shfl_xor((unsigned long long)cmx, o, 64));
        csq += __shfl_xor(csq, o, 64);
        ce += __shfl_xor(ce, o, 64);
        cm += __shfl_xor(cm, o, 64);
    }
    if (lane == 0u) {
        atomicAdd(&s_acc[GP_N], (unsigned long long)cn);
        atomicMax(&s_acc[GP_MAX], (unsigned long long)cmx);
        atomicAdd(&s_acc[GP_SQ], (unsigned long long)csq);
        atomicAdd(&s_acc[GP_E], (unsigned long long)ce);
        atomicAdd(&s_acc[GP_M], (unsigned long long)cm);
    }
    __syncthreads();
    record_write(d, reinterpret_cast<const uint64_t *>(s_acc), 0);
}

__global__ __launch_bounds__(256) void k_smerge_b(const Dev *devs, const uint32_t *smap) {
    smerge_body(devs[smap[blockIdx.x]]);
}

// =====================================================================
// k_resolve: replace node codes by final spins in place and measure the
// configuration (runs once at the end of every sw_sweep call).
// =====================================================================
template <int TW, bool POTTS = false>
__device__ __forceinline__ void resolve_body(const Dev &d, const uint32_t tile) {
    constexpr int NT = TW * TW / 16;
    constexpr uint32_t RPT = TW / 16;
    constexpr int NWAVE = (NT + 63) / 64;
    constexpr int NPL = POTTS ? 3 : 1;
    constexpr uint32_t EW = (TW + 31) / 32;
    using Row = typename RowOf<TW>::T;
    __shared__ uint8_t s_tab[256];
    __shared__ Row s_up[NPL * (TW + 1)];
    __shared__ uint32_t s_eup[NPL * EW];
    __shared__ int32_t s_red[NWAVE][POTTS ? 6 : 2];

    const uint32_t tid = threadIdx.x;
    const uint32_t L = d.L, ntx = d.ntx;
    const uint32_t tx = tile % ntx, ty = tile / ntx;
    const uint64_t tsw = *d.tdev;
    const uint32_t pc = (uint32_t)(tsw & 1u), pp = pc ^ 1u;
    int8_t *sp = d.spins[pc];
    const uint32_t ly = tid / RPT, seg = tid % RPT, x0 = seg * 16u;
    const uint32_t gy = ty * TW + ly, gx0 = tx * TW + x0;
    const uint32_t east = ty * ntx + (tx + 1u == ntx ? 0u : tx + 1u);
    const uint32_t north = (ty + 1u == ntx ? 0u : ty + 1u) * ntx + tx;

    const uint4 v = *reinterpret_cast<const uint4 *>(sp + (size_t)gy * L + gx0);
    uint4 vn = make_uint4(0u, 0u, 0u, 0u);
    if (ly == TW - 1) {
        const uint32_t gyn = (gy + 1u == L) ? 0u : gy + 1u;
        vn = *reinterpret_cast<const uint4 *>(sp + (size_t)gyn * L + gx0);
    }
    uint32_t ve = 0;
    if (seg == RPT - 1) {
        const uint32_t gxe = (gx0 + 16u == L) ? 0u : gx0 + 16u;
        ve = (uint8_t)sp[(size_t)gy * L + gxe];
    }
    load_table<TW, POTTS>(d, tile, pp, s_tab, tid);
    if (tid < NPL * EW) s_eup[tid] = 0u;
    __syncthreads();
    uint32_t up = 0u, pl[3] = {0u, 0u, 0u};
    if constexpr (POTTS) {
        decode16_potts(v, s_tab, pl);
#pragma unroll
        for (int b = 0; b < 3; ++b) reinterpret_cast<uint16_t *>(s_up + b * (TW + 1))[ly * RPT + seg] = (uint16_t)pl[b];
        if (ly == TW - 1) {
            uint32_t pn[3];
            decode16_potts_remote<TW>(vn, north, d.rspin, pn);
#pragma unroll
            for (int b = 0; b < 3; ++b)
                reinterpret_cast<uint16_t *>(s_up + b * (TW + 1))[TW * RPT + seg] = (uint16_t)pn[b];
        }
        if (seg == RPT - 1) {
            const uint32_t ev = potts_byte<TW>(ve, east, d.rspin);
#pragma unroll
            for (uint32_t b = 0; b < 3u; ++b)
                if ((ev >> b) & 1u) atomicOr(&s_eup[b * EW + (ly >> 5)], 1u << (ly & 31u));
        }
    } else {
        up = decode16<TW>(v, s_tab);
        reinterpret_cast<uint16_t *>(s_up)[ly * RPT + seg] = (uint16_t)up;
        if (ly == TW - 1) {
            const uint32_t upn = decode16_remote(vn, north, d.rspin);
            reinterpret_cast<uint16_t *>(s_up)[TW * RPT + seg] = (uint16_t)upn;
        }
        if (seg == RPT - 1) {
            if (resolve_byte(ve, east, d.rspin) > 0) atomicOr(&s_eup[ly >> 5], 1u << (ly & 31u));
        }
    }
    __syncthreads();
    int32_t e_part, m_part = 0;
    uint32_t cpk[4] = {0u, 0u, 0u, 0u};
    uint32_t out[4] = {0u, 0u, 0u, 0u};
    if constexpr (POTTS) {
        uint32_t dE = 0u, dN = 0u;
#pragma unroll
        for (int b = 0; b < 3; ++b) {
            const Row rowv = s_up[b * (TW + 1) + ly];
            const uint32_t pN = (uint32_t)(s_up[b * (TW + 1) + ly + 1] >> x0) & 0xFFFFu;
            const uint32_t ebit = (s_eup[b * EW + (ly >> 5)] >> (ly & 31u)) & 1u;
            const uint32_t nxt = (x0 + 16u < (uint32_t)TW) ? ((uint32_t)(rowv >> (x0 + 16u)) & 1u) : ebit;
            dE |= pl[b] ^ ((pl[b] >> 1) | (nxt << 15));
            dN |= pl[b] ^ pN;
        }
        e_part = __popc(~dE & 0xFFFFu) + __popc(~dN & 0xFFFFu);
        potts_counts(pl, cpk);
#pragma unroll
        for (int q = 0; q < 16; ++q) {
            const uint32_t x = ((pl[0] >> q) & 1u) | (((pl[1] >> q) & 1u) << 1) | (((pl[2] >> q) & 1u) << 2);
            out[q >> 2] |= x << (8 * (q & 3));
        }
    } else {
        const Row rowv = s_up[ly];
        const uint32_t upN = (uint32_t)(s_up[ly + 1] >> x0) & 0xFFFFu;
        const uint32_t ebit = (s_eup[ly >> 5] >> (ly & 31u)) & 1u;
        const uint32_t nxt = (x0 + 16u < (uint32_t)TW) ? ((uint32_t)(rowv >> (x0 + 16u)) & 1u) : ebit;
        const uint32_t upE = (up >> 1) | (nxt << 15);
        e_part = 2 * (__popc(~(up ^ upE) & 0xFFFFu) + __popc(~(up ^ upN) & 0xFFFFu)) - 32;
        m_part = 2 * __popc(up) - 16;
#pragma unroll
        for (int q = 0; q < 16; ++q) out[q >> 2] |= (((up >> q) & 1u) ? 0x01u : 0xFFu) << (8 * (q & 3));
    }
    *reinterpret_cast<uint4 *>(sp + (size_t)gy * L + gx0) = make_uint4(out[0], out[1], out[2], out[3]);
#pragma unroll
    for (int o = 32; o > 0; o >>= 1) {
        e_part += __shfl_xor(e_part, o, 64);
        m_part += __shfl_xor(m_part, o, 64);
        if constexpr (POTTS) {
#pragma unroll
            for (int i = 0; i < 4; ++i) cpk[i] += __shfl_xor(cpk[i], o, 64);
        }
    }
    if ((tid & 63u) == 0u) {
        s_red[tid >> 6][0] = e_part;
        s_red[tid >> 6][1] = m_part;
        if constexpr (POTTS) {
#pragma unroll
            for (int i = 0; i < 4; ++i) s_red[tid >> 6][2 + i] = (int32_t)cpk[i];
        }
    }
    __syncthreads();
    if (tid == 0u) {
        int32_t e = 0, m = 0;
        for (int w = 0; w < NWAVE; ++w) {
            e += s_red[w][0];
            m += s_red[w][1];
        }
        int32_t *tp = d.tpart + (size_t)tile * kTilePart;
        tp[TP_E] = e;
        tp[TP_M] = m;
        if constexpr (POTTS) {
            for (int k = 0; k < 8; ++k) {
                int32_t c = 0;
                for (int w = 0; w < NWAVE; ++w) c += (int32_t)(((uint32_t)s_red[w][2 + k / 2] >> (16 * (k & 1))) & 0xFFFFu);
                tp[TP_CNT + k] = c;
            }
        }
    }
}

template <int TW, bool POTTS = false>
__global__ __launch_bounds__(TW *TW / 16) void k_resolve(Dev d) {
    resolve_body<TW, POTTS>(d, tile_of_block(blockIdx.x, d.ntiles));
}

template <int TW, bool POTTS = false>
__global__ __launch_bounds__(TW *TW / 16) void k_resolve_b(const Dev *devs, const uint32_t *map) {
    const uint32_t e = map[tile_of_block(blockIdx.x, gridDim.x)];
    resolve_body<TW, POTTS>(devs[e >> kMapShift], e & kMapMask);
}

// Initial spins (Fig. 1): hot = bit 0 of word 0 of Philox({s, 0, 2, 0}),
// cold = all +1; for the Potts model hot = floor(w q / 2^32) of that word,
// cold = all 0.  16 sites per thread.
__global__ __launch_bounds__(256) void k_init(Dev d, int cold) {
    const size_t n16 = d.nsite / 16u;
    const uint32_t pc = (uint32_t)(*d.tdev & 1u);
    int8_t *sp = d.spins[pc];
    const uint32_t fill = d.q ? 0u : 0x01010101u;
    for (size_t i = blockIdx.x * (size_t)256 + threadIdx.x; i < n16; i += (size_t)gridDim.x * 256) {
        uint32_t out[4] = {fill, fill, fill, fill};
        if (!cold) {
#pragma unroll
            for (int q = 0; q < 16; ++q) {
                uint32_t w0 = (uint32_t)(i * 16u + q), w1 = 0u, w2 = 2u, w3 = 0u;
                philox10(w0, w1, w2, w3, d.seed_lo, d.seed_hi);
                if (d.q)
                    out[q >> 2] |= (uint32_t)(((uint64_t)w0 * d.q) >> 32) << (8 * (q & 3));
                else if (w0 & 1u)
                    out[q >> 2] |= 0xFFu << (8 * (q & 3));
            }
        }
        *reinterpret_cast<uint4 *>(sp + i * 16u) = make_uint4(out[0], out[1], out[2], out[3]);
    }
}

__global__ __launch_bounds__(256) void k_zero_u64(uint64_t *p, size_t n) {
    for (size_t i = blockIdx.x * (size_t)256 + threadIdx.x; i < n; i += (size_t)gridDim.x * 256) p[i] = 0u;
}

inline uint32_t grid_for(size_t n, uint32_t per_block, uint32_t cap) {
    size_t g = (n + per_block - 1) / per_block;
    if (g < 1) g = 1;
    if (g > cap) g = cap;
    return (uint32_t)g;
}

}  // namespace

hipError_t launch_init(const Dev &d, int cold, hipStream_t s) {
    const size_t n16 = d.nsite / 16u;
    k_init<<<grid_for(n16, 256, 65536), 256, 0, s>>>(d, cold);
    return hipGetLastError();
}

hipError_t launch_stage(const Dev &d, int stage, hipStream_t s) {
    const size_t n = d.nsite;
    if (d.le_grid || d.brick) {  // labels in global memory (label equivalence, cubic bricks)
        if (stage == 0 && d.dense) k_zero_u64<<<grid_for(n + 1, 256, 65536), 256, 0, s>>>(d.dense, n + 1);
        if (stage != 4) {
            const hipError_t e = hipGetLastError();
            return e != hipSuccess ? e : launch_le_stage(d, stage, s);
        }
        k_record<<<(d.ngroups + kRecordGroups - 1) / kRecordGroups, 256, 0, s>>>(d, d.ngroups, 2);
        return hipGetLastError();
    }
    switch (stage) {
    case 0:  // bonds + tile-local clusters
        if (d.dense) k_zero_u64<<<grid_for(n + 1, 256, 65536), 256, 0, s>>>(d.dense, n + 1);
        if (d.q && d.tw == 64)
            k_tile<64, true><<<d.ntiles, 256, 0, s>>>(d);
        else if (d.q)
            k_tile<32, true><<<d.ntiles, 64, 0, s>>>(d);
        else if (d.tw == 64)
            k_tile<64><<<d.ntiles, 256, 0, s>>>(d);
        else
            k_tile<32><<<d.ntiles, 64, 0, s>>>(d);
        break;
    case 1: {  // cross-tile unions: inside groups of tiles, then between groups
        const uint32_t ngx = (d.ntx + kUG - 1u) / kUG, nwaves = 2u * ngx * d.ntx;
        if (d.tw == 64) {
            k_ulocal<64><<<ngx * ngx, 256, 0, s>>>(d);
            k_union<64><<<(nwaves + 3u) / 4u, 256, 0, s>>>(d);
        } else {
            k_ulocal<32><<<ngx * ngx, 256, 0, s>>>(d);
            k_union<32><<<(nwaves + 3u) / 4u, 256, 0, s>>>(d);
        }
        break;
    }
    case 2:  // flatten + cluster sizes
        k_flatten<kGroupTiles><<<d.ngroups, 256, 0, s>>>(d);
        if (d.labels) k_relabel<<<grid_for(n, 256, 65536), 256, 0, s>>>(d);
        break;
    case 3:  // spins of cross-tile clusters, statistics (and the record, on few groups)
        if (d.ngroups >= kRootsWide)
            k_roots<1><<<d.ngroups, 256, 0, s>>>(d);
        else if (d.ngroups > kRootsFold)
            k_roots<4><<<d.ngroups, 256, 0, s>>>(d);
        else
            k_roots_fold<<<d.ngroups, 256, 0, s>>>(d);
        break;
    case 4:  // record (folded by k_roots on few groups)
        if (d.ngroups > kRootsFold)
            k_record<<<(d.ngroups + kRecordGroups - 1) / kRecordGroups, 256, 0, s>>>(d, d.ngroups, 0);
        break;
    default:
        return hipErrorInvalidValue;
    }
    return hipGetLastError();
}

hipError_t launch_sweep(const Dev &d, hipStream_t s) {
    for (int stage = 0; stage < kStages; ++stage) {
        const hipError_t e = launch_stage(d, stage, s);
        if (e != hipSuccess) return e;
    }
    return hipSuccess;
}

hipError_t launch_resolve(const Dev &d, hipStream_t s) {
    if (d.le_grid || d.brick) return hipSuccess;  // those paths write final spins and full records
    if (d.q && d.tw == 64)
        k_resolve<64, true><<<d.ntiles, 256, 0, s>>>(d);
    else if (d.q)
        k_resolve<32, true><<<d.ntiles, 64, 0, s>>>(d);
    else if (d.tw == 64)
        k_resolve<64><<<d.ntiles, 256, 0, s>>>(d);
    else
        k_resolve<32><<<d.ntiles, 64, 0, s>>>(d);
    k_record<<<(d.ntiles + kRecordTiles - 1) / kRecordTiles, 256, 0, s>>>(d, d.ntiles, 1);
    return hipGetLastError();
}

hipError_t launch_batch_smerge(const BatchDev &b, hipStream_t s) {
    if (b.nsmall == 0) return hipSuccess;
    k_smerge_b<<<b.nsmall, 256, 0, s>>>(b.devs, b.smap);
    return hipGetLastError();
}

hipError_t launch_batch_stage(const BatchDev &b, int stage, hipStream_t s) {
    if (b.nall == 0) return hipSuccess;
    if (b.n == 0 && stage != 0) return hipSuccess;  // stages 1..4: replicas of the global merge
    switch (stage) {
    case 0:
        if (b.potts && b.tw == 64)
            k_tile_b<64, true><<<b.ntiles, 256, 0, s>>>(b.devs, b.tmap);
        else if (b.potts)
            k_tile_b<32, true><<<b.ntiles, 64, 0, s>>>(b.devs, b.tmap);
        else if (b.tw == 64)
            k_tile_b<64><<<b.ntiles, 256, 0, s>>>(b.devs, b.tmap);
        else
            k_tile_b<32><<<b.ntiles, 64, 0, s>>>(b.devs, b.tmap);
        break;
    case 1:
        if (b.tw == 64) {
            k_ulocal_b<64><<<b.nugroups, 256, 0, s>>>(b.devs, b.umap);
            k_union_b<64><<<b.nwmap / 4, 256, 0, s>>>(b.devs, b.wmap, b.nwE);
        } else {
            k_ulocal_b<32><<<b.nugroups, 256, 0, s>>>(b.devs, b.umap);
            k_union_b<32><<<b.nwmap / 4, 256, 0, s>>>(b.devs, b.wmap, b.nwE);
        }
        break;
    case 2:
        k_flatten_b<<<b.ngroups, 256, 0, s>>>(b.devs, b.gmap);
        break;
    case 3:  // and the records
        k_roots_b<<<b.ngroups, 256, 0, s>>>(b.devs, b.gmap);
        break;
    case 4:  // (folded by k_roots_b)
        break;
    default:
        return hipErrorInvalidValue;
    }
    return hipGetLastError();
}

hipError_t launch_batch_sweep(const BatchDev &b, hipStream_t s) {
    for (int stage = 0; stage < kStages; ++stage) {
        hipError_t e = launch_batch_stage(b, stage, s);
        if (e == hipSuccess && stage == 0) e = launch_batch_smerge(b, s);
        if (e != hipSuccess) return e;
    }
    return hipSuccess;
}

hipError_t launch_batch_resolve(const BatchDev &b, hipStream_t s) {
    if (b.nall == 0) return hipSuccess;
    if (b.potts && b.tw == 64)
        k_resolve_b<64, true><<<b.ntiles, 256, 0, s>>>(b.devs, b.tmap);
    else if (b.potts)
        k_resolve_b<32, true><<<b.ntiles, 64, 0, s>>>(b.devs, b.tmap);
    else if (b.tw == 64)
        k_resolve_b<64><<<b.ntiles, 256, 0, s>>>(b.devs, b.tmap);
    else
        k_resolve_b<32><<<b.ntiles, 64, 0, s>>>(b.devs, b.tmap);
    k_record_b<<<b.nall, 256, 0, s>>>(b.devs, b.amap, 1);
    return hipGetLastError();
}

}  // namespace swmi
