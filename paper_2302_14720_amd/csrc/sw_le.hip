// sw_le.hip -- the paper's own cluster formation (Sec. 2.3): label
// equivalence over the whole lattice in global memory, after Kalentev et
// al.  Every site starts labelled with its own index; a scan pass lets each
// site point the entry of its label at the smallest label among its bonded
// neighbours (an atomic minimum), an analysis pass makes each site follow
// its chain of references to the end and take that label, and the two
// repeat until a scan changes nothing.  The result is the smallest site of
// each cluster, the same canonical labels as the tile pipeline, so a sweep
// gives the same bits.  The paper drove the passes from a dynamic-
// parallelism kernel (Sec. 5); here one cooperative (persistent) kernel runs
// all passes with grid-wide barriers and polls a device-side flag.  This
// path exists to compare the paper's design with the tile pipeline.
#include <hip/hip_cooperative_groups.h>

#include "sw_internal.h"
#include "sw_philox.h"
#include "sw_uf.h"

namespace swmi {
namespace {

namespace cg = cooperative_groups;

constexpr uint32_t kLeMaxPasses = 1u << 16;

__device__ __forceinline__ uint32_t ld(const uint32_t *p) {
    return __hip_atomic_load(p, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
}
__device__ __forceinline__ void st(uint32_t *p, uint32_t v) {
    __hip_atomic_store(p, v, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
}

// Bonds (Sec. 2.1) of every site to E and N: two sites per Philox call,
// words 2(s&1)+d of counter {s>>1, t, 0, 0}.
__global__ __launch_bounds__(256) void k_le_bond(Dev d) {
    const uint32_t L = d.L;
    const size_t pairs = (size_t)L * L / 2u;
    const uint32_t t = (uint32_t)*d.tdev;
    const int8_t *sp = d.spins[0];
    for (size_t p = blockIdx.x * (size_t)256 + threadIdx.x; p < pairs; p += (size_t)gridDim.x * 256) {
        const size_t s0 = 2u * p;
        const uint32_t y = (uint32_t)(s0 / L), x = (uint32_t)(s0 % L);
        const size_t row = (size_t)y * L, up = (size_t)(y + 1u == L ? 0u : y + 1u) * L;
        const int8_t a = sp[s0], b = sp[s0 + 1u];
        const int8_t ea = b, eb = sp[row + (x + 2u == L ? 0u : x + 2u)];
        const int8_t na = sp[up + x], nb = sp[up + x + 1u];
        uint32_t w0 = (uint32_t)p, w1 = t, w2 = 0u, w3 = 0u;
        philox10(w0, w1, w2, w3, d.seed_lo, d.seed_hi);
        const uint32_t T = d.T;
        const uint32_t m0 = (uint32_t)(a == ea && w0 < T) | ((uint32_t)(a == na && w1 < T) << 1);
        const uint32_t m1 = (uint32_t)(b == eb && w2 < T) | ((uint32_t)(b == nb && w3 < T) << 1);
        *reinterpret_cast<uint16_t *>(d.le_mask + s0) = (uint16_t)(m0 | (m1 << 8));
    }
}

// Bonds of the simple cubic lattice to +x, +y and +z: one Philox call per
// site, words 0, 1, 2 of counter {s, t, 4, 0}.
__global__ __launch_bounds__(256) void k_le_bond3(Dev d) {
    const uint32_t L = d.L, LL = L * L;
    const uint32_t N = (uint32_t)d.nsite;
    const uint32_t t = (uint32_t)*d.tdev;
    const int8_t *sp = d.spins[0];
    // N <= 1616^3, so s + the grid stride stays below 2^32
    for (uint32_t s = blockIdx.x * 256u + threadIdx.x; s < N; s += gridDim.x * 256u) {
        const uint32_t x = s % L, yz = s / L, y = yz % L, z = yz / L;
        const int8_t a = sp[s];
        const int8_t e = sp[x + 1u == L ? s - x : s + 1u];
        const int8_t n = sp[y + 1u == L ? s - y * L : s + L];
        const int8_t u = sp[z + 1u == L ? s - z * LL : s + LL];
        uint32_t w0 = s, w1 = t, w2 = 4u, w3 = 0u;
        philox10(w0, w1, w2, w3, d.seed_lo, d.seed_hi);
        const uint32_t T = d.T;
        d.le_mask[s] = (uint8_t)((uint32_t)(a == e && w0 < T) | ((uint32_t)(a == n && w1 < T) << 1) |
                                 ((uint32_t)(a == u && w2 < T) << 2));
    }
}

// All labelling passes in one cooperative launch.  Flags rotate over three
// words: pass k raises flag k mod 3, every thread reads it after the pass's
// last barrier, and flag (k+1) mod 3 is cleared at the start of pass k --
// its last readers finished with pass k-2.  Every thread therefore takes
// the same exit decision, and the pass cap bounds the loop.
// DIMS = 3: the scan looks at the six neighbours of the simple cubic lattice
// (bit 2 of a site's mask is its bond to +z).
template <int DIMS>
__global__ __launch_bounds__(256) void k_le_label(Dev d) {
    cg::grid_group g = cg::this_grid();
    const uint32_t L = d.L;
    const size_t N = d.nsite;
    const size_t gid = blockIdx.x * (size_t)256 + threadIdx.x, stride = (size_t)gridDim.x * 256;
    uint32_t *lab = d.labels;
    const uint8_t *mk = d.le_mask;
    uint32_t *ctl = d.le_ctl;
    for (size_t i = gid; i < N; i += stride) st(&lab[i], (uint32_t)i);
    if (gid == 0) {
        st(&ctl[0], 0u);
        st(&ctl[1], 0u);
        st(&ctl[2], 0u);
    }
    g.sync();
    uint32_t pass = 0;
    while (true) {
        const uint32_t f = pass % 3u;
        if (gid == 0) st(&ctl[(pass + 1u) % 3u], 0u);
        // scan: the entry of my label points at the smallest bonded label
        bool changed = false;
        for (size_t i = gid; i < N; i += stride) {
            const uint32_t l = ld(&lab[i]);
            uint32_t m = l;
            if (DIMS == 2) {
                const uint32_t y = (uint32_t)(i / L), x = (uint32_t)(i % L);
                const size_t row = (size_t)y * L;
                const size_t e = row + (x + 1u == L ? 0u : x + 1u), w = row + (x == 0u ? L - 1u : x - 1u);
                const size_t n = (size_t)(y + 1u == L ? 0u : y + 1u) * L + x;
                const size_t s = (size_t)(y == 0u ? L - 1u : y - 1u) * L + x;
                const uint32_t bm = mk[i], bw = mk[w], bs = mk[s];
                if (bm & 1u) m = min(m, ld(&lab[e]));
                if (bm & 2u) m = min(m, ld(&lab[n]));
                if (bw & 1u) m = min(m, ld(&lab[w]));
                if (bs & 2u) m = min(m, ld(&lab[s]));
            } else {
                const uint32_t si = (uint32_t)i, LL = L * L;
                const uint32_t x = si % L, yz = si / L, y = yz % L, z = yz / L;
                const uint32_t e = x + 1u == L ? si - x : si + 1u, w = x == 0u ? si + (L - 1u) : si - 1u;
                const uint32_t n = y + 1u == L ? si - y * L : si + L, s = y == 0u ? si + (L - 1u) * L : si - L;
                const uint32_t u = z + 1u == L ? si - z * LL : si + LL, dn = z == 0u ? si + (L - 1u) * LL : si - LL;
                const uint32_t bm = mk[si], bw = mk[w], bs = mk[s], bd = mk[dn];
                if (bm & 1u) m = min(m, ld(&lab[e]));
                if (bm & 2u) m = min(m, ld(&lab[n]));
                if (bm & 4u) m = min(m, ld(&lab[u]));
                if (bw & 1u) m = min(m, ld(&lab[w]));
                if (bs & 2u) m = min(m, ld(&lab[s]));
                if (bd & 4u) m = min(m, ld(&lab[dn]));
            }
            if (m < l) {
                atomicMin(&lab[l], m);
                changed = true;
            }
        }
        if (changed) st(&ctl[f], 1u);
        g.sync();
        // analysis: follow the chain of references to its end
        for (size_t i = gid; i < N; i += stride) {
            const uint32_t l = ld(&lab[i]);
            if (l == (uint32_t)i) continue;
            uint32_t r = l, q = ld(&lab[r]);
            while (q != r) {
                r = q;
                q = ld(&lab[r]);
            }
            if (r != l) st(&lab[i], r);
        }
        g.sync();
        ++pass;
        if (ld(&ctl[f]) == 0u || pass >= kLeMaxPasses) break;
    }
    if (gid == 0) {
        st(&ctl[LE_PASSES], pass);
        st(&ctl[LE_STATUS], ld(&ctl[(pass - 1u) % 3u]) != 0u ? 1u : 0u);
    }
}

// New spin of every cluster (Sec. 2.4) at its root; sizes cleared.  For the
// Ising model a wavefront's 64 sites lie in one 128-site block, so the
// Philox call of the cluster-spin rule is the same for all its lanes.
__global__ __launch_bounds__(256) void k_le_roots(Dev d) {
    const size_t N = d.nsite;
    const uint32_t t = (uint32_t)*d.tdev;
    for (size_t i = blockIdx.x * (size_t)256 + threadIdx.x; i < N; i += (size_t)gridDim.x * 256) {
        if (d.labels[i] != (uint32_t)i) continue;
        d.le_rsp[i] = d.q ? potts_spin((uint32_t)i, t, d.q, d.seed_lo, d.seed_hi)
                          : cluster_spin((uint32_t)i, t, d.seed_lo, d.seed_hi);
        d.le_cnt[i] = 0u;
    }
}

// Every site takes its cluster's spin; cluster sizes are counted per
// workgroup in an LDS hash (kLeChunk sites each), then added to the roots.
constexpr uint32_t kLeHash = 2048;
__global__ __launch_bounds__(256) void k_le_flip(Dev d) {
    __shared__ uint32_t hk[kLeHash];
    __shared__ uint32_t hv[kLeHash];
    for (uint32_t i = threadIdx.x; i < kLeHash; i += 256u) {
        hk[i] = 0xFFFFFFFFu;
        hv[i] = 0u;
    }
    __syncthreads();
    const size_t N = d.nsite;
    const size_t b0 = (size_t)blockIdx.x * kLeChunk, b1 = min(b0 + kLeChunk, N);
    int8_t *sp = d.spins[0];
    for (size_t i = b0 + threadIdx.x; i < b1; i += 256u) {
        const uint32_t r = d.labels[i];
        sp[i] = d.le_rsp[r];
        uint32_t h = (r * 2654435761u) >> 21;
        bool placed = false;
        for (int probe = 0; probe < 64 && !placed; ++probe) {
            uint32_t cur = __hip_atomic_load(&hk[h], __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_WORKGROUP);
            if (cur == 0xFFFFFFFFu) {
                const uint32_t old = atomicCAS(&hk[h], 0xFFFFFFFFu, r);
                cur = old == 0xFFFFFFFFu ? r : old;
            }
            if (cur == r) {
                atomicAdd(&hv[h], 1u);
                placed = true;
            }
            h = (h + 1u) & (kLeHash - 1u);
        }
        if (!placed) atomicAdd(&d.le_cnt[r], 1u);
    }
    __syncthreads();
    for (uint32_t i = threadIdx.x; i < kLeHash; i += 256u)
        if (hk[i] != 0xFFFFFFFFu) atomicAdd(&d.le_cnt[hk[i]], hv[i]);
}

// Statistics of the new configuration and of the sweep's clusters, per
// workgroup of kLeChunk sites, into the group partials (GP_* layout).
__global__ __launch_bounds__(256) void k_le_stats(Dev d) {
    __shared__ unsigned long long s_acc[GP_END];
    for (uint32_t i = threadIdx.x; i < (uint32_t)GP_END; i += 256u) s_acc[i] = 0ull;
    __syncthreads();
    const uint32_t L = d.L;
    const size_t N = d.nsite;
    const size_t b0 = (size_t)blockIdx.x * kLeChunk, b1 = min(b0 + kLeChunk, N);
    const int8_t *sp = d.spins[0];
    const bool cubic = d.dims == 3u;
    int64_t e = 0, m = 0;
    uint64_t n = 0, mx = 0, sq = 0;
    __shared__ unsigned int s_cnt[kMaxQ];
    if (threadIdx.x < (uint32_t)kMaxQ) s_cnt[threadIdx.x] = 0u;
    __syncthreads();
    for (size_t i = b0 + threadIdx.x; i < b1; i += 256u) {
        const int32_t si = sp[i];
        int32_t se, sn, su = 0;
        if (cubic) {  // +x, +y, +z neighbours of site (z L + y) L + x
            const uint32_t s = (uint32_t)i, LL = L * L;
            const uint32_t x = s % L, yz = s / L, y = yz % L, z = yz / L;
            se = sp[x + 1u == L ? s - x : s + 1u];
            sn = sp[y + 1u == L ? s - y * L : s + L];
            su = sp[z + 1u == L ? s - z * LL : s + LL];
        } else {
            const uint32_t y = (uint32_t)(i / L), x = (uint32_t)(i % L);
            se = sp[(size_t)y * L + (x + 1u == L ? 0u : x + 1u)];
            sn = sp[(size_t)(y + 1u == L ? 0u : y + 1u) * L + x];
        }
        if (d.q) {  // Potts: equal pairs and value populations
            e += (si == se) + (si == sn) + (cubic && si == su);
            atomicAdd(&s_cnt[(uint32_t)si < (uint32_t)kMaxQ ? si : 0], 1u);
        } else {
            e += si * se + si * sn + si * su;
            m += si;
        }
        if (d.labels[i] == (uint32_t)i) {
            const uint32_t S = d.le_cnt[i];
            ++n;
            mx = max(mx, (uint64_t)S);
            sq += (uint64_t)S * S;
            atomicAdd(&s_acc[GP_HIST + (31 - __clz((int)max(S, 1u)))], 1ull);
            if (d.dense) atomicAdd(reinterpret_cast<unsigned long long *>(&d.dense[S]), 1ull);
        }
    }
#pragma unroll
    for (int o = 32; o > 0; o >>= 1) {
        e += __shfl_xor(e, o, 64);
        m += __shfl_xor(m, o, 64);
        n += __shfl_xor(n, o, 64);
        mx = max(mx, (uint64_t)__shfl_xor((unsigned long long)mx, o, 64));
        sq += __shfl_xor(sq, o, 64);
    }
    if ((threadIdx.x & 63u) == 0u) {
        atomicAdd(&s_acc[GP_E], (unsigned long long)e);
        atomicAdd(&s_acc[GP_M], (unsigned long long)m);
        atomicAdd(&s_acc[GP_N], (unsigned long long)n);
        atomicMax(&s_acc[GP_MAX], (unsigned long long)mx);
        atomicAdd(&s_acc[GP_SQ], (unsigned long long)sq);
    }
    __syncthreads();
    if (threadIdx.x < (uint32_t)kMaxQ) s_acc[GP_CNT + threadIdx.x] = s_cnt[threadIdx.x];
    __syncthreads();
    uint64_t *gp = d.gpart + (size_t)blockIdx.x * kGroupPart;
    for (uint32_t i = threadIdx.x; i < (uint32_t)GP_END; i += 256u) gp[i] = s_acc[i];
}

// =====================================================================
// Simple cubic lattice on 16^3 bricks (the default for dims = 3): bonds and
// the connected components of the bonds inside each brick in LDS; then one
// union-find in global memory over the bonds that cross brick faces, with
// the label array itself as the parent array; then every label is pointed
// at its root.  Roots are always the smallest index (sw_uf.h), so the final
// label of a site is the smallest site of its cluster, as on the other
// paths.  Cluster sizes are summed from the brick-local component sizes
// (one atomic per local component); the statistics and the record are
// those of the label-equivalence path.
// =====================================================================
__device__ __forceinline__ uint32_t byte_of(const uint4 &v, uint32_t j) {
    const uint32_t w = j < 4u ? v.x : j < 8u ? v.y : j < 12u ? v.z : v.w;
    return (w >> (8u * (j & 3u))) & 0xFFu;
}

// One workgroup per brick; thread (y, z) owns the brick's x-row of 16 sites
// at (y, z).  A site's brick-local index (z * 16 + y) * 16 + x orders the
// sites of a brick as their global indices do, so the local root (smallest
// local index) is the component's smallest site.
__global__ __launch_bounds__(256) void k_brick3(Dev d) {
    __shared__ uint32_t s_par[kBrick * kBrick * kBrick];
    __shared__ uint32_t s_ex[kBrick * kBrick];
    const uint32_t L = d.L, nb = L / kBrick;
    const uint32_t b = blockIdx.x;
    const uint32_t bx = b % nb, by = (b / nb) % nb, bz = b / (nb * nb);
    const uint32_t tid = threadIdx.x, y = tid & 15u, z = tid >> 4;
    const uint32_t gx0 = bx * kBrick, gy = by * kBrick + y, gz = bz * kBrick + z;
    const uint32_t gyn = gy + 1u == L ? 0u : gy + 1u, gzn = gz + 1u == L ? 0u : gz + 1u;
    const uint32_t s0 = (gz * L + gy) * L + gx0;  // N < 2^32
    const int8_t *sp = d.spins[0];
    const uint4 v = *reinterpret_cast<const uint4 *>(sp + s0);
    const uint4 vy = *reinterpret_cast<const uint4 *>(sp + (gz * L + gyn) * L + gx0);
    const uint4 vz = *reinterpret_cast<const uint4 *>(sp + (gzn * L + gy) * L + gx0);
    const uint32_t ex = (uint8_t)sp[(gz * L + gy) * L + (gx0 + kBrick == L ? 0u : gx0 + kBrick)];
    const uint32_t t = (uint32_t)*d.tdev, T = d.T;

    // bonds (Sec. 2.1): one Philox call per site, words 0, 1, 2 of counter
    // {s, t, 4, 0} for +x, +y, +z; bonds join equal spins (Ising) or values
    uint32_t EX = 0u, EY = 0u, EZ = 0u, mk[4] = {0u, 0u, 0u, 0u};
#pragma unroll
    for (uint32_t j = 0; j < 16u; ++j) {
        uint32_t w0 = s0 + j, w1 = t, w2 = 4u, w3 = 0u;
        philox10(w0, w1, w2, w3, d.seed_lo, d.seed_hi);
        const uint32_t a = byte_of(v, j), e = j < 15u ? byte_of(v, j + 1u) : ex;
        const uint32_t n = byte_of(vy, j), u = byte_of(vz, j);
        const uint32_t bxj = (uint32_t)(a == e && w0 < T), byj = (uint32_t)(a == n && w1 < T);
        const uint32_t bzj = (uint32_t)(a == u && w2 < T);
        EX |= bxj << j;
        EY |= byj << j;
        EZ |= bzj << j;
        mk[j >> 2] |= (bxj | (byj << 1) | (bzj << 2)) << (8u * (j & 3u));
    }

    // brick-local clusters: every site points at the start of its x-run,
    // then the +y and +z bonds inside the brick join runs (one union per
    // group of consecutive bonds between the same two runs)
    const uint32_t EXi = EX & 0x7FFFu;
    const uint32_t base = tid * kBrick;
    s_ex[tid] = EXi;
    {
        uint32_t cur = base;
#pragma unroll
        for (uint32_t j = 0; j < 16u; ++j) {
            if (j == 0u || !((EXi >> (j - 1u)) & 1u)) cur = base + j;
            s_par[base + j] = cur;
        }
    }
    __syncthreads();
    if (y < 15u) {
        const uint32_t E1 = s_ex[tid + 1u];
        uint32_t R = EY & ~((EY << 1) & (EXi << 1) & (E1 << 1)) & 0xFFFFu;
        while (R) {
            const uint32_t j = (uint32_t)__ffs((int)R) - 1u;
            R &= R - 1u;
            lds_union(s_par, base + j, base + j + kBrick);
        }
    }
    if (z < 15u) {
        const uint32_t E1 = s_ex[tid + kBrick];
        uint32_t R = EZ & ~((EZ << 1) & (EXi << 1) & (E1 << 1)) & 0xFFFFu;
        while (R) {
            const uint32_t j = (uint32_t)__ffs((int)R) - 1u;
            R &= R - 1u;
            lds_union(s_par, base + j, base + j + kBrick * kBrick);
        }
    }
    __syncthreads();
    // local component sizes in the high halves of the roots' words: one add
    // per x-run (a run lies in one component)
    uint32_t rt[16];
#pragma unroll
    for (uint32_t j = 0; j < 16u; ++j) rt[j] = lds_root(s_par, base + j);
#pragma unroll
    for (uint32_t j = 0; j < 16u; ++j) {
        if (j != 0u && ((EXi >> (j - 1u)) & 1u)) continue;
        const uint32_t rest = (~EXi >> j) | 0x8000u;  // bit i set: the run ends at j + i
        const uint32_t len = (uint32_t)__ffs((int)rest);
        atomicAdd(&s_par[rt[j]], len << 16);
    }
    __syncthreads();
    // labels = the global index of the local root; a local root (bit 3 of
    // its mask byte) keeps its component size in le_cnt
    uint32_t lab[16];
#pragma unroll
    for (uint32_t j = 0; j < 16u; ++j) {
        const uint32_t r = rt[j];
        lab[j] = ((bz * kBrick + (r >> 8)) * L + by * kBrick + ((r >> 4) & 15u)) * L + bx * kBrick + (r & 15u);
        if (r == base + j) {
            mk[j >> 2] |= 8u << (8u * (j & 3u));
            d.le_cnt[s0 + j] = lds_load(&s_par[r]) >> 16;
        }
    }
    *reinterpret_cast<uint4 *>(d.le_mask + s0) = make_uint4(mk[0], mk[1], mk[2], mk[3]);
    uint32_t *bf = d.bface + (size_t)b * 512u;
    bf[tid] = ((EX >> 15) & 1u) ? lab[15] : kMapNone;
    bf[256u + tid] = lab[0];
    uint4 *lp = reinterpret_cast<uint4 *>(d.labels + s0);
    lp[0] = make_uint4(lab[0], lab[1], lab[2], lab[3]);
    lp[1] = make_uint4(lab[4], lab[5], lab[6], lab[7]);
    lp[2] = make_uint4(lab[8], lab[9], lab[10], lab[11]);
    lp[3] = make_uint4(lab[12], lab[13], lab[14], lab[15]);
}

// Bonds across brick faces: one thread per site of the +x, +y and +z faces
// of every brick (768 per brick); a bonded site joins the set of its
// neighbour in the next brick.  Neighbouring face sites whose bonds join
// the same two brick-local roots need one union.
__global__ __launch_bounds__(256) void k_bunion3(Dev d) {
    const uint32_t L = d.L, nb = L / kBrick, LL = L * L;
    const uint32_t gid = blockIdx.x * 256u + threadIdx.x;
    const uint32_t brick = gid / 768u, r = gid % 768u, f = r >> 8, i = r & 255u;
    const uint32_t bx = brick % nb, by = (brick / nb) % nb, bz = brick / (nb * nb);
    const uint32_t lx = f == 0u ? 15u : (i & 15u);
    const uint32_t ly = f == 1u ? 15u : (f == 0u ? (i & 15u) : (i >> 4));
    const uint32_t lz = f == 2u ? 15u : (i >> 4);
    const uint32_t gx = bx * kBrick + lx, gy = by * kBrick + ly, gz = bz * kBrick + lz;
    const uint32_t s = (gz * L + gy) * L + gx;
    const uint32_t nbr = f == 0u ? (gx + 1u == L ? s - gx : s + 1u)
                       : f == 1u ? (gy + 1u == L ? s - gy * L : s + L)
                                 : (gz + 1u == L ? s - gz * LL : s + LL);
    bool has;
    uint32_t a, c;
    if (f == 0u) {  // x faces: their sites are L apart, so read the brick's face records
        const uint32_t nbk = (bz * nb + by) * nb + (bx + 1u == nb ? 0u : bx + 1u);
        a = d.bface[(size_t)brick * 512u + i];
        has = a != kMapNone;
        c = has ? d.bface[(size_t)nbk * 512u + 256u + i] : 0u;
        if (!has) a = 0u;
        (void)nbr;
    } else {
        has = ((uint32_t)d.le_mask[s] >> f) & 1u;
        a = has ? g_load(&d.labels[s]) : 0u;
        c = has ? g_load(&d.labels[nbr]) : 0u;
    }
    // the previous lane holds the previous site of the same face row
    const uint32_t pa = __shfl_up(a, 1, 64), pc = __shfl_up(c, 1, 64);
    const int ph = __shfl_up((int)has, 1, 64);
    const bool dup = (threadIdx.x & 63u) != 0u && (i & 15u) != 0u && ph && pa == a && pc == c;
    if (has && !dup) g_union(d.labels, a, c);
}

// Every local root points at its final root (reads only ancestors, so
// concurrent rewrites by other threads are harmless); other sites still
// point at their local root.
__global__ __launch_bounds__(256) void k_bflat3(Dev d) {
    const uint32_t N = (uint32_t)d.nsite;
    for (uint32_t s = blockIdx.x * 256u + threadIdx.x; s < N; s += gridDim.x * 256u) {
        if (!(d.le_mask[s] & 8u)) continue;
        const uint32_t l = g_load(&d.labels[s]);
        uint32_t r = l;
        while (true) {
            const uint32_t p = g_load(&d.labels[r]);
            if (p == r) break;
            r = p;
        }
        if (r != l) g_store(&d.labels[s], r);
    }
}

// Final labels, new spins (Sec. 2.4) and cluster sizes.  Every site draws
// its cluster's spin from the cluster's root itself (the draw depends only
// on the root, so no pass has to wait for the roots' draws), and every
// local root that is not its cluster's root adds its component size to the
// root's.
__global__ __launch_bounds__(256) void k_brelabel3(Dev d) {
    const uint32_t N = (uint32_t)d.nsite, t = (uint32_t)*d.tdev;
    int8_t *sp = d.spins[0];
    for (uint32_t s = blockIdx.x * 256u + threadIdx.x; s < N; s += gridDim.x * 256u) {
        const bool local_root = (d.le_mask[s] & 8u) != 0u;
        const uint32_t l = d.labels[s];
        const uint32_t r = local_root ? l : d.labels[l];
        if (!local_root) d.labels[s] = r;
        sp[s] = d.q ? potts_spin(r, t, d.q, d.seed_lo, d.seed_hi) : cluster_spin(r, t, d.seed_lo, d.seed_hi);
        if (local_root && r != s) atomicAdd(&d.le_cnt[r], d.le_cnt[s]);
    }
}

// Brick path: the statistics of the new configuration and of the sweep's
// clusters (those of k_le_stats, in the same group partials: workgroup b
// covers sites [kLeChunk b, kLeChunk (b + 1)), one x-segment of 16 sites
// per thread, whose spins and labels come in 16-byte loads; L is a multiple
// of 16, so a segment lies in one row and L^3 is a multiple of kLeChunk).
// Potts value populations are counted in registers, 16 bits per value, and
// added once per wavefront.
__global__ __launch_bounds__(256) void k_bstats3(Dev d) {
    static_assert(kLeChunk == 256u * 16u, "one 16-site segment per thread");
    __shared__ unsigned long long s_acc[GP_END];
    __shared__ unsigned int s_cnt[kMaxQ];
    for (uint32_t i = threadIdx.x; i < (uint32_t)GP_END; i += 256u) s_acc[i] = 0ull;
    if (threadIdx.x < (uint32_t)kMaxQ) s_cnt[threadIdx.x] = 0u;
    __syncthreads();
    const uint32_t L = d.L, LL = L * L;
    const uint32_t s0 = blockIdx.x * kLeChunk + 16u * threadIdx.x;
    const uint32_t x0 = s0 % L, yz = s0 / L, y = yz % L, z = yz / L;
    const int8_t *sp = d.spins[0];
    // +x, +y, +z neighbours of the segment (periodic)
    const uint4 v = *reinterpret_cast<const uint4 *>(sp + s0);
    const uint4 vy = *reinterpret_cast<const uint4 *>(sp + (y + 1u == L ? s0 - y * L : s0 + L));
    const uint4 vz = *reinterpret_cast<const uint4 *>(sp + (z + 1u == L ? s0 - z * LL : s0 + LL));
    const uint32_t vx = (uint8_t)sp[x0 + 16u == L ? s0 - x0 : s0 + 16u];
    const uint4 *lp = reinterpret_cast<const uint4 *>(d.labels + s0);
    const uint4 a0 = lp[0], a1 = lp[1], a2 = lp[2], a3 = lp[3];
    const uint32_t lab[16] = {a0.x, a0.y, a0.z, a0.w, a1.x, a1.y, a1.z, a1.w,
                              a2.x, a2.y, a2.z, a2.w, a3.x, a3.y, a3.z, a3.w};
    int32_t e = 0, m = 0;
    uint64_t c01 = 0u, c23 = 0u;  // Potts populations of values 0-3 and 4-7
#pragma unroll
    for (uint32_t j = 0; j < 16u; ++j) {
        const uint32_t bs = byte_of(v, j), bx = j < 15u ? byte_of(v, j + 1u) : vx;
        const uint32_t by = byte_of(vy, j), bz = byte_of(vz, j);
        if (d.q) {
            e += (int32_t)(bs == bx) + (int32_t)(bs == by) + (int32_t)(bs == bz);
            const uint64_t one = 1ull << (16u * (bs & 3u));
            if (bs < 4u)
                c01 += one;
            else
                c23 += one;
        } else {
            const int32_t si = (int8_t)bs;
            e += si * ((int8_t)bx + (int8_t)by + (int8_t)bz);
            m += si;
        }
    }
    uint64_t n = 0, mx = 0, sq = 0;
#pragma unroll
    for (uint32_t j = 0; j < 16u; ++j) {
        if (lab[j] != s0 + j) continue;
        const uint32_t S = d.le_cnt[s0 + j];
        ++n;
        mx = max(mx, (uint64_t)S);
        sq += (uint64_t)S * S;
        atomicAdd(&s_acc[GP_HIST + (31 - __clz((int)max(S, 1u)))], 1ull);
        if (d.dense) atomicAdd(reinterpret_cast<unsigned long long *>(&d.dense[S]), 1ull);
    }
    int64_t e64 = e, m64 = m;
#pragma unroll
    for (int o = 32; o > 0; o >>= 1) {
        e64 += __shfl_xor(e64, o, 64);
        m64 += __shfl_xor(m64, o, 64);
        n += __shfl_xor(n, o, 64);
        mx = max(mx, (uint64_t)__shfl_xor((unsigned long long)mx, o, 64));
        sq += __shfl_xor(sq, o, 64);
        c01 += __shfl_xor(c01, o, 64);  // at most 64 * 16 per value: no carry between fields
        c23 += __shfl_xor(c23, o, 64);
    }
    if ((threadIdx.x & 63u) == 0u) {
        atomicAdd(&s_acc[GP_E], (unsigned long long)e64);
        atomicAdd(&s_acc[GP_M], (unsigned long long)m64);
        atomicAdd(&s_acc[GP_N], (unsigned long long)n);
        atomicMax(&s_acc[GP_MAX], (unsigned long long)mx);
        atomicAdd(&s_acc[GP_SQ], (unsigned long long)sq);
        if (d.q) {
#pragma unroll
            for (uint32_t k = 0; k < 4u; ++k) {
                atomicAdd(&s_cnt[k], (unsigned int)((c01 >> (16u * k)) & 0xFFFFu));
                if (4u + k < (uint32_t)kMaxQ) atomicAdd(&s_cnt[4u + k], (unsigned int)((c23 >> (16u * k)) & 0xFFFFu));
            }
        }
    }
    __syncthreads();
    if (threadIdx.x < (uint32_t)kMaxQ) s_acc[GP_CNT + threadIdx.x] = s_cnt[threadIdx.x];
    __syncthreads();
    uint64_t *gp = d.gpart + (size_t)blockIdx.x * kGroupPart;
    for (uint32_t i = threadIdx.x; i < (uint32_t)GP_END; i += 256u) gp[i] = s_acc[i];
}

inline uint32_t grid_cap(size_t n, uint32_t per, uint32_t cap) {
    size_t g = (n + per - 1) / per;
    return (uint32_t)(g < 1 ? 1 : g > cap ? cap : g);
}

}  // namespace

uint32_t le_grid_size(uint32_t dims) {
    int dev = 0, cus = 0, per = 0;
    if (hipGetDevice(&dev) != hipSuccess) return 0;
    if (hipDeviceGetAttribute(&cus, hipDeviceAttributeMultiprocessorCount, dev) != hipSuccess) return 0;
    const hipError_t e = dims == 3u ? hipOccupancyMaxActiveBlocksPerMultiprocessor(&per, k_le_label<3>, 256, 0)
                                   : hipOccupancyMaxActiveBlocksPerMultiprocessor(&per, k_le_label<2>, 256, 0);
    if (e != hipSuccess) return 0;
    return (uint32_t)(cus * (per < 1 ? 1 : per));
}

hipError_t launch_le_stage(const Dev &d, int stage, hipStream_t s) {
    const size_t N = d.nsite;
    const bool cubic = d.dims == 3u;
    switch (stage) {
    case 0:
        if (d.brick) {
            const uint32_t nb = d.L / kBrick;
            k_brick3<<<nb * nb * nb, 256, 0, s>>>(d);
        } else if (cubic) {
            k_le_bond3<<<grid_cap(N, 256, 65536), 256, 0, s>>>(d);
        } else {
            k_le_bond<<<grid_cap(N / 2, 256, 65536), 256, 0, s>>>(d);
        }
        break;
    case 1: {
        if (d.brick) {
            const uint32_t nb = d.L / kBrick;
            k_bunion3<<<nb * nb * nb * 3u, 256, 0, s>>>(d);
            k_bflat3<<<grid_cap(N, 256, 65536), 256, 0, s>>>(d);
            break;
        }
        Dev dd = d;
        void *args[] = {&dd};
        const void *fn = cubic ? reinterpret_cast<const void *>(k_le_label<3>)
                               : reinterpret_cast<const void *>(k_le_label<2>);
        return hipLaunchCooperativeKernel(fn, dim3(d.le_grid), dim3(256), args, 0, s);
    }
    case 2:
        if (d.brick) {
            k_brelabel3<<<grid_cap(N, 256, 65536), 256, 0, s>>>(d);
            break;
        }
        k_le_roots<<<grid_cap(N, 256, 65536), 256, 0, s>>>(d);
        k_le_flip<<<(uint32_t)((N + kLeChunk - 1) / kLeChunk), 256, 0, s>>>(d);
        break;
    case 3:
        if (d.brick) {
            k_bstats3<<<(uint32_t)(N / kLeChunk), 256, 0, s>>>(d);
            break;
        }
        k_le_stats<<<(uint32_t)((N + kLeChunk - 1) / kLeChunk), 256, 0, s>>>(d);
        break;
    default:
        return hipErrorInvalidValue;
    }
    return hipGetLastError();
}

}  // namespace swmi
