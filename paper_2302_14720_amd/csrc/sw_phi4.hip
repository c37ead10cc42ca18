// sw_phi4.hip -- the O(4) phi^4 theory on the L^4 periodic lattice (paper
// Sec. 3): one multicluster update of the Wolff embedding per sweep.
//
// Fields are unit 4-vectors (the self-coupling lambda and the radial update
// are not given in the paper; with |phi| = 1, the lambda -> infinity limit,
// the cluster update alone samples exp(2 kappa sum_<xy> phi_x . phi_y)).
// A sweep t:
//   k_phi_proj    every site projects its field on the sweep's random
//                 direction r (unnormalised, drawn by 4-ball rejection from
//                 Philox({k, t, 5, 0})); parents and sizes are reset
//   k_phi_bond    link (x, mu) is bonded (eq. 2) iff a = ((p_x p_y) 4 kappa)
//                 / (r . r) > 0 and its word (word mu of Philox({x, t, 7, 0}))
//                 times 2^-32 is below 1 - E(a); bonded sites are joined by
//                 the lock-free union-find of sw_uf.h (smaller index is root)
//   k_phi_flat    every site points at its root (the cluster's smallest
//                 site); sizes are counted at the roots
//   k_phi_flip    a cluster whose root's Philox bit ({root >> 7, t, 6, 0},
//                 bit root mod 128) is set is reflected (eq. 3):
//                 phi -= ((2 p_x) / (r . r)) r
//   k_phi_record  exact int64 sums of rint(2^32 phi_x . phi_y) over links and
//                 of rint(2^32 phi_x^a), cluster statistics at the roots;
//                 the last workgroup writes the sweep's record
// Every floating-point value is an IEEE double produced by one correctly
// rounded operation at a time in the order written (no multiply-add is
// contracted in this file), so the results are a function of the inputs
// alone, and equal to any other evaluation in the same order.
#pragma clang fp contract(off)

#include <math.h>
#include <string.h>

#include <algorithm>
#include <cmath>
#include <new>
#include <string>

#include "sw_host.h"
#include "sw_philox.h"
#include "sw_uf.h"

namespace swmi {
namespace {

constexpr int kPhiBlock = 256;
constexpr int kPhiMaxL = 64;
constexpr double kPhiMaxKappa = 4.0;
// accumulator words: e, m[4], n, max, sum_sq, hist[33], completion counter
enum { PA_E = 0, PA_M = 1, PA_N = 5, PA_MAX = 6, PA_SQ = 7, PA_HIST = 8, PA_END = 41, PA_COUNT = 48 };
constexpr int kPhiAccWords = 64;

struct PhiDev {
    double *phi;      // [N][4] fields
    double *proj;     // [N] projection of phi_x on r (unnormalised)
    uint32_t *parent; // [N] union-find parents, then roots (labels)
    uint32_t *csize;  // [N] cluster size at roots
    double *dir;      // [8] r[4], r . r of the current sweep
    uint64_t *acc;    // [kPhiAccWords]
    uint64_t *tdev;   // [0] index of the next sweep
    sw_phi4_obs *ring;
    uint32_t L, N, ring_cap, seed_lo, seed_hi;
    double kappa;
};

__device__ __forceinline__ double phi_uniform(uint32_t w) { return ((double)w + 0.5) * 0x1p-31 - 1.0; }

__device__ __forceinline__ double dot4(double a0, double a1, double a2, double a3, double b0, double b1, double b2,
                                       double b3) {
    return ((a0 * b0 + a1 * b1) + a2 * b2) + a3 * b3;
}

// The sweep's random direction: the first of up to 64 candidates
// (Philox({k, t, 5, 0}) as four uniforms in (-1, 1)) inside the unit ball;
// (1, 0, 0, 0) if none is.  Every thread draws the same sequence.
__device__ __forceinline__ void phi_direction(uint32_t t, uint32_t k0, uint32_t k1, double r[4], double &rr) {
    for (uint32_t k = 0; k < 64u; ++k) {
        uint32_t w0 = k, w1 = t, w2 = 5u, w3 = 0u;
        philox10(w0, w1, w2, w3, k0, k1);
        const double v0 = phi_uniform(w0), v1 = phi_uniform(w1), v2 = phi_uniform(w2), v3 = phi_uniform(w3);
        const double vv = dot4(v0, v1, v2, v3, v0, v1, v2, v3);
        if (vv < 1.0) {
            r[0] = v0;
            r[1] = v1;
            r[2] = v2;
            r[3] = v3;
            rr = vv;
            return;
        }
    }
    r[0] = 1.0;
    r[1] = r[2] = r[3] = 0.0;
    rr = 1.0;
}

// exp(-a) for the bond test: halve a to at most 1/8 (k times), Taylor
// polynomial of degree 13 in Horner form with rounded 1/j, square k times.
__device__ __forceinline__ double phi_expm(double a) {
    double b = a;
    int k = 0;
    while (b > 0.125) {
        b = b * 0.5;
        ++k;
    }
    double q = 1.0;
#pragma unroll
    for (int j = 13; j >= 1; --j) q = 1.0 - (q * b) * (1.0 / (double)j);
    for (int i = 0; i < k; ++i) q = q * q;
    return q;
}

// x + mu-hat on the periodic L^4 lattice (x_0 fastest)
__device__ __forceinline__ uint32_t phi_step(uint32_t x, uint32_t L, uint32_t mu) {
    uint32_t stride = 1u;
    for (uint32_t d = 0; d < mu; ++d) stride *= L;
    const uint32_t c = (x / stride) % L;
    return c + 1u == L ? x - c * stride : x + stride;
}

__global__ __launch_bounds__(kPhiBlock) void k_phi_init(PhiDev d, int cold) {
    const uint32_t x = blockIdx.x * kPhiBlock + threadIdx.x;
    if (x >= d.N) return;
    double f0 = 1.0, f1 = 0.0, f2 = 0.0, f3 = 0.0;
    if (!cold) {
        for (uint32_t k = 0; k < 64u; ++k) {
            uint32_t w0 = x, w1 = k, w2 = 8u, w3 = 0u;
            philox10(w0, w1, w2, w3, d.seed_lo, d.seed_hi);
            const double v0 = phi_uniform(w0), v1 = phi_uniform(w1), v2 = phi_uniform(w2), v3 = phi_uniform(w3);
            const double vv = dot4(v0, v1, v2, v3, v0, v1, v2, v3);
            if (vv < 1.0) {
                const double len = sqrt(vv);
                f0 = v0 / len;
                f1 = v1 / len;
                f2 = v2 / len;
                f3 = v3 / len;
                break;
            }
        }
    }
    double4 *p = reinterpret_cast<double4 *>(d.phi);
    p[x] = make_double4(f0, f1, f2, f3);
}

__global__ __launch_bounds__(kPhiBlock) void k_phi_proj(PhiDev d) {
    const uint32_t x = blockIdx.x * kPhiBlock + threadIdx.x;
    const uint32_t t = (uint32_t)*d.tdev;
    double r[4], rr;
    phi_direction(t, d.seed_lo, d.seed_hi, r, rr);
    if (x == 0u) {
        d.dir[0] = r[0];
        d.dir[1] = r[1];
        d.dir[2] = r[2];
        d.dir[3] = r[3];
        d.dir[4] = rr;
    }
    if (x >= d.N) return;
    const double4 f = reinterpret_cast<const double4 *>(d.phi)[x];
    d.proj[x] = dot4(f.x, f.y, f.z, f.w, r[0], r[1], r[2], r[3]);
    d.parent[x] = x;
    d.csize[x] = 0u;
}

__global__ __launch_bounds__(kPhiBlock) void k_phi_bond(PhiDev d) {
    const uint32_t x = blockIdx.x * kPhiBlock + threadIdx.x;
    if (x >= d.N) return;
    const uint32_t t = (uint32_t)*d.tdev;
    const double rr = d.dir[4];
    const double k4 = 4.0 * d.kappa;
    const double px = d.proj[x];
    uint32_t w[4] = {x, t, 7u, 0u};
    philox10(w[0], w[1], w[2], w[3], d.seed_lo, d.seed_hi);
    uint32_t nb[4];
    bool bond[4];
#pragma unroll
    for (uint32_t mu = 0; mu < 4u; ++mu) {
        nb[mu] = phi_step(x, d.L, mu);
        const double a = ((px * d.proj[nb[mu]]) * k4) / rr;
        bond[mu] = false;
        if (a > 0.0) {
            const double u = (double)w[mu] * 0x1p-32;
            bond[mu] = u < 1.0 - phi_expm(a);
        }
    }
#pragma unroll
    for (uint32_t mu = 0; mu < 4u; ++mu)
        if (bond[mu]) g_union(d.parent, x, nb[mu]);
}

__global__ __launch_bounds__(kPhiBlock) void k_phi_flat(PhiDev d) {
    const uint32_t x = blockIdx.x * kPhiBlock + threadIdx.x;
    const bool valid = x < d.N;
    uint32_t root = 0u;
    if (valid) {
        root = x;
        while (true) {
            const uint32_t p = g_load(&d.parent[root]);
            if (p == root) break;
            root = p;
        }
        if (root != x) g_store(&d.parent[x], root);
    }
    // one atomic per distinct root of the wavefront
    const uint32_t lane = threadIdx.x & 63u;
    bool pending = valid;
    while (true) {
        const uint64_t act = __ballot(pending);
        if (act == 0ull) break;
        const uint32_t leader = (uint32_t)__ffsll((unsigned long long)act) - 1u;
        const uint32_t lr = __shfl(root, (int)leader, 64);
        const bool mine = pending && root == lr;
        const uint64_t same = __ballot(mine);
        if (lane == leader) atomicAdd(&d.csize[lr], (uint32_t)__popcll(same));
        if (mine) pending = false;
    }
}

__global__ __launch_bounds__(kPhiBlock) void k_phi_flip(PhiDev d) {
    const uint32_t x = blockIdx.x * kPhiBlock + threadIdx.x;
    if (x >= d.N) return;
    const uint32_t t = (uint32_t)*d.tdev;
    const uint32_t root = d.parent[x];
    uint32_t w0 = root >> 7, w1 = t, w2 = 6u, w3 = 0u;
    philox10(w0, w1, w2, w3, d.seed_lo, d.seed_hi);
    const uint32_t q = (root >> 5) & 3u;
    const uint32_t w = q == 0 ? w0 : q == 1 ? w1 : q == 2 ? w2 : w3;
    if (((w >> (root & 31u)) & 1u) == 0u) return;
    const double r0 = d.dir[0], r1 = d.dir[1], r2 = d.dir[2], r3 = d.dir[3], rr = d.dir[4];
    double4 *p = reinterpret_cast<double4 *>(d.phi);
    double4 f = p[x];
    const double c = (2.0 * d.proj[x]) / rr;
    f.x = f.x - c * r0;
    f.y = f.y - c * r1;
    f.z = f.z - c * r2;
    f.w = f.w - c * r3;
    p[x] = f;
}

__device__ __forceinline__ int64_t fix32(double v) { return (int64_t)rint(v * 0x1p32); }

__global__ __launch_bounds__(kPhiBlock) void k_phi_record(PhiDev d) {
    __shared__ uint32_t s_hist[33];
    __shared__ int64_t s_red[kPhiBlock / 64][8];
    __shared__ int s_last;
    const uint32_t tid = threadIdx.x, lane = tid & 63u, wv = tid >> 6;
    const uint32_t x = blockIdx.x * kPhiBlock + tid;
    if (tid < 33u) s_hist[tid] = 0u;
    __syncthreads();
    int64_t e = 0, m0 = 0, m1 = 0, m2 = 0, m3 = 0;
    uint64_t n = 0, mx = 0, sq = 0;
    if (x < d.N) {
        const double4 *p = reinterpret_cast<const double4 *>(d.phi);
        const double4 f = p[x];
#pragma unroll
        for (uint32_t mu = 0; mu < 4u; ++mu) {
            const double4 g = p[phi_step(x, d.L, mu)];
            e += fix32(dot4(f.x, f.y, f.z, f.w, g.x, g.y, g.z, g.w));
        }
        m0 = fix32(f.x);
        m1 = fix32(f.y);
        m2 = fix32(f.z);
        m3 = fix32(f.w);
        if (d.parent[x] == x) {
            const uint64_t S = d.csize[x];
            n = 1u;
            mx = S;
            sq = S * S;
            atomicAdd(&s_hist[63 - __clzll((long long)S)], 1u);
        }
    }
#pragma unroll
    for (int o = 32; o > 0; o >>= 1) {
        e += __shfl_xor(e, o, 64);
        m0 += __shfl_xor(m0, o, 64);
        m1 += __shfl_xor(m1, o, 64);
        m2 += __shfl_xor(m2, o, 64);
        m3 += __shfl_xor(m3, o, 64);
        n += __shfl_xor(n, o, 64);
        mx = max(mx, (uint64_t)__shfl_xor((unsigned long long)mx, o, 64));
        sq += __shfl_xor(sq, o, 64);
    }
    if (lane == 0u) {
        s_red[wv][0] = e;
        s_red[wv][1] = m0;
        s_red[wv][2] = m1;
        s_red[wv][3] = m2;
        s_red[wv][4] = m3;
        s_red[wv][5] = (int64_t)n;
        s_red[wv][6] = (int64_t)mx;
        s_red[wv][7] = (int64_t)sq;
    }
    __syncthreads();
    unsigned long long *acc = reinterpret_cast<unsigned long long *>(d.acc);
    if (tid < 8u) {
        int64_t v = 0;
        for (int w = 0; w < kPhiBlock / 64; ++w)
            v = tid == 6u ? max(v, s_red[w][tid]) : v + s_red[w][tid];
        const uint32_t slot = tid < 5u ? PA_E + tid : tid == 5u ? PA_N : tid == 6u ? PA_MAX : PA_SQ;
        if (tid == 6u)
            atomicMax(&acc[slot], (unsigned long long)v);
        else if (v != 0)
            atomicAdd(&acc[slot], (unsigned long long)v);
    }
    if (tid < 33u && s_hist[tid]) atomicAdd(&acc[PA_HIST + tid], (unsigned long long)s_hist[tid]);
    __threadfence();
    __syncthreads();
    if (tid == 0u) s_last = atomicAdd(&acc[PA_COUNT], 1ull) == (unsigned long long)gridDim.x - 1ull;
    __syncthreads();
    if (!s_last) return;
    __threadfence();
    // the last workgroup: the record of sweep t, then clear for the next
    __shared__ uint64_t s_tot[PA_END];
    if (tid < (uint32_t)PA_END) {
        s_tot[tid] = __hip_atomic_load(&acc[tid], __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
        __hip_atomic_store(&acc[tid], 0ull, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
    }
    if (tid == (uint32_t)PA_END) __hip_atomic_store(&acc[PA_COUNT], 0ull, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
    __syncthreads();
    const uint64_t tsw = *d.tdev;
    sw_phi4_obs *rec = &d.ring[tsw % d.ring_cap];
    if (tid < 33u) rec->hist_log2[tid] = s_tot[PA_HIST + tid];
    if (tid == 0u) {
        rec->sweep = tsw;
        const int64_t ef = (int64_t)s_tot[PA_E];
        rec->e_fix = ef;
        rec->action = -(2.0 * d.kappa) * ((double)ef * 0x1p-32);
        double ms = 0.0;
        for (int a = 0; a < 4; ++a) {
            const int64_t ma = (int64_t)s_tot[PA_M + a];
            rec->m_fix[a] = ma;
            const double v = (double)ma * 0x1p-32;
            ms = ms + v * v;
        }
        rec->m_abs = sqrt(ms);
        rec->n_clusters = s_tot[PA_N];
        rec->max_cluster = s_tot[PA_MAX];
        rec->sum_sq_sizes = s_tot[PA_SQ];
    }
    __syncthreads();
    if (tid == 0u) {
        *d.tdev = tsw + 1u;
        __threadfence();
    }
}

constexpr int kPhiStages = 5;

hipError_t phi_launch_stage(const PhiDev &d, int stage, hipStream_t s) {
    const uint32_t g = (d.N + kPhiBlock - 1) / kPhiBlock;
    switch (stage) {
    case 0: k_phi_proj<<<g, kPhiBlock, 0, s>>>(d); break;
    case 1: k_phi_bond<<<g, kPhiBlock, 0, s>>>(d); break;
    case 2: k_phi_flat<<<g, kPhiBlock, 0, s>>>(d); break;
    case 3: k_phi_flip<<<g, kPhiBlock, 0, s>>>(d); break;
    case 4: k_phi_record<<<g, kPhiBlock, 0, s>>>(d); break;
    default: return hipErrorInvalidValue;
    }
    return hipGetLastError();
}

hipError_t phi_launch_sweep(const PhiDev &d, hipStream_t s) {
    for (int i = 0; i < kPhiStages; ++i) {
        const hipError_t e = phi_launch_stage(d, i, s);
        if (e != hipSuccess) return e;
    }
    return hipSuccess;
}

struct PhiLayout {
    size_t phi, proj, parent, csize, dir, acc, tdev, ring, total;
};

PhiLayout phi_layout(int32_t L, int64_t ring) {
    const size_t N = (size_t)L * L * L * L;
    PhiLayout lo;
    size_t off = 0;
    auto take = [&](size_t b) {
        const size_t o = off;
        off += align_up(b);
        return o;
    };
    lo.phi = take(N * 4 * sizeof(double));
    lo.proj = take(N * sizeof(double));
    lo.parent = take(N * sizeof(uint32_t));
    lo.csize = take(N * sizeof(uint32_t));
    lo.dir = take(8 * sizeof(double));
    lo.acc = take(kPhiAccWords * sizeof(uint64_t));
    lo.tdev = take(sizeof(uint64_t));
    lo.ring = take((size_t)ring * sizeof(sw_phi4_obs));
    lo.total = off;
    return lo;
}

int phi_validate(int32_t L, double kappa, int32_t init, int64_t ring) {
    if (L < 2 || L > kPhiMaxL) return fail(SW_EINVAL, "L must be in [2, 64] for the phi^4 lattice (N = L^4)");
    if (!(kappa >= 0.0 && kappa <= kPhiMaxKappa)) return fail(SW_EINVAL, "kappa must be finite and in [0, 4]");
    if (init != SW_INIT_HOT && init != SW_INIT_COLD) return fail(SW_EINVAL, "init must be SW_INIT_HOT or SW_INIT_COLD");
    if (ring < 0 || ring > (int64_t)1 << 24) return fail(SW_EINVAL, "ring must be in [0, 2^24]");
    return SW_OK;
}

}  // namespace
}  // namespace swmi

using swmi::fail;
using swmi::hip_fail;

struct sw_phi4 {
    swmi::PhiDev dev;
    hipStream_t stream;
    bool own_stream;
    void *ws;
    bool own_ws;
    hipGraph_t graph;
    hipGraphExec_t gexec;
    bool graph_tried;
    uint64_t next_sweep;
    uint64_t first_valid;
    int device;
};

namespace {

int phi_ensure_device(const sw_phi4 *p) {
    int cur = -1;
    HIP_TRY(hipGetDevice(&cur));
    if (cur != p->device) HIP_TRY(hipSetDevice(p->device));
    return SW_OK;
}

int phi_set_tdev(sw_phi4 *p, uint64_t t) {
    HIP_TRY(hipMemcpyAsync(p->dev.tdev, &t, sizeof(t), hipMemcpyHostToDevice, p->stream));
    HIP_TRY(hipStreamSynchronize(p->stream));
    p->next_sweep = t;
    p->first_valid = t;
    return SW_OK;
}

// One sweep captured into a graph; on any capture failure the kernels are
// launched directly.
void phi_ensure_graph(sw_phi4 *p) {
    if (p->graph_tried) return;
    p->graph_tried = true;
    if (p->stream == nullptr) return;
    if (hipStreamBeginCapture(p->stream, hipStreamCaptureModeThreadLocal) != hipSuccess) {
        (void)hipGetLastError();
        return;
    }
    const hipError_t le = swmi::phi_launch_sweep(p->dev, p->stream);
    hipGraph_t g = nullptr;
    const hipError_t ce = hipStreamEndCapture(p->stream, &g);
    if (le != hipSuccess || ce != hipSuccess || g == nullptr) {
        if (g) (void)hipGraphDestroy(g);
        (void)hipGetLastError();
        return;
    }
    hipGraphExec_t ge = nullptr;
    if (hipGraphInstantiate(&ge, g, nullptr, nullptr, 0) != hipSuccess) {
        (void)hipGraphDestroy(g);
        (void)hipGetLastError();
        return;
    }
    p->graph = g;
    p->gexec = ge;
}

}  // namespace

extern "C" {

size_t sw_phi4_workspace_bytes(int32_t L, int64_t ring) {
    if (swmi::phi_validate(L, 0.0, SW_INIT_HOT, ring) != SW_OK) return 0;
    return swmi::phi_layout(L, ring ? ring : swmi::kDefaultRing).total;
}

int sw_phi4_create(int32_t L, double kappa, uint64_t seed, int32_t init, int64_t ring, void *dev_workspace,
                   size_t ws_bytes, void *hip_stream, sw_phi4 **out) {
    using namespace swmi;
    if (!out) return fail(SW_EINVAL, "out is NULL");
    *out = nullptr;
    int rc = phi_validate(L, kappa, init, ring);
    if (rc != SW_OK) return rc;
    if (ring == 0) ring = kDefaultRing;
    const PhiLayout lo = phi_layout(L, ring);
    if (dev_workspace && ws_bytes < lo.total)
        return fail(SW_ENOMEM, "workspace too small: need " + std::to_string(lo.total) + " bytes");
    if (dev_workspace && ((uintptr_t)dev_workspace % kAlign) != 0)
        return fail(SW_EINVAL, "workspace must be 256-byte aligned");
    sw_phi4 *p = new (std::nothrow) sw_phi4();
    if (!p) return fail(SW_ENOMEM, "host allocation failed");
    hipError_t e = hipGetDevice(&p->device);
    if (e != hipSuccess) {
        delete p;
        return hip_fail(e, "hipGetDevice");
    }
    if (dev_workspace) {
        p->ws = dev_workspace;
        p->own_ws = false;
    } else {
        e = hipMalloc(&p->ws, lo.total);
        if (e != hipSuccess) {
            (void)hipGetLastError();
            delete p;
            return fail(SW_ENOMEM, "hipMalloc of " + std::to_string(lo.total) + " bytes failed");
        }
        p->own_ws = true;
    }
    if (hip_stream || dev_workspace) {
        p->stream = (hipStream_t)hip_stream;
        p->own_stream = false;
    } else {
        e = hipStreamCreateWithFlags(&p->stream, hipStreamNonBlocking);
        if (e != hipSuccess) {
            if (p->own_ws) (void)hipFree(p->ws);
            delete p;
            return hip_fail(e, "hipStreamCreateWithFlags");
        }
        p->own_stream = true;
    }
    char *base = (char *)p->ws;
    PhiDev &d = p->dev;
    d.phi = (double *)(base + lo.phi);
    d.proj = (double *)(base + lo.proj);
    d.parent = (uint32_t *)(base + lo.parent);
    d.csize = (uint32_t *)(base + lo.csize);
    d.dir = (double *)(base + lo.dir);
    d.acc = (uint64_t *)(base + lo.acc);
    d.tdev = (uint64_t *)(base + lo.tdev);
    d.ring = (sw_phi4_obs *)(base + lo.ring);
    d.L = (uint32_t)L;
    d.N = (uint32_t)((size_t)L * L * L * L);
    d.ring_cap = (uint32_t)ring;
    d.seed_lo = (uint32_t)(seed & 0xFFFFFFFFu);
    d.seed_hi = (uint32_t)(seed >> 32);
    d.kappa = kappa;
    e = hipMemsetAsync(p->ws, 0, lo.total, p->stream);
    if (e == hipSuccess) e = hipStreamSynchronize(p->stream);
    if (e != hipSuccess) {
        rc = hip_fail(e, "clearing the workspace");
        sw_phi4_destroy(p);
        return rc;
    }
    rc = sw_phi4_reset(p, init);
    if (rc != SW_OK) {
        const std::string msg = last_error();
        sw_phi4_destroy(p);
        return fail(rc, msg);
    }
    *out = p;
    return SW_OK;
}

int sw_phi4_reset(sw_phi4 *p, int32_t init) {
    if (!p) return fail(SW_EINVAL, "phi4 sim is NULL");
    if (init != SW_INIT_HOT && init != SW_INIT_COLD) return fail(SW_EINVAL, "init must be SW_INIT_HOT or SW_INIT_COLD");
    int rc = phi_ensure_device(p);
    if (rc != SW_OK) return rc;
    rc = phi_set_tdev(p, 0);
    if (rc != SW_OK) return rc;
    const uint32_t g = (p->dev.N + swmi::kPhiBlock - 1) / swmi::kPhiBlock;
    swmi::k_phi_init<<<g, swmi::kPhiBlock, 0, p->stream>>>(p->dev, init == SW_INIT_COLD ? 1 : 0);
    HIP_TRY(hipGetLastError());
    HIP_TRY(hipStreamSynchronize(p->stream));
    return SW_OK;
}

int sw_phi4_sweep(sw_phi4 *p, int64_t n) {
    if (!p) return fail(SW_EINVAL, "phi4 sim is NULL");
    if (n < 0) return fail(SW_EINVAL, "n must be >= 0");
    if (n == 0) return SW_OK;
    int rc = phi_ensure_device(p);
    if (rc != SW_OK) return rc;
    phi_ensure_graph(p);
    for (int64_t i = 0; i < n; ++i) {
        if (p->gexec)
            HIP_TRY(hipGraphLaunch(p->gexec, p->stream));
        else
            HIP_TRY(swmi::phi_launch_sweep(p->dev, p->stream));
    }
    p->next_sweep += (uint64_t)n;
    return SW_OK;
}

int sw_phi4_sync(sw_phi4 *p) {
    if (!p) return fail(SW_EINVAL, "phi4 sim is NULL");
    int rc = phi_ensure_device(p);
    if (rc != SW_OK) return rc;
    HIP_TRY(hipStreamSynchronize(p->stream));
    return SW_OK;
}

int sw_phi4_profile(sw_phi4 *p, int64_t n, double *ms, int32_t nk) {
    if (!p || !ms) return fail(SW_EINVAL, "phi4 sim or ms is NULL");
    if (n < 1) return fail(SW_EINVAL, "n must be >= 1");
    if (nk < swmi::kPhiStages) return fail(SW_ERANGE, "nk must be >= 5");
    int rc = phi_ensure_device(p);
    if (rc != SW_OK) return rc;
    constexpr int kEv = swmi::kPhiStages + 1;
    hipEvent_t ev[kEv];
    for (int i = 0; i < kEv; ++i) {
        const hipError_t e = hipEventCreate(&ev[i]);
        if (e != hipSuccess) {
            for (int j = 0; j < i; ++j) (void)hipEventDestroy(ev[j]);
            return hip_fail(e, "hipEventCreate");
        }
    }
    double acc[swmi::kPhiStages] = {0};
    hipError_t e = hipSuccess;
    for (int64_t i = 0; i < n && e == hipSuccess; ++i) {
        e = hipEventRecord(ev[0], p->stream);
        for (int st = 0; st < swmi::kPhiStages && e == hipSuccess; ++st) {
            e = swmi::phi_launch_stage(p->dev, st, p->stream);
            if (e == hipSuccess) e = hipEventRecord(ev[st + 1], p->stream);
        }
        if (e == hipSuccess) e = hipEventSynchronize(ev[kEv - 1]);
        for (int st = 0; st < swmi::kPhiStages && e == hipSuccess; ++st) {
            float f = 0.f;
            e = hipEventElapsedTime(&f, ev[st], ev[st + 1]);
            acc[st] += f;
        }
        if (e == hipSuccess) p->next_sweep += 1u;
    }
    for (int i = 0; i < kEv; ++i) (void)hipEventDestroy(ev[i]);
    if (e != hipSuccess) return hip_fail(e, "sw_phi4_profile");
    for (int i = 0; i < nk; ++i) ms[i] = i < swmi::kPhiStages ? acc[i] / (double)n : 0.0;
    return SW_OK;
}

int sw_phi4_series(sw_phi4 *p, int64_t first, int64_t count, sw_phi4_obs *out) {
    if (!p) return fail(SW_EINVAL, "phi4 sim is NULL");
    if (count < 0 || (count > 0 && !out)) return fail(SW_EINVAL, "bad count or NULL out");
    const int64_t lo = std::max<int64_t>((int64_t)p->first_valid, (int64_t)p->next_sweep - (int64_t)p->dev.ring_cap);
    if (first < lo || first + count > (int64_t)p->next_sweep)
        return fail(SW_ERANGE, "records requested outside the sweeps run and held in the ring");
    if (count == 0) return SW_OK;
    int rc = phi_ensure_device(p);
    if (rc != SW_OK) return rc;
    HIP_TRY(hipStreamSynchronize(p->stream));
    const int64_t cap = p->dev.ring_cap;
    int64_t done = 0;
    while (done < count) {
        const int64_t slot = (first + done) % cap;
        const int64_t run = std::min(count - done, cap - slot);
        HIP_TRY(hipMemcpy(out + done, p->dev.ring + slot, (size_t)run * sizeof(sw_phi4_obs), hipMemcpyDeviceToHost));
        done += run;
    }
    return SW_OK;
}

int sw_phi4_get_field(sw_phi4 *p, double *host, int64_t n) {
    if (!p || !host) return fail(SW_EINVAL, "phi4 sim or host is NULL");
    if (n != 4 * (int64_t)p->dev.N) return fail(SW_ERANGE, "n must equal 4 L^4");
    int rc = phi_ensure_device(p);
    if (rc != SW_OK) return rc;
    HIP_TRY(hipStreamSynchronize(p->stream));
    HIP_TRY(hipMemcpy(host, p->dev.phi, (size_t)n * sizeof(double), hipMemcpyDeviceToHost));
    return SW_OK;
}

int sw_phi4_set_field(sw_phi4 *p, const double *host, int64_t n, uint64_t next_sweep) {
    if (!p || !host) return fail(SW_EINVAL, "phi4 sim or host is NULL");
    if (n != 4 * (int64_t)p->dev.N) return fail(SW_ERANGE, "n must equal 4 L^4");
    for (int64_t i = 0; i < n; ++i)
        if (!std::isfinite(host[i])) return fail(SW_EINVAL, "field component " + std::to_string(i) + " is not finite");
    int rc = phi_ensure_device(p);
    if (rc != SW_OK) return rc;
    HIP_TRY(hipStreamSynchronize(p->stream));
    HIP_TRY(hipMemcpy(p->dev.phi, host, (size_t)n * sizeof(double), hipMemcpyHostToDevice));
    return phi_set_tdev(p, next_sweep);
}

int sw_phi4_get_labels(sw_phi4 *p, uint32_t *host, int64_t n) {
    if (!p || !host) return fail(SW_EINVAL, "phi4 sim or host is NULL");
    if (n != (int64_t)p->dev.N) return fail(SW_ERANGE, "n must equal L^4");
    if (p->next_sweep == p->first_valid) return fail(SW_ESTATE, "no sweep has run since create / reset / set_field");
    int rc = phi_ensure_device(p);
    if (rc != SW_OK) return rc;
    HIP_TRY(hipStreamSynchronize(p->stream));
    HIP_TRY(hipMemcpy(host, p->dev.parent, (size_t)n * sizeof(uint32_t), hipMemcpyDeviceToHost));
    return SW_OK;
}

int64_t sw_phi4_sites(const sw_phi4 *p) { return p ? (int64_t)p->dev.N : -1; }

int64_t sw_phi4_next_sweep(const sw_phi4 *p) { return p ? (int64_t)p->next_sweep : -1; }

void sw_phi4_destroy(sw_phi4 *p) {
    if (!p) return;
    if (phi_ensure_device(p) == SW_OK && p->stream) (void)hipStreamSynchronize(p->stream);
    if (p->gexec) (void)hipGraphExecDestroy(p->gexec);
    if (p->graph) (void)hipGraphDestroy(p->graph);
    if (p->own_ws && p->ws) (void)hipFree(p->ws);
    if (p->own_stream && p->stream) (void)hipStreamDestroy(p->stream);
    delete p;
}

}  // extern "C"
