// sw_api.hip -- host runtime and C ABI of libswmi (declared in swmi.h).
//
// A sim owns (or borrows) one device workspace carved into the buffers of
// sw_internal.h, one stream, and one captured hipGraph holding the kernels
// of a single sweep; sw_sweep(n) replays that graph n times and ends with
// k_resolve, so between calls the spin buffer always holds final +-1 spins.
#include <math.h>
#include <stdio.h>
#include <string.h>

#include <algorithm>
#include <new>
#include <string>
#include <vector>

#include "sw_host.h"

using swmi::Dev;
using swmi::Layout;
using swmi::align_up;
using swmi::bond_threshold;
using swmi::fail;
using swmi::hip_fail;
using swmi::kAlign;
using swmi::kDefaultRing;
using swmi::layout_of;
using swmi::make_dev;
using swmi::resolve_tile;
using swmi::validate;

namespace swmi {

namespace {
thread_local std::string g_err;
}

int fail(int code, const std::string &msg) {
    g_err = msg;
    return code;
}

int hip_fail(hipError_t e, const char *what) {
    return fail(SW_EHIP, std::string(what) + ": " + hipGetErrorString(e));
}

const std::string &last_error() { return g_err; }

// Bond probability p = 1 - exp(-2 beta J) (Sec. 2.1, read with the factor 2J
// that puts T_c at 2/ln(1+sqrt 2)), as a 32-bit threshold: P(bond) = T/2^32.
uint32_t bond_threshold(double beta, double J) {
    const double p = -expm1(-2.0 * beta * J);
    if (!(p > 0.0)) return 0u;
    const double scaled = floor(ldexp(p, 32));
    if (scaled >= 4294967296.0) return 0xFFFFFFFFu;
    return (uint32_t)scaled;
}

int resolve_tile(const sw_config &c) {
    // the Potts model fits its values below the node codes of a 64-wide
    // tile only for q <= 4
    if (c.tile == 0) return (c.L % 64 == 0 && c.q <= 4) ? 64 : 32;
    return c.tile;
}

size_t sites_of(const sw_config &c) {
    const size_t L = (size_t)c.L;
    return c.dims == 3 ? L * L * L : L * L;
}

int validate(const sw_config *c) {
    if (!c) return fail(SW_EINVAL, "config is NULL");
    if (c->dims != 0 && c->dims != 2 && c->dims != 3) return fail(SW_EINVAL, "dims must be 0, 2 or 3");
    if (c->dims == 3) {
        if (c->L < 16 || c->L > 1616 || c->L % 16 != 0)
            return fail(SW_EINVAL, "L of the simple cubic lattice must be a multiple of 16 in [16, 1616]");
    } else if (c->L < 32 || c->L > 32768 || c->L % 32 != 0) {
        return fail(SW_EINVAL, "L must be a multiple of 32 in [32, 32768]");
    }
    if (!(c->beta >= 0.0) || !isfinite(c->beta)) return fail(SW_EINVAL, "beta must be finite and >= 0");
    if (!(c->J > 0.0) || !isfinite(c->J)) return fail(SW_EINVAL, "J must be finite and > 0");
    if (c->init != SW_INIT_HOT && c->init != SW_INIT_COLD) return fail(SW_EINVAL, "init must be SW_INIT_HOT or SW_INIT_COLD");
    if (c->tile != 0 && c->tile != 32 && c->tile != 64) return fail(SW_EINVAL, "tile must be 0, 32 or 64");
    if (c->tile == 64 && c->L % 64 != 0 && c->dims != 3)
        return fail(SW_EINVAL, "tile 64 needs L to be a multiple of 64");
    if ((c->flags & ~(SW_FLAG_LABELS | SW_FLAG_DENSE_HIST | SW_FLAG_LABEL_EQUIV)) != 0u)
        return fail(SW_EINVAL, "unknown flag bits");
    if (c->ring < 0 || c->ring > (int64_t)1 << 30) return fail(SW_EINVAL, "ring must be in [0, 2^30]");
    if (c->q != 0 && (c->q < 2 || c->q > swmi::kMaxQ))
        return fail(SW_EINVAL, "q must be 0 (Ising) or in [2, 8] (Potts)");
    if (c->q > 4 && c->tile == 64 && !(c->flags & SW_FLAG_LABEL_EQUIV) && c->dims != 3)
        return fail(SW_EINVAL, "the q-state Potts model with q > 4 uses 32-wide tiles (tile 0 or 32)");
    return SW_OK;
}

Layout layout_of(const sw_config &c) {
    const size_t L = (size_t)c.L, N = sites_of(c);
    // the label-equivalence path and the cubic bricks keep labels in global
    // memory and no tile structures; their group partials are one per
    // kLeChunk sites
    const bool le = (c.flags & SW_FLAG_LABEL_EQUIV) != 0u || c.dims == 3;
    const size_t tw = (size_t)resolve_tile(c);
    const size_t ntiles = le ? 0 : (L / tw) * (L / tw);
    const size_t ngroups = le ? (N + swmi::kLeChunk - 1) / swmi::kLeChunk
                              : (ntiles + swmi::kGroupTiles - 1) / swmi::kGroupTiles;
    const size_t nodes = ntiles * swmi::kNodeSlots;
    const size_t ring = (size_t)(c.ring > 0 ? c.ring : kDefaultRing);
    Layout o{};
    size_t off = 0;
    auto take = [&](size_t bytes) {
        const size_t at = off;
        off = align_up(off + bytes);
        return at;
    };
    o.spins[0] = take(N);
    o.spins[1] = le ? o.spins[0] : take(N);  // final spins in place
    o.parent[0] = take(nodes * 4);
    o.parent[1] = take(nodes * 4);
    o.nk[0] = take(ntiles * 4);
    o.nk[1] = take(ntiles * 4);
    o.key = take(nodes * 4);
    o.nsize = take(nodes * 4);
    o.rspin = take(nodes);
    o.edge = take(ntiles * 4 * tw);
    o.xb = take(ntiles * 16);
    o.tpart = take(ntiles * swmi::kTilePart * 4);
    o.gpart = take(ngroups * swmi::kGroupPart * 8);
    o.acc = take(swmi::kAccWords * 8);
    o.tdev = take(8);
    o.ring = take(ring * sizeof(sw_obs));
    o.labels = (le || (c.flags & SW_FLAG_LABELS)) ? take(N * 4) : 0;
    o.dense = (c.flags & SW_FLAG_DENSE_HIST) ? take((N + 1) * 8) : 0;
    o.le_mask = le ? take(N) : 0;
    o.le_cnt = le ? take(N * 4) : 0;
    o.le_rsp = le ? take(N) : 0;
    o.le_ctl = le ? take(64) : 0;
    // cubic bricks: the x-face labels of every brick, so that the face
    // unions read them contiguously
    const bool brick = c.dims == 3 && !(c.flags & SW_FLAG_LABEL_EQUIV);
    o.bface = brick ? take(N / 4096 * 512 * 4) : 0;
    o.total = off;
    return o;
}

// The device view of one lattice whose buffers start at `base`.
Dev make_dev(const sw_config &c, char *base, const Layout &lo) {
    Dev d;
    memset(&d, 0, sizeof(d));
    d.L = (uint32_t)c.L;
    d.tw = (uint32_t)resolve_tile(c);
    d.ntx = d.L / d.tw;
    d.ntiles = d.ntx * d.ntx;
    d.dims = c.dims == 3 ? 3u : 2u;
    d.nsite = sites_of(c);
    d.ngroups = (d.ntiles + swmi::kGroupTiles - 1) / swmi::kGroupTiles;
    // Potts coupling: one J per equal pair, p = 1 - exp(-beta J) (the Ising
    // threshold at half the coupling)
    d.q = (uint32_t)c.q;
    d.T = c.q ? bond_threshold(0.5 * c.beta, c.J) : bond_threshold(c.beta, c.J);
    d.seed_lo = (uint32_t)(c.seed & 0xFFFFFFFFu);
    d.seed_hi = (uint32_t)(c.seed >> 32);
    d.ring_cap = (uint32_t)c.ring;
    d.J = c.J;
    for (int i = 0; i < 2; ++i) {
        d.spins[i] = (int8_t *)(base + lo.spins[i]);
        d.parent[i] = (uint32_t *)(base + lo.parent[i]);
        d.nk[i] = (uint32_t *)(base + lo.nk[i]);
    }
    d.key = (uint32_t *)(base + lo.key);
    d.nsize = (uint32_t *)(base + lo.nsize);
    d.rspin = (int8_t *)(base + lo.rspin);
    d.edge = (uint8_t *)(base + lo.edge);
    d.xb = (uint64_t *)(base + lo.xb);
    d.tpart = (int32_t *)(base + lo.tpart);
    d.gpart = (uint64_t *)(base + lo.gpart);
    d.acc = (uint64_t *)(base + lo.acc);
    d.tdev = (uint64_t *)(base + lo.tdev);
    d.ring = (sw_obs *)(base + lo.ring);
    const bool le = (c.flags & SW_FLAG_LABEL_EQUIV) != 0u || c.dims == 3;
    d.labels = (le || (c.flags & SW_FLAG_LABELS)) ? (uint32_t *)(base + lo.labels) : nullptr;
    d.dense = (c.flags & SW_FLAG_DENSE_HIST) ? (uint64_t *)(base + lo.dense) : nullptr;
    if (le) {
        d.ntiles = 0;
        d.ntx = 0;
        d.ngroups = (uint32_t)((d.nsite + swmi::kLeChunk - 1) / swmi::kLeChunk);
        if (c.dims == 3 && !(c.flags & SW_FLAG_LABEL_EQUIV)) {
            d.brick = 1u;
            d.tw = swmi::kBrick;
            d.bface = (uint32_t *)(base + lo.bface);
        }
        d.le_mask = (uint8_t *)(base + lo.le_mask);
        d.le_cnt = (uint32_t *)(base + lo.le_cnt);
        d.le_rsp = (int8_t *)(base + lo.le_rsp);
        d.le_ctl = (uint32_t *)(base + lo.le_ctl);
    }
    return d;
}

}  // namespace swmi

struct sw_sim {
    sw_config cfg;
    Dev dev;
    hipStream_t stream;
    bool own_stream;
    void *ws;
    size_t ws_bytes;
    bool own_ws;
    hipGraph_t graph;
    hipGraphExec_t gexec;
    bool graph_tried;
    uint64_t next_sweep;   // host mirror of *dev.tdev
    uint64_t first_valid;  // first sweep whose record exists
    int device;
};

namespace {

int ensure_device(const sw_sim *s) {
    int cur = -1;
    HIP_TRY(hipGetDevice(&cur));
    if (cur != s->device) HIP_TRY(hipSetDevice(s->device));
    return SW_OK;
}

int set_tdev(sw_sim *s, uint64_t t) {
    HIP_TRY(hipMemcpyAsync(s->dev.tdev, &t, sizeof(t), hipMemcpyHostToDevice, s->stream));
    HIP_TRY(hipStreamSynchronize(s->stream));
    s->next_sweep = t;
    s->first_valid = t;
    return SW_OK;
}

void drop_graph(sw_sim *s) {
    if (s->gexec) (void)hipGraphExecDestroy(s->gexec);
    if (s->graph) (void)hipGraphDestroy(s->graph);
    s->gexec = nullptr;
    s->graph = nullptr;
    s->graph_tried = false;
}

// Captures one sweep into a graph (not on the legacy null stream, which
// cannot be captured); on any capture failure the sweeps are launched
// directly, with the same kernels.
void ensure_graph(sw_sim *s) {
    if (s->graph_tried) return;
    s->graph_tried = true;
    if (s->stream == nullptr) return;
    if (hipStreamBeginCapture(s->stream, hipStreamCaptureModeThreadLocal) != hipSuccess) {
        (void)hipGetLastError();
        return;
    }
    const hipError_t le = swmi::launch_sweep(s->dev, s->stream);
    hipGraph_t g = nullptr;
    const hipError_t ce = hipStreamEndCapture(s->stream, &g);
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
    s->graph = g;
    s->gexec = ge;
}

}  // namespace

extern "C" {

const char *sw_last_error(void) { return swmi::last_error().c_str(); }

int sw_config_init(sw_config *cfg, int32_t L, double beta, double J, uint64_t seed) {
    if (!cfg) return fail(SW_EINVAL, "cfg is NULL");
    memset(cfg, 0, sizeof(*cfg));
    cfg->L = L;
    cfg->beta = beta;
    cfg->J = J;
    cfg->seed = seed;
    cfg->init = SW_INIT_HOT;
    cfg->tile = 0;
    cfg->flags = 0u;
    cfg->ring = 0;
    return SW_OK;
}

size_t sw_workspace_bytes_ex(const sw_config *cfg) {
    if (validate(cfg) != SW_OK) return 0;
    return layout_of(*cfg).total;
}

size_t sw_workspace_bytes(int32_t L) {
    sw_config c;
    sw_config_init(&c, L, 0.0, 1.0, 0);
    return sw_workspace_bytes_ex(&c);
}

int sw_create_ex(const sw_config *cfg, void *dev_workspace, size_t ws_bytes, void *hip_stream, sw_sim **out) {
    if (!out) return fail(SW_EINVAL, "out is NULL");
    *out = nullptr;
    int rc = validate(cfg);
    if (rc != SW_OK) return rc;
    const Layout lo = layout_of(*cfg);
    if (dev_workspace && ws_bytes < lo.total)
        return fail(SW_ENOMEM, "workspace too small: need " + std::to_string(lo.total) + " bytes");
    if (dev_workspace && ((uintptr_t)dev_workspace % kAlign) != 0)
        return fail(SW_EINVAL, "workspace must be 256-byte aligned");

    sw_sim *s = new (std::nothrow) sw_sim();
    if (!s) return fail(SW_ENOMEM, "host allocation failed");
    s->cfg = *cfg;
    if (s->cfg.ring == 0) s->cfg.ring = kDefaultRing;
    hipError_t e = hipGetDevice(&s->device);
    if (e != hipSuccess) {
        delete s;
        return hip_fail(e, "hipGetDevice");
    }
    if (dev_workspace) {
        s->ws = dev_workspace;
        s->ws_bytes = ws_bytes;
        s->own_ws = false;
        s->stream = (hipStream_t)hip_stream;
        s->own_stream = false;
    } else {
        e = hipMalloc(&s->ws, lo.total);
        if (e != hipSuccess) {
            (void)hipGetLastError();
            delete s;
            return fail(SW_ENOMEM, "hipMalloc of " + std::to_string(lo.total) + " bytes failed");
        }
        s->ws_bytes = lo.total;
        s->own_ws = true;
        if (hip_stream) {
            s->stream = (hipStream_t)hip_stream;
            s->own_stream = false;
        } else {
            e = hipStreamCreateWithFlags(&s->stream, hipStreamNonBlocking);
            if (e != hipSuccess) {
                (void)hipFree(s->ws);
                delete s;
                return hip_fail(e, "hipStreamCreateWithFlags");
            }
            s->own_stream = true;
        }
    }
    const sw_config &c = s->cfg;
    s->dev = make_dev(c, (char *)s->ws, lo);
    if (c.flags & SW_FLAG_LABEL_EQUIV) {
        s->dev.le_grid = swmi::le_grid_size(s->dev.dims);
        if (s->dev.le_grid == 0) {
            sw_destroy(s);
            return fail(SW_EHIP, "cannot size the cooperative labelling launch");
        }
    }

    // Everything starts at zero: no nodes in either parity, empty accumulators.
    e = hipMemsetAsync(s->ws, 0, lo.total, s->stream);
    if (e == hipSuccess) e = hipStreamSynchronize(s->stream);
    if (e != hipSuccess) {
        rc = hip_fail(e, "clearing the workspace");
        sw_destroy(s);
        return rc;
    }
    rc = sw_reset(s, c.init);
    if (rc != SW_OK) {
        const std::string msg = swmi::last_error();
        sw_destroy(s);
        return fail(rc, msg);
    }
    *out = s;
    return SW_OK;
}

int sw_create_in(int32_t L, double beta, double J, uint64_t seed, void *dev_workspace, size_t ws_bytes,
                 void *hip_stream, sw_sim **out) {
    if (!dev_workspace) return fail(SW_EINVAL, "dev_workspace is NULL");
    sw_config c;
    sw_config_init(&c, L, beta, J, seed);
    return sw_create_ex(&c, dev_workspace, ws_bytes, hip_stream, out);
}

int sw_create(int32_t L, double beta, double J, uint64_t seed, sw_sim **out) {
    sw_config c;
    sw_config_init(&c, L, beta, J, seed);
    return sw_create_ex(&c, nullptr, 0, nullptr, out);
}

int sw_reset(sw_sim *s, int init_mode) {
    if (!s) return fail(SW_EINVAL, "sim is NULL");
    if (init_mode != SW_INIT_HOT && init_mode != SW_INIT_COLD)
        return fail(SW_EINVAL, "init_mode must be SW_INIT_HOT or SW_INIT_COLD");
    int rc = ensure_device(s);
    if (rc != SW_OK) return rc;
    rc = set_tdev(s, 0);
    if (rc != SW_OK) return rc;
    HIP_TRY(swmi::launch_init(s->dev, init_mode == SW_INIT_COLD ? 1 : 0, s->stream));
    HIP_TRY(hipStreamSynchronize(s->stream));
    return SW_OK;
}

int sw_sweep(sw_sim *s, int64_t n) {
    if (!s) return fail(SW_EINVAL, "sim is NULL");
    if (n < 0) return fail(SW_EINVAL, "n must be >= 0");
    if (n == 0) return SW_OK;
    int rc = ensure_device(s);
    if (rc != SW_OK) return rc;
    ensure_graph(s);
    for (int64_t i = 0; i < n; ++i) {
        if (s->gexec)
            HIP_TRY(hipGraphLaunch(s->gexec, s->stream));
        else
            HIP_TRY(swmi::launch_sweep(s->dev, s->stream));
    }
    HIP_TRY(swmi::launch_resolve(s->dev, s->stream));
    s->next_sweep += (uint64_t)n;
    return SW_OK;
}

int sw_profile(sw_sim *s, int64_t n, double *ms, int32_t nk) {
    if (!s || !ms) return fail(SW_EINVAL, "sim or ms is NULL");
    if (n < 1) return fail(SW_EINVAL, "n must be >= 1");
    if (nk < swmi::kStages + 1) return fail(SW_ERANGE, "nk must be >= 6");
    int rc = ensure_device(s);
    if (rc != SW_OK) return rc;
    constexpr int kEv = swmi::kStages + 1;
    hipEvent_t ev[kEv];
    for (int i = 0; i < kEv; ++i) {
        const hipError_t e = hipEventCreate(&ev[i]);
        if (e != hipSuccess) {
            for (int j = 0; j < i; ++j) (void)hipEventDestroy(ev[j]);
            return hip_fail(e, "hipEventCreate");
        }
    }
    double acc[swmi::kStages + 1] = {0};
    hipError_t e = hipSuccess;
    for (int64_t i = 0; i < n && e == hipSuccess; ++i) {
        e = hipEventRecord(ev[0], s->stream);
        for (int st = 0; st < swmi::kStages && e == hipSuccess; ++st) {
            e = swmi::launch_stage(s->dev, st, s->stream);
            if (e == hipSuccess) e = hipEventRecord(ev[st + 1], s->stream);
        }
        if (e == hipSuccess) e = hipEventSynchronize(ev[kEv - 1]);
        for (int st = 0; st < swmi::kStages && e == hipSuccess; ++st) {
            float t = 0.f;
            e = hipEventElapsedTime(&t, ev[st], ev[st + 1]);
            acc[st] += t;
        }
    }
    if (e == hipSuccess) {
        e = hipEventRecord(ev[0], s->stream);
        if (e == hipSuccess) e = swmi::launch_resolve(s->dev, s->stream);
        if (e == hipSuccess) e = hipEventRecord(ev[1], s->stream);
        if (e == hipSuccess) e = hipEventSynchronize(ev[1]);
        float t = 0.f;
        if (e == hipSuccess) e = hipEventElapsedTime(&t, ev[0], ev[1]);
        acc[swmi::kStages] = t;
    }
    for (int i = 0; i < kEv; ++i) (void)hipEventDestroy(ev[i]);
    if (e != hipSuccess) return hip_fail(e, "sw_profile");
    s->next_sweep += (uint64_t)n;
    for (int st = 0; st < swmi::kStages; ++st) ms[st] = acc[st] / (double)n;
    ms[swmi::kStages] = acc[swmi::kStages];
    for (int32_t i = swmi::kStages + 1; i < nk; ++i) ms[i] = 0.0;
    return SW_OK;
}

int sw_sync(sw_sim *s) {
    if (!s) return fail(SW_EINVAL, "sim is NULL");
    int rc = ensure_device(s);
    if (rc != SW_OK) return rc;
    HIP_TRY(hipStreamSynchronize(s->stream));
    return SW_OK;
}

int sw_series(sw_sim *s, int64_t first, int64_t count, sw_obs *out) {
    if (!s) return fail(SW_EINVAL, "sim is NULL");
    if (count < 0 || (count > 0 && !out)) return fail(SW_EINVAL, "bad count or NULL out");
    if (count == 0) return SW_OK;
    if (first < (int64_t)s->first_valid || first + count > (int64_t)s->next_sweep)
        return fail(SW_ERANGE, "records requested outside the sweeps run since the last reset / set_spins");
    const uint64_t cap = s->dev.ring_cap;
    if ((uint64_t)(s->next_sweep - (uint64_t)first) > cap)
        return fail(SW_ERANGE, "records requested have left the ring");
    int rc = ensure_device(s);
    if (rc != SW_OK) return rc;
    HIP_TRY(hipStreamSynchronize(s->stream));
    int64_t done = 0;
    while (done < count) {
        const uint64_t idx = (uint64_t)(first + done) % cap;
        const int64_t chunk = (int64_t)std::min<uint64_t>((uint64_t)(count - done), cap - idx);
        HIP_TRY(hipMemcpyAsync(out + done, s->dev.ring + idx, (size_t)chunk * sizeof(sw_obs), hipMemcpyDeviceToHost,
                               s->stream));
        done += chunk;
    }
    HIP_TRY(hipStreamSynchronize(s->stream));
    return SW_OK;
}

int sw_observables(sw_sim *s, sw_obs *out) {
    if (!s || !out) return fail(SW_EINVAL, "sim or out is NULL");
    if (s->next_sweep == s->first_valid) return fail(SW_ESTATE, "no sweep has run since the last reset / set_spins");
    return sw_series(s, (int64_t)s->next_sweep - 1, 1, out);
}

int sw_cluster_hist(sw_sim *s, uint64_t *counts, int64_t len) {
    if (!s || !counts) return fail(SW_EINVAL, "sim or counts is NULL");
    if (!s->dev.dense) return fail(SW_ESTATE, "sim was created without SW_FLAG_DENSE_HIST");
    const int64_t n = (int64_t)s->dev.nsite;
    if (len < n + 1) return fail(SW_ERANGE, "len must be >= N + 1");
    if (s->next_sweep == s->first_valid) return fail(SW_ESTATE, "no sweep has run since the last reset / set_spins");
    int rc = ensure_device(s);
    if (rc != SW_OK) return rc;
    HIP_TRY(hipMemcpyAsync(counts, s->dev.dense, (size_t)(n + 1) * 8, hipMemcpyDeviceToHost, s->stream));
    HIP_TRY(hipStreamSynchronize(s->stream));
    return SW_OK;
}

int sw_get_spins(sw_sim *s, int8_t *host, int64_t n) {
    if (!s || !host) return fail(SW_EINVAL, "sim or host is NULL");
    if (n != (int64_t)s->dev.nsite) return fail(SW_ERANGE, "n must equal the number of sites");
    int rc = ensure_device(s);
    if (rc != SW_OK) return rc;
    HIP_TRY(hipMemcpyAsync(host, s->dev.spins[s->next_sweep & 1u], (size_t)n, hipMemcpyDeviceToHost, s->stream));
    HIP_TRY(hipStreamSynchronize(s->stream));
    return SW_OK;
}

int sw_set_spins(sw_sim *s, const int8_t *host, int64_t n, uint64_t next_sweep) {
    if (!s || !host) return fail(SW_EINVAL, "sim or host is NULL");
    if (n != (int64_t)s->dev.nsite) return fail(SW_ERANGE, "n must equal the number of sites");
    const int32_t q = s->cfg.q;
    for (int64_t i = 0; i < n; ++i) {
        if (q == 0 && host[i] != 1 && host[i] != -1) return fail(SW_EINVAL, "spins must be +1 or -1");
        if (q != 0 && (host[i] < 0 || host[i] >= q)) return fail(SW_EINVAL, "Potts spins must be in 0..q-1");
    }
    int rc = ensure_device(s);
    if (rc != SW_OK) return rc;
    HIP_TRY(hipStreamSynchronize(s->stream));
    HIP_TRY(hipMemcpyAsync(s->dev.spins[next_sweep & 1u], host, (size_t)n, hipMemcpyHostToDevice, s->stream));
    return set_tdev(s, next_sweep);
}

int sw_get_labels(sw_sim *s, uint32_t *host, int64_t n) {
    if (!s || !host) return fail(SW_EINVAL, "sim or host is NULL");
    if (!s->dev.labels) return fail(SW_ESTATE, "sim was created without SW_FLAG_LABELS");
    if (n != (int64_t)s->dev.nsite) return fail(SW_ERANGE, "n must equal the number of sites");
    if (s->next_sweep == s->first_valid) return fail(SW_ESTATE, "no sweep has run since the last reset / set_spins");
    int rc = ensure_device(s);
    if (rc != SW_OK) return rc;
    HIP_TRY(hipMemcpyAsync(host, s->dev.labels, (size_t)n * 4, hipMemcpyDeviceToHost, s->stream));
    HIP_TRY(hipStreamSynchronize(s->stream));
    return SW_OK;
}

int32_t sw_label_passes(sw_sim *s) {
    if (!s || !s->dev.le_ctl) return -1;
    if (ensure_device(s) != SW_OK) return -1;
    uint32_t v[2] = {0, 0};
    if (hipStreamSynchronize(s->stream) != hipSuccess) return -1;
    if (hipMemcpy(v, s->dev.le_ctl + swmi::LE_PASSES, sizeof(v), hipMemcpyDeviceToHost) != hipSuccess) return -1;
    return v[1] ? -2 : (int32_t)v[0];
}

uint32_t sw_threshold(const sw_sim *s) { return s ? s->dev.T : 0u; }
int64_t sw_next_sweep(const sw_sim *s) { return s ? (int64_t)s->next_sweep : -1; }
int32_t sw_lattice(const sw_sim *s) { return s ? (int32_t)s->dev.L : 0; }
int32_t sw_tile(const sw_sim *s) { return s ? (s->dev.le_grid ? 0 : (int32_t)s->dev.tw) : 0; }  // brick side for cubic
int64_t sw_sites(const sw_sim *s) { return s ? (int64_t)s->dev.nsite : -1; }

void sw_destroy(sw_sim *s) {
    if (!s) return;
    (void)ensure_device(s);
    (void)hipStreamSynchronize(s->stream);
    drop_graph(s);
    if (s->own_ws && s->ws) (void)hipFree(s->ws);
    if (s->own_stream && s->stream) (void)hipStreamDestroy(s->stream);
    delete s;
}

}  // extern "C"

// ===================================================================== batches

// Launch groups of a batch: Ising and Potts replicas, each with 64-wide or
// 32-wide tiles, run different instantiations of the tile kernels.
constexpr int kBatchGroups = 4;

struct sw_batch {
    std::vector<sw_config> cfg;
    std::vector<Dev> dev;      // host copies of the replicas' device views
    std::vector<uint8_t> lds;  // 1 where the replica's merge runs in LDS
    swmi::BatchDev bd[kBatchGroups];
    hipStream_t stream;
    bool own_stream;
    // the LDS merges run on a second stream (default priority) beside the
    // global merge, forked after the tile kernels and joined before the
    // next sweep
    hipStream_t side;
    hipEvent_t fork, join;
    void *ws;
    size_t ws_bytes;
    bool own_ws;
    hipGraph_t graph;
    hipGraphExec_t gexec;
    bool graph_tried;
    uint64_t next_sweep;
    uint64_t first_valid;
    int device;
};

namespace {

constexpr int64_t kDefaultBatchRing = 1024;

int batch_group(const Dev &d) { return (d.q ? 2 : 0) + (d.tw == 64 ? 0 : 1); }

struct BatchPlan {
    std::vector<sw_config> cfg;
    std::vector<size_t> base;   // workspace offset of every replica
    std::vector<uint8_t> lds;   // merge in LDS
    size_t devs, maps, total;
    size_t map_words;
};

// Validates the replica table and lays out the batch workspace: the
// replicas' buffers one after another, then the Dev table and the maps.
// q: NULL for Ising replicas, else the Potts q of every replica (0: Ising,
// 2..8: Potts).  tiles: NULL (every replica takes `tile`), else the tile
// width of every replica (0 automatic, 32, 64).  merge: NULL (automatic),
// else per replica SW_MERGE_AUTO / SW_MERGE_LDS / SW_MERGE_GLOBAL.
int plan_batch(int32_t n, const int32_t *L, const double *beta, const double *J, const uint64_t *seed,
               const int32_t *q, const int32_t *tiles, const int32_t *merge, int32_t init, int64_t ring,
               int32_t tile, BatchPlan *p) {
    if (n < 1 || n > swmi::kMaxReplicas)
        return fail(SW_EINVAL, "the number of replicas must be in [1, " + std::to_string(swmi::kMaxReplicas) + "]");
    if (!L || !beta || !J || !seed) return fail(SW_EINVAL, "replica arrays must not be NULL");
    if (init != SW_INIT_HOT && init != SW_INIT_COLD) return fail(SW_EINVAL, "init must be SW_INIT_HOT or SW_INIT_COLD");
    if (tile != 0 && tile != 32 && tile != 64) return fail(SW_EINVAL, "tile must be 0, 32 or 64");
    p->cfg.assign((size_t)n, sw_config{});
    p->base.assign((size_t)n, 0);
    p->lds.assign((size_t)n, 0);
    size_t off = 0;
    swmi::BatchMaps m[kBatchGroups];
    for (int32_t r = 0; r < n; ++r) {
        const std::string who = "replica " + std::to_string(r) + ": ";
        sw_config &c = p->cfg[(size_t)r];
        sw_config_init(&c, L[r], beta[r], J[r], seed[r]);
        c.q = q ? q[r] : 0;
        if (c.q != 0 && (c.q < 2 || c.q > swmi::kMaxQ)) return fail(SW_EINVAL, who + "Potts q must be 0 or in [2, 8]");
        c.init = init;
        c.tile = tiles ? tiles[r] : tile;
        if (c.tile != 0 && c.tile != 32 && c.tile != 64) return fail(SW_EINVAL, who + "tile must be 0, 32 or 64");
        c.ring = ring > 0 ? ring : kDefaultBatchRing;
        const int rc = validate(&c);
        if (rc != SW_OK) return fail(rc, who + swmi::last_error());
        c.tile = resolve_tile(c);
        const int32_t mg = merge ? merge[r] : SW_MERGE_AUTO;
        if (mg != SW_MERGE_AUTO && mg != SW_MERGE_LDS && mg != SW_MERGE_GLOBAL)
            return fail(SW_EINVAL, who + "merge must be SW_MERGE_AUTO, SW_MERGE_LDS or SW_MERGE_GLOBAL");
        const uint32_t nt = (uint32_t)((c.L / c.tile) * (c.L / c.tile));
        if (mg == SW_MERGE_LDS && nt > swmi::kSmallTiles)
            return fail(SW_EINVAL, who + "the LDS merge takes at most " + std::to_string(swmi::kSmallTiles) + " tiles");
        p->lds[(size_t)r] = (mg != SW_MERGE_GLOBAL && nt <= swmi::kSmallTiles) ? 1u : 0u;
        const Layout lo = layout_of(c);
        p->base[(size_t)r] = off;
        off = align_up(off + lo.total);
        const Dev d = make_dev(c, nullptr, lo);
        m[batch_group(d)].add((uint32_t)r, d, p->lds[(size_t)r] != 0);
    }
    p->map_words = 0;
    for (const swmi::BatchMaps &g : m) p->map_words += g.words();
    auto take = [&](size_t bytes) {
        const size_t at = off;
        off = align_up(off + bytes);
        return at;
    };
    p->devs = take((size_t)n * sizeof(Dev));
    p->maps = take(p->map_words * 4);
    p->total = off;
    return SW_OK;
}

int batch_device(const sw_batch *b) {
    int cur = -1;
    HIP_TRY(hipGetDevice(&cur));
    if (cur != b->device) HIP_TRY(hipSetDevice(b->device));
    return SW_OK;
}

void batch_drop_graph(sw_batch *b) {
    if (b->gexec) (void)hipGraphExecDestroy(b->gexec);
    if (b->graph) (void)hipGraphDestroy(b->graph);
    b->gexec = nullptr;
    b->graph = nullptr;
    b->graph_tried = false;
}

hipError_t batch_launch_sweep(const sw_batch *b) {
    bool small = false, large = false;
    for (int g = 0; g < kBatchGroups; ++g) {
        small = small || b->bd[g].nsmall > 0;
        large = large || b->bd[g].n > 0;
    }
    hipError_t e = hipSuccess;
    for (int g = 0; g < kBatchGroups && e == hipSuccess; ++g) e = swmi::launch_batch_stage(b->bd[g], 0, b->stream);
    // the LDS merges beside the global merge when both kinds are present
    const bool fork = small && large && b->side != nullptr;
    hipStream_t ss = fork ? b->side : b->stream;
    if (e == hipSuccess && fork) e = hipEventRecord(b->fork, b->stream);
    if (e == hipSuccess && fork) e = hipStreamWaitEvent(b->side, b->fork, 0);
    for (int g = 0; g < kBatchGroups && e == hipSuccess; ++g) e = swmi::launch_batch_smerge(b->bd[g], ss);
    for (int stage = 1; stage < swmi::kStages && e == hipSuccess; ++stage)
        for (int g = 0; g < kBatchGroups && e == hipSuccess; ++g) e = swmi::launch_batch_stage(b->bd[g], stage, b->stream);
    if (e == hipSuccess && fork) e = hipEventRecord(b->join, b->side);
    if (e == hipSuccess && fork) e = hipStreamWaitEvent(b->stream, b->join, 0);
    return e;
}

// One batched sweep captured as a graph; on any capture failure the kernels
// are launched directly.
void batch_ensure_graph(sw_batch *b) {
    if (b->graph_tried) return;
    b->graph_tried = true;
    if (b->stream == nullptr) return;
    if (hipStreamBeginCapture(b->stream, hipStreamCaptureModeThreadLocal) != hipSuccess) {
        (void)hipGetLastError();
        return;
    }
    const hipError_t le = batch_launch_sweep(b);
    hipGraph_t g = nullptr;
    const hipError_t ce = hipStreamEndCapture(b->stream, &g);
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
    b->graph = g;
    b->gexec = ge;
}

int batch_check_replica(const sw_batch *b, int32_t r) {
    if (!b) return fail(SW_EINVAL, "batch is NULL");
    if (r < 0 || (size_t)r >= b->dev.size()) return fail(SW_ERANGE, "replica index out of range");
    return SW_OK;
}

size_t batch_bytes(int32_t n, const int32_t *L, const int32_t *q, const int32_t *tiles, const int32_t *merge,
                   int64_t ring, int32_t tile) {
    if (n < 1 || n > swmi::kMaxReplicas || !L) return 0;
    std::vector<double> beta((size_t)n, 0.0), J((size_t)n, 1.0);
    std::vector<uint64_t> seed((size_t)n, 0u);
    BatchPlan p;
    if (plan_batch(n, L, beta.data(), J.data(), seed.data(), q, tiles, merge, SW_INIT_HOT, ring, tile, &p) != SW_OK)
        return 0;
    return p.total;
}

int batch_create(int32_t n, const int32_t *L, const double *beta, const double *J, const uint64_t *seed,
                 const int32_t *q, const int32_t *tiles, const int32_t *merge, int32_t init, int64_t ring,
                 int32_t tile, void *dev_workspace, size_t ws_bytes, void *hip_stream, sw_batch **out) {
    if (!out) return fail(SW_EINVAL, "out is NULL");
    *out = nullptr;
    BatchPlan p;
    int rc = plan_batch(n, L, beta, J, seed, q, tiles, merge, init, ring, tile, &p);
    if (rc != SW_OK) return rc;
    if (dev_workspace && ws_bytes < p.total)
        return fail(SW_ENOMEM, "workspace too small: need " + std::to_string(p.total) + " bytes");
    if (dev_workspace && ((uintptr_t)dev_workspace % kAlign) != 0)
        return fail(SW_EINVAL, "workspace must be 256-byte aligned");
    sw_batch *b = new (std::nothrow) sw_batch();
    if (!b) return fail(SW_ENOMEM, "host allocation failed");
    hipError_t e = hipGetDevice(&b->device);
    if (e != hipSuccess) {
        delete b;
        return hip_fail(e, "hipGetDevice");
    }
    if (dev_workspace) {
        b->ws = dev_workspace;
        b->ws_bytes = ws_bytes;
        b->own_ws = false;
        b->stream = (hipStream_t)hip_stream;
        b->own_stream = false;
    } else {
        e = hipMalloc(&b->ws, p.total);
        if (e != hipSuccess) {
            (void)hipGetLastError();
            delete b;
            return fail(SW_ENOMEM, "hipMalloc of " + std::to_string(p.total) + " bytes failed");
        }
        b->ws_bytes = p.total;
        b->own_ws = true;
        if (hip_stream) {
            b->stream = (hipStream_t)hip_stream;
            b->own_stream = false;
        } else {
            e = hipStreamCreateWithFlags(&b->stream, hipStreamNonBlocking);
            if (e != hipSuccess) {
                (void)hipFree(b->ws);
                delete b;
                return hip_fail(e, "hipStreamCreateWithFlags");
            }
            b->own_stream = true;
        }
    }
    if (b->stream != nullptr) {  // (the legacy null stream runs everything in order on itself)
        e = hipStreamCreateWithFlags(&b->side, hipStreamNonBlocking);
        if (e == hipSuccess) e = hipEventCreateWithFlags(&b->fork, hipEventDisableTiming);
        if (e == hipSuccess) e = hipEventCreateWithFlags(&b->join, hipEventDisableTiming);
        if (e != hipSuccess) {
            rc = hip_fail(e, "creating the batch's second stream");
            sw_batch_destroy(b);
            return rc;
        }
    }
    char *base = (char *)b->ws;
    b->cfg = p.cfg;
    b->lds = p.lds;
    b->dev.resize(p.cfg.size());
    swmi::BatchMaps m[kBatchGroups];
    for (size_t r = 0; r < p.cfg.size(); ++r) {
        b->dev[r] = make_dev(p.cfg[r], base + p.base[r], layout_of(p.cfg[r]));
        m[batch_group(b->dev[r])].add((uint32_t)r, b->dev[r], p.lds[r] != 0);
    }
    std::vector<uint32_t> host;
    host.reserve(p.map_words);
    const uint32_t *dmaps = (const uint32_t *)(base + p.maps);
    for (int g = 0; g < kBatchGroups; ++g) {
        swmi::BatchDev &bd = b->bd[g];
        bd = swmi::BatchDev{};
        bd.devs = (const Dev *)(base + p.devs);
        bd.tw = (g & 1) ? 32u : 64u;
        bd.potts = g >= 2 ? 1u : 0u;
        m[g].emit(host, dmaps, bd);
    }

    e = hipMemsetAsync(b->ws, 0, p.total, b->stream);
    if (e == hipSuccess)
        e = hipMemcpyAsync(base + p.devs, b->dev.data(), b->dev.size() * sizeof(Dev), hipMemcpyHostToDevice,
                           b->stream);
    if (e == hipSuccess && !host.empty())
        e = hipMemcpyAsync(base + p.maps, host.data(), host.size() * 4, hipMemcpyHostToDevice, b->stream);
    if (e == hipSuccess) e = hipStreamSynchronize(b->stream);
    if (e != hipSuccess) {
        rc = hip_fail(e, "setting up the batch workspace");
        sw_batch_destroy(b);
        return rc;
    }
    rc = sw_batch_reset(b, init);
    if (rc != SW_OK) {
        const std::string msg = swmi::last_error();
        sw_batch_destroy(b);
        return fail(rc, msg);
    }
    *out = b;
    return SW_OK;
}

}  // namespace

extern "C" {

size_t sw_batch_workspace_bytes(int32_t n, const int32_t *L, int64_t ring, int32_t tile) {
    return batch_bytes(n, L, nullptr, nullptr, nullptr, ring, tile);
}

size_t sw_batch_workspace_bytes_potts(int32_t n, const int32_t *L, const int32_t *q, int64_t ring, int32_t tile) {
    if (!q) return 0;
    return batch_bytes(n, L, q, nullptr, nullptr, ring, tile);
}

size_t sw_batch_workspace_bytes_ex(int32_t n, const int32_t *L, const int32_t *q, const int32_t *tiles,
                                   const int32_t *merge, int64_t ring) {
    return batch_bytes(n, L, q, tiles, merge, ring, 0);
}

int sw_batch_create(int32_t n, const int32_t *L, const double *beta, const double *J, const uint64_t *seed,
                    int32_t init, int64_t ring, int32_t tile, void *dev_workspace, size_t ws_bytes,
                    void *hip_stream, sw_batch **out) {
    return batch_create(n, L, beta, J, seed, nullptr, nullptr, nullptr, init, ring, tile, dev_workspace, ws_bytes,
                        hip_stream, out);
}

int sw_batch_create_potts(int32_t n, const int32_t *L, const double *beta, const double *J, const uint64_t *seed,
                          const int32_t *q, int32_t init, int64_t ring, int32_t tile, void *dev_workspace,
                          size_t ws_bytes, void *hip_stream, sw_batch **out) {
    if (!q) {
        if (out) *out = nullptr;
        return fail(SW_EINVAL, "q must not be NULL");
    }
    for (int32_t r = 0; n > 0 && r < n; ++r)
        if (q[r] < 2 || q[r] > swmi::kMaxQ) {
            if (out) *out = nullptr;
            return fail(SW_EINVAL, "replica " + std::to_string(r) + ": Potts q must be in [2, 8]");
        }
    return batch_create(n, L, beta, J, seed, q, nullptr, nullptr, init, ring, tile, dev_workspace, ws_bytes,
                        hip_stream, out);
}

int sw_batch_create_ex(int32_t n, const int32_t *L, const double *beta, const double *J, const uint64_t *seed,
                       const int32_t *q, const int32_t *tiles, const int32_t *merge, int32_t init, int64_t ring,
                       void *dev_workspace, size_t ws_bytes, void *hip_stream, sw_batch **out) {
    return batch_create(n, L, beta, J, seed, q, tiles, merge, init, ring, 0, dev_workspace, ws_bytes, hip_stream,
                        out);
}

int sw_batch_reset(sw_batch *b, int32_t init_mode) {
    if (!b) return fail(SW_EINVAL, "batch is NULL");
    if (init_mode != SW_INIT_HOT && init_mode != SW_INIT_COLD)
        return fail(SW_EINVAL, "init_mode must be SW_INIT_HOT or SW_INIT_COLD");
    int rc = batch_device(b);
    if (rc != SW_OK) return rc;
    HIP_TRY(hipStreamSynchronize(b->stream));
    const uint64_t zero = 0;
    for (const Dev &d : b->dev) {
        HIP_TRY(hipMemcpyAsync(d.tdev, &zero, sizeof(zero), hipMemcpyHostToDevice, b->stream));
        HIP_TRY(swmi::launch_init(d, init_mode == SW_INIT_COLD ? 1 : 0, b->stream));
    }
    HIP_TRY(hipStreamSynchronize(b->stream));
    b->next_sweep = 0;
    b->first_valid = 0;
    return SW_OK;
}

int sw_batch_sweep(sw_batch *b, int64_t n) {
    if (!b) return fail(SW_EINVAL, "batch is NULL");
    if (n < 0) return fail(SW_EINVAL, "n must be >= 0");
    if (n == 0) return SW_OK;
    int rc = batch_device(b);
    if (rc != SW_OK) return rc;
    batch_ensure_graph(b);
    for (int64_t i = 0; i < n; ++i) {
        if (b->gexec)
            HIP_TRY(hipGraphLaunch(b->gexec, b->stream));
        else
            HIP_TRY(batch_launch_sweep(b));
    }
    for (int g = 0; g < kBatchGroups; ++g) HIP_TRY(swmi::launch_batch_resolve(b->bd[g], b->stream));
    b->next_sweep += (uint64_t)n;
    return SW_OK;
}

int sw_batch_sync(sw_batch *b) {
    if (!b) return fail(SW_EINVAL, "batch is NULL");
    int rc = batch_device(b);
    if (rc != SW_OK) return rc;
    HIP_TRY(hipStreamSynchronize(b->stream));
    return SW_OK;
}

int sw_batch_series(sw_batch *b, int32_t r, int64_t first, int64_t count, sw_obs *out) {
    int rc = batch_check_replica(b, r);
    if (rc != SW_OK) return rc;
    if (count < 0 || (count > 0 && !out)) return fail(SW_EINVAL, "bad count or NULL out");
    if (count == 0) return SW_OK;
    if (first < (int64_t)b->first_valid || first + count > (int64_t)b->next_sweep)
        return fail(SW_ERANGE, "records requested outside the sweeps run since the last reset");
    const Dev &d = b->dev[(size_t)r];
    const uint64_t cap = d.ring_cap;
    if ((uint64_t)(b->next_sweep - (uint64_t)first) > cap) return fail(SW_ERANGE, "records requested have left the ring");
    rc = batch_device(b);
    if (rc != SW_OK) return rc;
    HIP_TRY(hipStreamSynchronize(b->stream));
    int64_t done = 0;
    while (done < count) {
        const uint64_t idx = (uint64_t)(first + done) % cap;
        const int64_t chunk = (int64_t)std::min<uint64_t>((uint64_t)(count - done), cap - idx);
        HIP_TRY(hipMemcpyAsync(out + done, d.ring + idx, (size_t)chunk * sizeof(sw_obs), hipMemcpyDeviceToHost,
                               b->stream));
        done += chunk;
    }
    HIP_TRY(hipStreamSynchronize(b->stream));
    return SW_OK;
}

int sw_batch_observables(sw_batch *b, sw_obs *out) {
    if (!b || !out) return fail(SW_EINVAL, "batch or out is NULL");
    if (b->next_sweep == b->first_valid) return fail(SW_ESTATE, "no sweep has run since the last reset");
    int rc = batch_device(b);
    if (rc != SW_OK) return rc;
    HIP_TRY(hipStreamSynchronize(b->stream));
    const uint64_t t = b->next_sweep - 1u;
    for (size_t r = 0; r < b->dev.size(); ++r) {
        const Dev &d = b->dev[r];
        HIP_TRY(hipMemcpyAsync(out + r, d.ring + t % d.ring_cap, sizeof(sw_obs), hipMemcpyDeviceToHost, b->stream));
    }
    HIP_TRY(hipStreamSynchronize(b->stream));
    return SW_OK;
}

int sw_batch_get_spins(sw_batch *b, int32_t r, int8_t *host, int64_t n) {
    int rc = batch_check_replica(b, r);
    if (rc != SW_OK) return rc;
    if (!host) return fail(SW_EINVAL, "host is NULL");
    const Dev &d = b->dev[(size_t)r];
    if (n != (int64_t)d.L * d.L) return fail(SW_ERANGE, "n must equal L*L of the replica");
    rc = batch_device(b);
    if (rc != SW_OK) return rc;
    HIP_TRY(hipMemcpyAsync(host, d.spins[b->next_sweep & 1u], (size_t)n, hipMemcpyDeviceToHost, b->stream));
    HIP_TRY(hipStreamSynchronize(b->stream));
    return SW_OK;
}

int32_t sw_batch_size(const sw_batch *b) { return b ? (int32_t)b->dev.size() : 0; }
int64_t sw_batch_next_sweep(const sw_batch *b) { return b ? (int64_t)b->next_sweep : -1; }
int32_t sw_batch_lattice(const sw_batch *b, int32_t r) {
    return (b && r >= 0 && (size_t)r < b->dev.size()) ? (int32_t)b->dev[(size_t)r].L : 0;
}
uint32_t sw_batch_threshold(const sw_batch *b, int32_t r) {
    return (b && r >= 0 && (size_t)r < b->dev.size()) ? b->dev[(size_t)r].T : 0u;
}
int32_t sw_batch_tile(const sw_batch *b) {
    if (!b || b->dev.empty()) return 0;
    const uint32_t tw = b->dev[0].tw;
    for (const Dev &d : b->dev)
        if (d.tw != tw) return 0;
    return (int32_t)tw;
}
int32_t sw_batch_replica_tile(const sw_batch *b, int32_t r) {
    return (b && r >= 0 && (size_t)r < b->dev.size()) ? (int32_t)b->dev[(size_t)r].tw : 0;
}
int32_t sw_batch_replica_merge(const sw_batch *b, int32_t r) {
    if (!b || r < 0 || (size_t)r >= b->dev.size()) return 0;
    return b->lds[(size_t)r] ? SW_MERGE_LDS : SW_MERGE_GLOBAL;
}

void sw_batch_destroy(sw_batch *b) {
    if (!b) return;
    (void)batch_device(b);
    (void)hipStreamSynchronize(b->stream);
    batch_drop_graph(b);
    if (b->side) {
        (void)hipStreamSynchronize(b->side);
        (void)hipStreamDestroy(b->side);
    }
    if (b->fork) (void)hipEventDestroy(b->fork);
    if (b->join) (void)hipEventDestroy(b->join);
    if (b->own_ws && b->ws) (void)hipFree(b->ws);
    if (b->own_stream && b->stream) (void)hipStreamDestroy(b->stream);
    delete b;
}

}  // extern "C"
