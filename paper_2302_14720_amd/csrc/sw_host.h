// sw_host.h -- host-side helpers shared by the C ABI (sw_api.hip) and the
// serving runtime (sw_server.hip): error reporting, validation, and the
// carving of one lattice's device buffers out of a workspace.
#pragma once

#include <string>
#include <vector>

#include "sw_internal.h"

namespace swmi {

constexpr size_t kAlign = 256;
constexpr int64_t kDefaultRing = 4096;

inline size_t align_up(size_t v) { return (v + kAlign - 1) & ~(kAlign - 1); }

// Sets the thread's last-error message and returns code.
int fail(int code, const std::string &msg);
int hip_fail(hipError_t e, const char *what);
// The thread's last-error message.
const std::string &last_error();

// Bond probability p = 1 - exp(-2 beta J) as a 32-bit threshold.
uint32_t bond_threshold(double beta, double J);

struct Layout {
    size_t spins[2], parent[2], nk[2], key, nsize, rspin, edge, xb, tpart, gpart, acc, tdev, ring, labels,
        dense, le_mask, le_cnt, le_rsp, le_ctl, bface, total;
};

int resolve_tile(const sw_config &c);
int validate(const sw_config *c);
Layout layout_of(const sw_config &c);
Dev make_dev(const sw_config &c, char *base, const Layout &lo);

// Host-side work maps of one launch group of a batch (one tile width, Ising
// or Potts): add() files the replica in slot `slot` of the Dev table under
// the global merge, or under the LDS merge (k_smerge_b) when `small` is set
// and it has at most kSmallTiles tiles; emit() appends the maps to `host`
// (which will be copied to dev_base) and points the BatchDev at them.
struct BatchMaps {
    std::vector<uint32_t> t, w, wn, g, u, r, s, a;  // w / wn: tiles with an E / N group edge
    void add(uint32_t slot, const Dev &d, bool small) {
        const uint32_t tag = slot << kMapShift;
        a.push_back(slot);
        for (uint32_t i = 0; i < d.ntiles; ++i) t.push_back(tag | i);
        if (small && d.ntiles <= kSmallTiles) {
            s.push_back(slot);
            return;
        }
        r.push_back(slot);
        // edges between kUG x kUG groups of tiles (those inside a group are
        // joined by k_ulocal): the last tile column / row of every group
        for (uint32_t i = 0; i < d.ntiles; ++i) {
            const uint32_t tx = i % d.ntx, ty = i / d.ntx;
            if (tx % kUG == kUG - 1u || tx + 1u == d.ntx) w.push_back(tag | i);
            if (ty % kUG == kUG - 1u || ty + 1u == d.ntx) wn.push_back(tag | i);
        }
        for (uint32_t i = 0; i < d.ngroups; ++i) g.push_back(tag | i);
        const uint32_t ngx = (d.ntx + kUG - 1u) / kUG;
        for (uint32_t i = 0; i < ngx * ngx; ++i) u.push_back(tag | i);
    }
    size_t words() const {
        return t.size() + ((w.size() + wn.size() + 3u) & ~size_t(3)) + g.size() + u.size() + r.size() + s.size() +
               a.size();
    }
    void emit(std::vector<uint32_t> &host, const uint32_t *dev_base, BatchDev &b) const {
        const size_t at = host.size();
        b.ntiles = (uint32_t)t.size();
        b.nwmap = (uint32_t)((w.size() + wn.size() + 3u) & ~size_t(3));
        b.nwE = (uint32_t)w.size();
        b.ngroups = (uint32_t)g.size();
        b.nugroups = (uint32_t)u.size();
        b.n = (uint32_t)r.size();
        b.nsmall = (uint32_t)s.size();
        b.nall = (uint32_t)a.size();
        host.insert(host.end(), t.begin(), t.end());
        host.insert(host.end(), w.begin(), w.end());
        host.insert(host.end(), wn.begin(), wn.end());
        host.resize(at + b.ntiles + b.nwmap, kMapNone);
        host.insert(host.end(), g.begin(), g.end());
        host.insert(host.end(), u.begin(), u.end());
        host.insert(host.end(), r.begin(), r.end());
        host.insert(host.end(), s.begin(), s.end());
        host.insert(host.end(), a.begin(), a.end());
        const uint32_t *p = dev_base + at;
        b.tmap = p;
        b.wmap = p + b.ntiles;
        b.gmap = b.wmap + b.nwmap;
        b.umap = b.gmap + b.ngroups;
        b.rmap = b.umap + b.nugroups;
        b.smap = b.rmap + b.n;
        b.amap = b.smap + b.nsmall;
    }
};

}  // namespace swmi

#define HIP_TRY(expr)                                             \
    do {                                                          \
        hipError_t e_ = (expr);                                   \
        if (e_ != hipSuccess) return swmi::hip_fail(e_, #expr);   \
    } while (0)
