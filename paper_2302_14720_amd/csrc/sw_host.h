// sw_host.h -- host-side helpers shared by the C ABI (sw_api.hip) and the
// serving runtime (sw_server.hip): error reporting, validation, and the
// carving of one lattice's device buffers out of a workspace.
#pragma once

#include <string>

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

}  // namespace swmi

#define HIP_TRY(expr)                                             \
    do {                                                          \
        hipError_t e_ = (expr);                                   \
        if (e_ != hipSuccess) return swmi::hip_fail(e_, #expr);   \
    } while (0)
