// sw_uf.h -- lock-free union-find on parent arrays in LDS (workgroup scope)
// and in global memory (device scope).  Roots are the smallest index of
// their set: a root is linked under the root with the smaller index, so
// every parent is smaller than its child and the structure stays a forest
// whatever order concurrent unions run in.
#pragma once

#include <hip/hip_runtime.h>
#include <stdint.h>

namespace swmi {

__device__ __forceinline__ uint32_t lds_load(uint32_t *p) {
    return __hip_atomic_load(p, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_WORKGROUP);
}
// Path halving lowers entries with atomicMin: a plain store could overwrite
// a fully compressed entry (the root) with a larger ancestor read earlier by
// another thread, whereas with min-updates every entry only ever decreases
// towards its root.
__device__ __forceinline__ uint32_t lds_find(uint32_t *par, uint32_t a) {
    while (true) {
        const uint32_t p = lds_load(&par[a]);
        if (p == a) return a;
        const uint32_t gp = lds_load(&par[p]);
        if (gp == p) return p;
        atomicMin(&par[a], gp);
        a = gp;
    }
}
// Root of a once the unions are done (read-only; parents are the low 16
// bits, the high half of a root's word may hold other data).
__device__ __forceinline__ uint32_t lds_root(const uint32_t *par, uint32_t a) {
    while (true) {
        const uint32_t p = par[a] & 0xFFFFu;
        if (p == a) return a;
        a = p;
    }
}
__device__ __forceinline__ void lds_union(uint32_t *par, uint32_t a, uint32_t b) {
    while (true) {
        a = lds_find(par, a);
        b = lds_find(par, b);
        if (a == b) return;
        if (a > b) { const uint32_t tmp = a; a = b; b = tmp; }
        uint32_t expected = b;
        if (__hip_atomic_compare_exchange_strong(&par[b], &expected, a, __ATOMIC_RELAXED,
                                                 __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_WORKGROUP))
            return;
    }
}

__device__ __forceinline__ uint32_t g_load(uint32_t *p) {
    return __hip_atomic_load(p, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
}
__device__ __forceinline__ void g_store(uint32_t *p, uint32_t v) {
    __hip_atomic_store(p, v, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
}
// Union in global memory.  Both finds advance together, one level per
// round of loads (their loads overlap), with path splitting: every entry
// passed is re-pointed at its grandparent, which is an ancestor whatever
// other unions did meanwhile.  The two paths meeting below their roots (a
// common parent) already shows one set.
__device__ __forceinline__ void g_union(uint32_t *par, uint32_t a, uint32_t b) {
    while (true) {
        uint32_t pa = g_load(&par[a]), pb = g_load(&par[b]);
        while (pa != a || pb != b) {
            if (pa == pb) return;
            const uint32_t ga = g_load(&par[pa]), gb = g_load(&par[pb]);
            if (ga != pa) g_store(&par[a], ga);
            if (gb != pb) g_store(&par[b], gb);
            a = pa;
            b = pb;
            pa = ga;
            pb = gb;
        }
        if (a == b) return;
        if (a > b) { const uint32_t tmp = a; a = b; b = tmp; }
        uint32_t expected = b;
        if (__hip_atomic_compare_exchange_strong(&par[b], &expected, a, __ATOMIC_RELAXED,
                                                 __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT))
            return;
    }
}

}  // namespace swmi
