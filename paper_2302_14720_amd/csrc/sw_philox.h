// sw_philox.h -- the counter-based generator every random decision of a
// sweep uses (device side; the test oracle has its own implementation).
#pragma once

#include <hip/hip_runtime.h>
#include <stdint.h>

namespace swmi {

// Philox4x32-10 (Salmon et al., SC'11): ten rounds of two 32x32->64-bit
// products; the key advances by the Weyl constants between rounds.
__device__ __forceinline__ void philox10(uint32_t &x0, uint32_t &x1, uint32_t &x2,
                                         uint32_t &x3, uint32_t k0, uint32_t k1) {
#pragma unroll
    for (int r = 0; r < 10; ++r) {
        const uint64_t pa = (uint64_t)0xD2511F53u * x0;
        const uint64_t pb = (uint64_t)0xCD9E8D57u * x2;
        // three-input xor in one v_bitop3 (truth table 0x96)
        const uint32_t n0 = __builtin_amdgcn_bitop3_b32((uint32_t)(pb >> 32), x1, k0, 0x96);
        const uint32_t n2 = __builtin_amdgcn_bitop3_b32((uint32_t)(pa >> 32), x3, k1, 0x96);
        x1 = (uint32_t)pb;
        x3 = (uint32_t)pa;
        x0 = n0;
        x2 = n2;
        k0 += 0x9E3779B9u;
        k1 += 0xBB67AE85u;
    }
}

// New spin (+1 / -1) of the cluster whose smallest site is r in sweep t:
// bit r mod 128 of the 128-bit output for counter {r >> 7, t, 1, 0}.
__device__ __forceinline__ int8_t cluster_spin(uint32_t r, uint32_t t, uint32_t k0, uint32_t k1) {
    uint32_t w0 = r >> 7, w1 = t, w2 = 1u, w3 = 0u;
    philox10(w0, w1, w2, w3, k0, k1);
    const uint32_t q = (r >> 5) & 3u;
    const uint32_t w = q == 0 ? w0 : q == 1 ? w1 : q == 2 ? w2 : w3;
    return ((w >> (r & 31u)) & 1u) ? (int8_t)-1 : (int8_t)1;
}

// New value (0..q-1) of the Potts cluster whose smallest site is r in sweep
// t: floor(w q / 2^32) of word r mod 4 of the output for counter
// {r >> 2, t, 3, 0}.
__device__ __forceinline__ int8_t potts_spin(uint32_t r, uint32_t t, uint32_t q, uint32_t k0, uint32_t k1) {
    uint32_t w0 = r >> 2, w1 = t, w2 = 3u, w3 = 0u;
    philox10(w0, w1, w2, w3, k0, k1);
    const uint32_t qq = r & 3u;
    const uint32_t w = qq == 0 ? w0 : qq == 1 ? w1 : qq == 2 ? w2 : w3;
    return (int8_t)(((uint64_t)w * q) >> 32);
}

}  // namespace swmi
