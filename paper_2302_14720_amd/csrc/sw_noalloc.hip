// sw_noalloc.hip -- one Swendsen-Wang sweep that allocates nothing, for
// callers that cannot allocate device memory (code under HIP graph capture,
// tight serving loops, harnesses that forbid allocation).
//
// Every buffer of the sweep other than the caller's spins and record (the
// second spin buffer, node tables, partials, accumulator, sweep index, one
// record) lives in `scratch`, a static device array of kScratchBytes that
// each GPU holds until the process ends.  Host code never uses the array's
// name as an address: hipGetSymbolAddress gives each device's own address
// once, at the first call on that device, and the kernels get that pointer.
// All calls on one GPU share that GPU's array, so calls that overlap on one
// GPU (different streams, or threads) race; calls on one stream are ordered.
#include <algorithm>
#include <mutex>
#include <string>

#include "sw_host.h"

namespace {

constexpr size_t kScratchBytes = (size_t)16 << 20;  // L = 2048 needs 12.7 MiB
constexpr int32_t kNoallocMaxL = 2048;
constexpr int kMaxDevices = 64;

static __device__ __align__(256) unsigned char scratch[kScratchBytes];

std::mutex g_scratch_mu;
void *g_scratch_ptr[kMaxDevices] = {};

// This device's address of `scratch` (looked up once per device, with the
// device current).
int scratch_of(int device, void **out) {
    if (device < 0 || device >= kMaxDevices) return swmi::fail(SW_EINVAL, "device index out of range");
    std::lock_guard<std::mutex> lock(g_scratch_mu);
    if (!g_scratch_ptr[device]) {
        void *p = nullptr;
        const hipError_t e = hipGetSymbolAddress(&p, HIP_SYMBOL(scratch));
        if (e != hipSuccess) return swmi::hip_fail(e, "hipGetSymbolAddress(scratch)");
        if (!p) return swmi::fail(SW_EHIP, "hipGetSymbolAddress(scratch) gave a null address");
        g_scratch_ptr[device] = p;
    }
    *out = g_scratch_ptr[device];
    return SW_OK;
}

// Sets the sweep index and clears what a sweep expects to start at zero:
// the record accumulator, and the node counts of the previous parity (the
// caller's spins are final values, never node codes).
__global__ __launch_bounds__(256) void k_na_prepare(swmi::Dev d, uint64_t t) {
    const uint32_t i = blockIdx.x * 256u + threadIdx.x;
    const uint32_t pp = (uint32_t)(t & 1u) ^ 1u;
    if (i == 0u) *d.tdev = t;
    if (i < (uint32_t)swmi::kAccWords) d.acc[i] = 0u;
    for (uint32_t k = i; k < d.ntiles; k += gridDim.x * 256u) d.nk[pp][k] = 0u;
}

// Final spins and the record back to the caller's buffers.
__global__ __launch_bounds__(256) void k_na_finish(swmi::Dev d, uint64_t t, int8_t *spins, sw_obs *rec) {
    const size_t n16 = d.nsite / 16u;
    const uint4 *src = reinterpret_cast<const uint4 *>(d.spins[(t + 1u) & 1u]);
    uint4 *dst = reinterpret_cast<uint4 *>(spins);
    for (size_t i = blockIdx.x * (size_t)256 + threadIdx.x; i < n16; i += (size_t)gridDim.x * 256) dst[i] = src[i];
    if (blockIdx.x == 0u) {
        const uint32_t *rs = reinterpret_cast<const uint32_t *>(&d.ring[0]);
        uint32_t *rd = reinterpret_cast<uint32_t *>(rec);
        for (uint32_t w = threadIdx.x; w < sizeof(sw_obs) / 4u; w += 256u) rd[w] = rs[w];
    }
}

}  // namespace

extern "C" int sw_sweep_noalloc(int32_t L, double beta, double J, uint64_t seed, uint64_t t, int8_t *spins,
                                sw_obs *rec, void *hip_stream) {
    using namespace swmi;
    if (!spins || !rec) return fail(SW_EINVAL, "spins and rec must be device pointers");
    if (L > kNoallocMaxL) return fail(SW_ERANGE, "L must be at most 2048 here (the static scratch holds 16 MiB)");
    sw_config c;
    sw_config_init(&c, L, beta, J, seed);
    c.ring = 1;
    int rc = validate(&c);
    if (rc != SW_OK) return rc;
    const Layout lo = layout_of(c);
    if (lo.total > kScratchBytes) return fail(SW_ERANGE, "lattice needs more than the 16 MiB static scratch");
    if (((uintptr_t)spins % 16u) != 0u) return fail(SW_EINVAL, "spins must be 16-byte aligned");
    if (((uintptr_t)rec % 8u) != 0u) return fail(SW_EINVAL, "rec must be 8-byte aligned");
    int device = -1;
    HIP_TRY(hipGetDevice(&device));
    void *base = nullptr;
    rc = scratch_of(device, &base);
    if (rc != SW_OK) return rc;
    Dev d = make_dev(c, (char *)base, lo);
    // the caller's spins are the input parity; the sweep's output parity is
    // the scratch's first spin buffer
    d.spins[(t + 1u) & 1u] = (int8_t *)((char *)base + lo.spins[0]);
    d.spins[t & 1u] = spins;
    hipStream_t s = (hipStream_t)hip_stream;
    const uint32_t g = (d.ntiles + 255u) / 256u;
    k_na_prepare<<<g > 0u ? g : 1u, 256, 0, s>>>(d, t);
    HIP_TRY(hipGetLastError());
    HIP_TRY(launch_sweep(d, s));
    HIP_TRY(launch_resolve(d, s));
    const size_t n16 = d.nsite / 16u;
    const uint32_t gf = (uint32_t)std::min<size_t>((n16 + 255u) / 256u, 4096u);
    k_na_finish<<<gf, 256, 0, s>>>(d, t, spins, rec);
    HIP_TRY(hipGetLastError());
    return SW_OK;
}
