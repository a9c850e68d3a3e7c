// Integer-ALU rate probes (measurement aid): the throughput of the instruction mixes the layer
// kernels run, measured on the whole chip with no memory traffic, for the "alu" roofs of the
// benchmark.
//
// Each thread keeps PR_CHAINS independent chains in registers and runs `iters` rounds; every
// round applies one operation of the probed kind to every chain, so the compiler can neither
// drop nor merge the work (each result feeds the next round, and the sums go to a sink).  The
// grid fills every CU at the occupancy the kernels reach.  Kinds:
//   HE_PROBE_BFLY    the Shoup Cooley-Tukey butterfly of the NTT kernels (lazy, values < 4q)
//   HE_PROBE_GSBFLY  the Gentleman-Sande butterfly of the inverse kernels
//   HE_PROBE_MAD64   32 x 32 -> 64-bit multiply-add, the MAC's inner product
//   HE_PROBE_ADD     32-bit add (one full-rate vector instruction per operation)
//   HE_PROBE_MULLO   32-bit multiply, low half
//   HE_PROBE_MULHI   32-bit multiply, high half
#include <hip/hip_runtime.h>

#include "../../include/he.h"
#include "he_device.h"

namespace {

constexpr int PR_CHAINS = 8;
constexpr int PR_THREADS = 256;

template <int KIND>
__global__ void __launch_bounds__(PR_THREADS) k_probe(uint32_t iters, uint32_t q, uint32_t *sink) {
    const uint32_t tid = blockIdx.x * PR_THREADS + threadIdx.x;
    uint32_t x[PR_CHAINS], y[PR_CHAINS];
    uint64_t a[PR_CHAINS];
#pragma unroll
    for (int i = 0; i < PR_CHAINS; ++i) {
        x[i] = (tid * 2654435761u + i * 40503u) % q;
        y[i] = (tid * 2246822519u + i * 97u + 1u) % q;
        a[i] = 0;
    }
    const uint32_t q2 = 2 * q;
    const uint32_t w = (q / 3u) | 1u, wsh = (uint32_t)(((uint64_t)w << 32) / q);
    for (uint32_t r = 0; r < iters; ++r) {
#pragma unroll
        for (int i = 0; i < PR_CHAINS; ++i) {
            if constexpr (KIND == HE_PROBE_BFLY) {
                ct_bfly(x[i], y[i], w, wsh, q, q2);
            } else if constexpr (KIND == HE_PROBE_GSBFLY) {
                gs_bfly(x[i], y[i], w, wsh, q, q2);
            } else if constexpr (KIND == HE_PROBE_MAD64) {
                // each product takes its factor from another chain's running sum: one v_mad_u64_u32
                // per operation, nothing the compiler can fold across rounds
                a[i] += (uint64_t)x[i] * (uint32_t)(a[(i + 1) % PR_CHAINS] >> 32);
            } else if constexpr (KIND == HE_PROBE_ADD) {
                x[i] = x[i] + y[i];
                y[i] = y[i] + x[i];
            } else if constexpr (KIND == HE_PROBE_MULLO) {
                x[i] = x[i] * y[i];
                y[i] = y[i] * x[i];
            } else {
                x[i] = __umulhi(x[i], y[i]);
                y[i] = __umulhi(y[i], x[i]);
            }
        }
    }
    uint32_t s = 0;
#pragma unroll
    for (int i = 0; i < PR_CHAINS; ++i) s ^= x[i] ^ y[i] ^ (uint32_t)a[i] ^ (uint32_t)(a[i] >> 32);
    if (s == 0x9e3779b9u) sink[0] = s;      // practically never: keeps the work observable
}

}  // namespace

extern "C" int he_probe_rate(uint32_t kind, uint32_t iters, double *ops_per_s, double *ms) {
    if (!ops_per_s || iters == 0 || kind < HE_PROBE_BFLY || kind > HE_PROBE_MULHI) return HE_EINVAL;
    int dev = 0, cus = 0;
    if (hipGetDevice(&dev) != hipSuccess ||
        hipDeviceGetAttribute(&cus, hipDeviceAttributeMultiprocessorCount, dev) != hipSuccess)
        return HE_EDEVICE;
    // eight 256-thread workgroups per CU: eight waves per SIMD
    const uint32_t grid = (uint32_t)cus * 8u;
    const uint32_t q = 1073692673u;
    uint32_t *sink = nullptr;
    hipEvent_t e0 = nullptr, e1 = nullptr;
    if (hipMalloc((void **)&sink, 4) != hipSuccess) return HE_ENOMEM;
    int rc = HE_OK;
    if (hipEventCreate(&e0) != hipSuccess || hipEventCreate(&e1) != hipSuccess) rc = HE_EDEVICE;
    // operations per chain and round: a butterfly, a multiply-add, or the two dependent ops of the
    // other kinds
    double per_round = PR_CHAINS;
    if (kind == HE_PROBE_ADD || kind == HE_PROBE_MULLO || kind == HE_PROBE_MULHI) per_round = 2.0 * PR_CHAINS;
    auto launch = [&](uint32_t n) -> hipError_t {
        switch (kind) {
            case HE_PROBE_BFLY: hipLaunchKernelGGL(k_probe<HE_PROBE_BFLY>, dim3(grid), dim3(PR_THREADS), 0, nullptr, n, q, sink); break;
            case HE_PROBE_GSBFLY: hipLaunchKernelGGL(k_probe<HE_PROBE_GSBFLY>, dim3(grid), dim3(PR_THREADS), 0, nullptr, n, q, sink); break;
            case HE_PROBE_MAD64: hipLaunchKernelGGL(k_probe<HE_PROBE_MAD64>, dim3(grid), dim3(PR_THREADS), 0, nullptr, n, q, sink); break;
            case HE_PROBE_ADD: hipLaunchKernelGGL(k_probe<HE_PROBE_ADD>, dim3(grid), dim3(PR_THREADS), 0, nullptr, n, q, sink); break;
            case HE_PROBE_MULLO: hipLaunchKernelGGL(k_probe<HE_PROBE_MULLO>, dim3(grid), dim3(PR_THREADS), 0, nullptr, n, q, sink); break;
            case HE_PROBE_MULHI: hipLaunchKernelGGL(k_probe<HE_PROBE_MULHI>, dim3(grid), dim3(PR_THREADS), 0, nullptr, n, q, sink); break;
            default: return hipErrorInvalidValue;
        }
        return hipGetLastError();
    };
    float t = 0.f;
    if (rc == HE_OK) {
        // warm-up, then the timed launch
        if (launch(iters / 8u + 1u) != hipSuccess || hipEventRecord(e0, nullptr) != hipSuccess ||
            launch(iters) != hipSuccess || hipEventRecord(e1, nullptr) != hipSuccess ||
            hipEventSynchronize(e1) != hipSuccess || hipEventElapsedTime(&t, e0, e1) != hipSuccess)
            rc = HE_EDEVICE;
    }
    if (rc == HE_OK) {
        *ops_per_s = (double)grid * PR_THREADS * iters * per_round / (t * 1e-3);
        if (ms) *ms = t;
    }
    if (e0) hipEventDestroy(e0);
    if (e1) hipEventDestroy(e1);
    hipFree(sink);
    return rc;
}
