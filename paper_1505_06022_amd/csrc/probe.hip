// Memory microbenchmark for the traversal's roofline: chains of dependent
// random 16-byte reads, the access pattern of an incoherent stackless walk
// with its box and triangle arithmetic taken out.
#include "pm_device.h"
#include "runtime.h"

namespace {

constexpr int kProbeBlock = 64;  // one wavefront per workgroup, as the incoherent walk launches

// Lane l starts at row (l * 0x9E3779B1) & mask and takes `steps` reads; after
// row (x, y, z, w) it moves to row (x ^ salt) & mask, salt = l * 0x85EBCA77.
// out[l] = XOR of all words read (keeps every read live; checkable on the host).
__global__ __launch_bounds__(kProbeBlock) void k_chase(const uint4 *__restrict__ rows, uint32_t mask, uint32_t n_lanes,
                                                       uint32_t steps, uint32_t *__restrict__ out) {
    const uint32_t lane = pmd::xcd_block(blockIdx.x, gridDim.x) * kProbeBlock + threadIdx.x;
    if (lane >= n_lanes) return;
    uint32_t r = (lane * 0x9E3779B1u) & mask;
    const uint32_t salt = lane * 0x85EBCA77u;
    uint32_t acc = 0u;
    for (uint32_t s = 0; s < steps; ++s) {
        const uint4 q = rows[r];
        acc ^= (q.x ^ q.y) ^ (q.z ^ q.w);
        r = (q.x ^ salt) & mask;
    }
    out[lane] = acc;
}

}  // namespace

namespace pm {

int launch_chase(const uint32_t *rows, int32_t log2_rows, uint32_t n_lanes, uint32_t steps, uint32_t *out,
                 hipStream_t s) {
    const uint32_t mask = (uint32_t)((uint64_t(1) << log2_rows) - 1u);
    hipLaunchKernelGGL(k_chase, dim3((n_lanes + kProbeBlock - 1) / kProbeBlock), dim3(kProbeBlock), 0, s,
                       (const uint4 *)rows, mask, n_lanes, steps, out);
    PM_HIP(hipGetLastError());
    return PM_OK;
}

}  // namespace pm
