// Memory microbenchmarks for the rooflines: chains of dependent random 16-byte
// reads (the access pattern of an incoherent stackless walk with its box and
// triangle arithmetic taken out), and streaming copy / read of a buffer (the
// achievable HBM bandwidth).
#include <algorithm>

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

constexpr int kStreamBlock = 256;
constexpr int kStreamUnroll = 4;  // 16-byte accesses in flight per thread

// Grid-stride over n16 16-byte words, kStreamUnroll per thread per step, each
// step's words kStreamBlock apart so a wavefront's accesses are contiguous.
// kCopy: dst = src; otherwise the XOR of every word read goes to *out (one
// atomic per wavefront).
template <bool kCopy>
__global__ __launch_bounds__(kStreamBlock) void k_stream(const uint4 *__restrict__ src, uint4 *__restrict__ dst,
                                                         uint64_t n16, uint32_t *__restrict__ out) {
    const uint64_t span = (uint64_t)kStreamBlock * kStreamUnroll;
    uint32_t acc = 0u;
    for (uint64_t base = (uint64_t)blockIdx.x * span; base < n16; base += (uint64_t)gridDim.x * span) {
        uint4 v[kStreamUnroll];
#pragma unroll
        for (int u = 0; u < kStreamUnroll; ++u) {
            const uint64_t i = base + (uint64_t)u * kStreamBlock + threadIdx.x;
            v[u] = i < n16 ? src[i] : make_uint4(0u, 0u, 0u, 0u);
        }
#pragma unroll
        for (int u = 0; u < kStreamUnroll; ++u) {
            const uint64_t i = base + (uint64_t)u * kStreamBlock + threadIdx.x;
            if (kCopy) {
                if (i < n16) dst[i] = v[u];
            } else {
                acc ^= (v[u].x ^ v[u].y) ^ (v[u].z ^ v[u].w);
            }
        }
    }
    if (!kCopy) {  // one atomic per workgroup
        __shared__ uint32_t lds[kStreamBlock / 64];
        for (int off = 32; off > 0; off >>= 1) acc ^= __shfl_xor(acc, off);
        if ((threadIdx.x & 63) == 0) lds[threadIdx.x >> 6] = acc;
        __syncthreads();
        if (threadIdx.x == 0) {
            uint32_t w = 0u;
            for (int i = 0; i < kStreamBlock / 64; ++i) w ^= lds[i];
            atomicXor(out, w);
        }
    }
}

}  // namespace

namespace pm {

int launch_stream(const void *src, void *dst, uint64_t n_bytes, int32_t mode, uint32_t *out, hipStream_t s) {
    const uint64_t n16 = n_bytes / 16;
    const uint64_t span = (uint64_t)kStreamBlock * kStreamUnroll;
    // the read reduces once per workgroup, so it takes fewer, longer workgroups
    const uint32_t grid = (uint32_t)std::min<uint64_t>((n16 + span - 1) / span, mode == 0 ? 32768u : 4096u);
    if (mode == 0)
        hipLaunchKernelGGL(k_stream<true>, dim3(grid), dim3(kStreamBlock), 0, s, (const uint4 *)src, (uint4 *)dst,
                           n16, out);
    else
        hipLaunchKernelGGL(k_stream<false>, dim3(grid), dim3(kStreamBlock), 0, s, (const uint4 *)src, (uint4 *)dst,
                           n16, out);
    PM_HIP(hipGetLastError());
    return PM_OK;
}


int launch_chase(const uint32_t *rows, int32_t log2_rows, uint32_t n_lanes, uint32_t steps, uint32_t *out,
                 hipStream_t s) {
    const uint32_t mask = (uint32_t)((uint64_t(1) << log2_rows) - 1u);
    hipLaunchKernelGGL(k_chase, dim3((n_lanes + kProbeBlock - 1) / kProbeBlock), dim3(kProbeBlock), 0, s,
                       (const uint4 *)rows, mask, n_lanes, steps, out);
    PM_HIP(hipGetLastError());
    return PM_OK;
}

}  // namespace pm
