// Exclusive scan of bucket counts (hashed-grid build), three passes:
// per-tile scan, scan of tile totals, add tile offsets.  The bucket count
// must be a multiple of kScanTile.  Internal linkage: each translation unit
// that includes this header gets its own copy of the kernels.
#pragma once
#include "sppm_dev.h"

namespace {

// Pass 1: per-tile exclusive scan into out[], tile totals into bsum[].
__global__ __launch_bounds__(pmd::kBlock) void k_scan_tiles(const uint32_t *__restrict__ in, uint32_t *__restrict__ out,
                                                            uint32_t *__restrict__ bsum) {
    __shared__ uint32_t lds[pmd::kBlock / 64];
    const uint32_t *src = in + (size_t)blockIdx.x * pmd::kScanTile + threadIdx.x * pmd::kScanItems;
    uint32_t vals[pmd::kScanItems];
    uint32_t s = 0;
#pragma unroll
    for (int i = 0; i < pmd::kScanItems; ++i) {
        vals[i] = src[i];
        s += vals[i];
    }
    uint32_t total;
    uint32_t ex = pmd::block_exscan(s, lds, total);
    uint32_t *dst = out + (size_t)blockIdx.x * pmd::kScanTile + threadIdx.x * pmd::kScanItems;
#pragma unroll
    for (int i = 0; i < pmd::kScanItems; ++i) {
        dst[i] = ex;
        ex += vals[i];
    }
    if (threadIdx.x == 0) bsum[blockIdx.x] = total;
}

// Pass 2: exclusive scan of nb tile totals in one block, kScanTile at a time
// with a running carry; bsum[nb] receives the grand total.
__global__ __launch_bounds__(pmd::kBlock) void k_scan_sums(uint32_t *__restrict__ bsum, uint32_t nb) {
    __shared__ uint32_t lds[pmd::kBlock / 64];
    uint32_t carry = 0;
    for (uint32_t base = 0; base < nb; base += pmd::kScanTile) {
        uint32_t vals[pmd::kScanItems];
        uint32_t s = 0;
#pragma unroll
        for (int i = 0; i < pmd::kScanItems; ++i) {
            uint32_t j = base + threadIdx.x * pmd::kScanItems + i;
            vals[i] = j < nb ? bsum[j] : 0u;
            s += vals[i];
        }
        uint32_t total;
        uint32_t ex = pmd::block_exscan(s, lds, total) + carry;
#pragma unroll
        for (int i = 0; i < pmd::kScanItems; ++i) {
            uint32_t j = base + threadIdx.x * pmd::kScanItems + i;
            if (j < nb) bsum[j] = ex;
            ex += vals[i];
        }
        carry += total;
        __syncthreads();
    }
    if (threadIdx.x == 0) bsum[nb] = carry;
}

// Pass 3: add tile offsets; write start[] and the scatter cursors fill[].
__global__ __launch_bounds__(pmd::kBlock) void k_scan_add(uint32_t *__restrict__ start, uint32_t *__restrict__ fill,
                                                          const uint32_t *__restrict__ bsum, uint32_t nb) {
    uint32_t off = bsum[blockIdx.x];
    size_t base = (size_t)blockIdx.x * pmd::kScanTile;
    for (int i = threadIdx.x; i < pmd::kScanTile; i += pmd::kBlock) {
        uint32_t v = start[base + i] + off;
        start[base + i] = v;
        fill[base + i] = v;
    }
    if (blockIdx.x == 0 && threadIdx.x == 0) start[(size_t)nb * pmd::kScanTile] = bsum[nb];
}

__global__ __launch_bounds__(pmd::kBlock) void k_fill_u32(uint32_t *__restrict__ p, uint32_t n, uint32_t v) {
    uint32_t i = blockIdx.x * pmd::kBlock + threadIdx.x;
    if (i < n) p[i] = v;
}

// counts[0..nbuckets) -> start[0..nbuckets], fill[0..nbuckets)
inline void launch_bucket_scan(uint32_t *counts, uint32_t *start, uint32_t *fill, uint32_t *bsum, uint32_t nbuckets,
                               hipStream_t st) {
    const uint32_t nb = nbuckets / pmd::kScanTile;
    hipLaunchKernelGGL(k_scan_tiles, dim3(nb), dim3(pmd::kBlock), 0, st, counts, start, bsum);
    hipLaunchKernelGGL(k_scan_sums, dim3(1), dim3(pmd::kBlock), 0, st, bsum, nb);
    hipLaunchKernelGGL(k_scan_add, dim3(nb), dim3(pmd::kBlock), 0, st, start, fill, bsum, nb);
}

}  // namespace
