// Closest-hit ray traversal of the multiple-threaded BVH (Sec. 3.1).
#include "pm_device.h"
#include "runtime.h"

namespace {

constexpr int kTraceBlock = 256;

// One ray per lane.  rays: [n][2] float4 = (o.xyz, tmin), (d.xyz, tmax).
template <bool kStats>
__global__ __launch_bounds__(kTraceBlock) void k_trace(pmd::Bvh bvh, const float4 *__restrict__ rays, int64_t n,
                                                       int32_t *__restrict__ hit, float *__restrict__ tout,
                                                       int32_t force_set, uint32_t *__restrict__ counters) {
    uint32_t blk = pmd::xcd_block(blockIdx.x, gridDim.x);
    int64_t i = (int64_t)blk * kTraceBlock + threadIdx.x;
    if (i >= n) return;
    float4 r0 = rays[2 * i], r1 = rays[2 * i + 1];
    pmd::V3 o = pmd::v3(r0.x, r0.y, r0.z), d = pmd::v3(r1.x, r1.y, r1.z);
    int set = force_set >= 0 ? force_set : pmd::link_set(d);
    pmd::TraceStats st{0u, 0u};
    float t;
    uint32_t kpos;
    int32_t h = pmd::closest_hit<kStats>(bvh, set, o, d, r0.w, r1.w, -1, t, kpos, st);
    hit[i] = h;
    tout[i] = t;
    if (kStats) {
        counters[2 * i] = st.boxes;
        counters[2 * i + 1] = st.tris;
    }
}

}  // namespace

namespace pm {

int upload_bvh(const HostBvh &h, hipStream_t s, pm_bvh *b) {
    b->n_tri = h.n_tri;
    b->n_nodes = h.n_nodes;
    b->n_leaves = h.n_leaves;
    b->depth = h.depth;
    b->max_leaf = h.max_leaf;
    b->sah_cost = h.sah_cost;
    b->build_ms = h.build_ms;
    for (int a = 0; a < 3; ++a) {
        b->lo[a] = h.lo[a];
        b->hi[a] = h.hi[a];
    }
    b->pos_of.assign((size_t)h.n_tri, 0);
    for (int64_t k = 0; k < h.n_tri; ++k) b->pos_of[h.tris[(size_t)k * kTriWords + 9]] = (int32_t)k;
    PM_HIP(hipGetDevice(&b->device));
    size_t nb = h.nodes.size() * sizeof(uint32_t), tb = h.tris.size() * sizeof(uint32_t);
    PM_HIP(hipMalloc(&b->d_nodes, nb));
    PM_HIP(hipMalloc(&b->d_tris, tb));
    PM_HIP(hipMemcpyAsync(b->d_nodes, h.nodes.data(), nb, hipMemcpyHostToDevice, s));
    PM_HIP(hipMemcpyAsync(b->d_tris, h.tris.data(), tb, hipMemcpyHostToDevice, s));
    // host vectors are freed by the caller: wait for the copies
    PM_HIP(hipStreamSynchronize(s));
    return PM_OK;
}

void free_bvh(pm_bvh *b) {
    if (b->d_nodes) (void)hipFree(b->d_nodes);
    if (b->d_tris) (void)hipFree(b->d_tris);
    b->d_nodes = nullptr;
    b->d_tris = nullptr;
}

int launch_trace(const pm_bvh *b, const float *rays, int64_t n, int32_t *hit, float *t, int link_set,
                 uint32_t *counters, hipStream_t s) {
    if (n == 0) return PM_OK;
    pmd::Bvh bvh{b->d_nodes, b->d_tris, (uint32_t)b->n_nodes};
    int64_t nblk = (n + kTraceBlock - 1) / kTraceBlock;
    if (nblk > 0x7fffffff) {
        set_error("too many rays for one launch");
        return PM_ERR_ARG;
    }
    dim3 grid((uint32_t)nblk), block(kTraceBlock);
    if (counters)
        hipLaunchKernelGGL(k_trace<true>, grid, block, 0, s, bvh, (const float4 *)rays, n, hit, t, link_set, counters);
    else
        hipLaunchKernelGGL(k_trace<false>, grid, block, 0, s, bvh, (const float4 *)rays, n, hit, t, link_set, counters);
    PM_HIP(hipGetLastError());
    return PM_OK;
}

}  // namespace pm
