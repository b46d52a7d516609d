// Closest-hit ray traversal of the multiple-threaded BVH (Sec. 3.1).
#include <algorithm>

#include "pm_device.h"
#include "runtime.h"

namespace {

constexpr int kTraceBlock = 256;
constexpr uint32_t kNoRay = 0xffffffffu;

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

// Persistent wavefronts with ray replacement (the scheduling idea of the
// paper's photon path regeneration, Sec. 3.3, applied to rays): every lane
// walks its ray one node per iteration; finished lanes publish their result
// and, once at least `refill` lanes of the wave are idle (or all are), the
// wave takes that many new ray indices from a global counter with one atomic.
// Every iteration advances each active ray to a strictly larger preorder
// index, so every wave exits once the counter passes n.
template <bool kStats>
__global__ __launch_bounds__(kTraceBlock) void k_trace_persistent(pmd::Bvh bvh, const float4 *__restrict__ rays,
                                                                  uint32_t n, int32_t *__restrict__ hit,
                                                                  float *__restrict__ tout, int32_t force_set,
                                                                  uint32_t *__restrict__ counters,
                                                                  uint32_t *__restrict__ next, uint32_t refill) {
    pmd::Walker w;
    pmd::TraceStats st{0u, 0u};
    uint32_t r = kNoRay;
    bool exhausted = false;
    w.i = 0;
    w.n = 0;
    for (;;) {
        if (r != kNoRay && w.done()) {
            hit[r] = w.best;
            tout[r] = w.t_hit();
            if (kStats) {
                counters[2 * (size_t)r] = st.boxes;
                counters[2 * (size_t)r + 1] = st.tris;
            }
            r = kNoRay;
        }
        bool idle = (r == kNoRay) && !exhausted;
        uint64_t idle_mask = __ballot(idle);
        uint64_t busy_mask = __ballot(r != kNoRay);
        if (idle_mask != 0ull && (busy_mask == 0ull || (uint32_t)__popcll(idle_mask) >= refill)) {
            uint32_t rr = pmd::wave_fetch_add(next, idle_mask, idle);
            if (idle) {
                if (rr < n) {
                    float4 r0 = rays[2 * (size_t)rr], r1 = rays[2 * (size_t)rr + 1];
                    pmd::V3 o = pmd::v3(r0.x, r0.y, r0.z), d = pmd::v3(r1.x, r1.y, r1.z);
                    int set = force_set >= 0 ? force_set : pmd::link_set(d);
                    w.init(bvh, set, o, d, r0.w, r1.w, -1);
                    st.boxes = st.tris = 0u;
                    r = rr;
                } else {
                    exhausted = true;
                }
            }
            busy_mask = __ballot(r != kNoRay);
        }
        if (busy_mask == 0ull) break;
        if (r != kNoRay) w.step<kStats>(bvh.tris, st);
    }
}

__global__ void k_reset_counter(uint32_t *next) {
    if (threadIdx.x == 0) *next = 0u;
}

}  // namespace

namespace pm {

pmd::Bvh make_device_bvh(const pm_bvh *b) {
    pmd::Bvh d;
    d.nodes = b->d_nodes;
    d.tris = b->d_tris;
    d.n_nodes = (uint32_t)b->n_nodes;
    for (int a = 0; a < 3; ++a) {
        d.qlo[a] = b->qlo[a];
        d.qstep[a] = b->qstep[a];
    }
    return d;
}

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
        b->qlo[a] = h.qlo[a];
        b->qstep[a] = h.qstep[a];
    }
    b->pos_of.assign((size_t)h.n_tri, 0);
    for (int64_t k = 0; k < h.n_tri; ++k) b->pos_of[h.tris[(size_t)k * kTriWords + 9]] = (int32_t)k;
    PM_HIP(hipGetDevice(&b->device));
    size_t nb = h.nodes.size() * sizeof(uint32_t), tb = h.tris.size() * sizeof(uint32_t);
    PM_HIP(hipMalloc(&b->d_nodes, nb));
    PM_HIP(hipMalloc(&b->d_tris, tb));
    PM_HIP(hipMalloc(&b->d_next, 64));
    PM_HIP(hipMemcpyAsync(b->d_nodes, h.nodes.data(), nb, hipMemcpyHostToDevice, s));
    PM_HIP(hipMemcpyAsync(b->d_tris, h.tris.data(), tb, hipMemcpyHostToDevice, s));
    // host vectors are freed by the caller: wait for the copies
    PM_HIP(hipStreamSynchronize(s));
    return PM_OK;
}

void free_bvh(pm_bvh *b) {
    if (b->d_nodes) (void)hipFree(b->d_nodes);
    if (b->d_tris) (void)hipFree(b->d_tris);
    if (b->d_next) (void)hipFree(b->d_next);
    b->d_nodes = nullptr;
    b->d_tris = nullptr;
    b->d_next = nullptr;
}

static int persistent_grid(hipStream_t s, int device, uint32_t &grid) {
    static int cached_dev = -1;
    static uint32_t cached = 0;
    if (cached_dev == device) {
        grid = cached;
        return PM_OK;
    }
    int cus = 0, per_cu = 0;
    PM_HIP(hipDeviceGetAttribute(&cus, hipDeviceAttributeMultiprocessorCount, device));
    PM_HIP(hipOccupancyMaxActiveBlocksPerMultiprocessor(&per_cu, k_trace_persistent<false>, kTraceBlock, 0));
    cached = (uint32_t)std::max(1, cus * std::max(1, per_cu));
    cached_dev = device;
    grid = cached;
    (void)s;
    return PM_OK;
}

int launch_trace(const pm_bvh *b, const float *rays, int64_t n, int32_t *hit, float *t, int link_set,
                 uint32_t *counters, int kernel, int refill, hipStream_t s) {
    if (n == 0) return PM_OK;
    pmd::Bvh bvh = make_device_bvh(b);
    if (kernel == 0) kernel = PM_TRACE_PER_RAY;
    if (kernel == PM_TRACE_PERSISTENT) {
        if (n >= (int64_t(1) << 31)) {
            set_error("too many rays for one launch");
            return PM_ERR_ARG;
        }
        uint32_t grid = 0;
        int rc = persistent_grid(s, b->device, grid);
        if (rc) return rc;
        uint32_t rf = refill > 0 ? (uint32_t)refill : 16u;
        hipLaunchKernelGGL(k_reset_counter, dim3(1), dim3(64), 0, s, b->d_next);
        if (counters)
            hipLaunchKernelGGL(k_trace_persistent<true>, dim3(grid), dim3(kTraceBlock), 0, s, bvh,
                               (const float4 *)rays, (uint32_t)n, hit, t, link_set, counters, b->d_next, rf);
        else
            hipLaunchKernelGGL(k_trace_persistent<false>, dim3(grid), dim3(kTraceBlock), 0, s, bvh,
                               (const float4 *)rays, (uint32_t)n, hit, t, link_set, counters, b->d_next, rf);
        PM_HIP(hipGetLastError());
        return PM_OK;
    }
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
