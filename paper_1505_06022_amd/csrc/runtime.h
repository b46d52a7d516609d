// Host runtime shared by the C ABI and the kernel launchers.
#pragma once
#include <hip/hip_runtime.h>

#include <cstdint>
#include <string>
#include <vector>

#include "bvh_build.h"
#include "pm.h"

namespace pm {

void set_error(const std::string &msg);
void clear_error();
const char *last_error();

// Record a HIP failure and return PM_ERR_HIP.
int hip_fail(hipError_t e, const char *what);

#define PM_HIP(call)                                   \
    do {                                               \
        hipError_t e_ = (call);                        \
        if (e_ != hipSuccess) return pm::hip_fail(e_, #call); \
    } while (0)

// Zeroed nodes after a BVH's six node arrays: a packet walk reads the node
// after the one it visits.
constexpr size_t kPadNodes = 1;

}  // namespace pm

struct pm_bvh {
    int64_t n_tri = 0, n_refs = 0, n_nodes = 0, n_leaves = 0;  // n_refs: triangle records
    int32_t depth = 0, max_leaf = 0;
    double sah_cost = 0.0, build_ms = 0.0;
    float lo[3] = {0, 0, 0}, hi[3] = {0, 0, 0};
    float qlo[3] = {0, 0, 0}, qstep[3] = {1, 1, 1};
    uint4 *d_nodes = nullptr;   // [6][n_nodes] 16-byte nodes, then kPadNodes zeroed nodes
    float4 *d_tris = nullptr;   // [n_refs][3]
    uint32_t *d_next = nullptr; // work counter of the persistent traversal kernel
    uint32_t *d_perm = nullptr; // ray order of the reordering traversal (perm_cap entries)
    uint64_t perm_cap = 0;
    uint32_t *d_order = nullptr; // bucket counts / starts / cursors of the ray reordering
    // streams of batches 1.. of pm_trace_rays_multi, and the events that fork
    // them from and join them to the caller's stream (created on first use)
    hipStream_t side[PM_MAX_TRACE_BATCHES] = {};
    hipEvent_t ev_fork = nullptr;
    hipEvent_t ev_join[PM_MAX_TRACE_BATCHES] = {};
    int device = 0;
    std::vector<int32_t> pos_of;  // original triangle index -> its first record in d_tris
};

namespace pmd {
struct Bvh;
}

namespace pm {

// Dependent random reads over 2^log2_rows 16-byte rows (memory microbenchmark).
// Streaming copy (mode 0) or read with an XOR of every word into *out (mode 1).
int launch_stream(const void *src, void *dst, uint64_t n_bytes, int32_t mode, uint32_t *out, hipStream_t s);
int launch_chase(const uint32_t *rows, int32_t log2_rows, uint32_t n_lanes, uint32_t steps, uint32_t *out,
                 hipStream_t s);

// Device view of a BVH handle (node/triangle pointers and the box grid).
pmd::Bvh make_device_bvh(const pm_bvh *b);

// Build the BVH on the device from sorted Morton codes (same layout as the
// host build); fills b.  The caller validates the inputs.
int build_bvh_gpu(const float *verts, const uint32_t *mats, int64_t n_tri, int max_leaf, double trav_cost,
                  hipStream_t s, pm_bvh *b);

// Upload a host-built BVH; fills b (device buffers owned by b).
int upload_bvh(const HostBvh &h, hipStream_t s, pm_bvh *b);
void free_bvh(pm_bvh *b);

// Validated arguments of one traced batch.  link_set < 0 selects by
// direction; block: threads per workgroup of the one-ray-per-lane kernels
// (64, 128 or 256); tile_w > 0: the rays are an image tile_w wide, taken in
// 8x8 tiles per wave; slice: rays per wavefront of the slice kernel.
struct TraceArgs {
    const float *rays = nullptr;
    int64_t n = 0;
    int32_t *hit = nullptr;
    float *t = nullptr;
    int link_set = -1, kernel = PM_TRACE_AUTO, refill = 0, reorder = 0, block = 0, tile_w = 0, slice = 0;
    uint32_t *counters = nullptr;
};

// Launch the closest-hit kernel for one batch.
int launch_trace(const pm_bvh *b, const TraceArgs &a, hipStream_t s);

// The bucketed trace (reorder 1 or 2) on the library's static per-device
// scratch: no allocation; n <= PM_NOALLOC_MAX_RAYS; b must be on the current
// device.
int launch_trace_noalloc(const pm_bvh *b, const TraceArgs &a, hipStream_t s);

// Batches 1.. on the handle's own streams, forked from and joined to s.
int launch_trace_multi(pm_bvh *b, const TraceArgs *batches, int32_t n_batches, hipStream_t s);

}  // namespace pm
