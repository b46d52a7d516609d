// Closest-hit ray traversal of the multiple-threaded BVH (Sec. 3.1).
#include <algorithm>
#include <atomic>
#include <mutex>

#include "pm_device.h"
#include "runtime.h"
#include "sppm_scan.h"

namespace {

static_assert(pmd::kPacketRun >= 1 && pmd::kPacketRun - 1 <= (int)pm::kPadNodes, "packet reads past the pad nodes");

constexpr int kTraceBlock = 256;
constexpr int kDefaultWalkBlock = 256;  // workgroup of the one-ray-per-lane kernels
constexpr uint32_t kNoRay = 0xffffffffu;

// Walk orders: one ray per lane, one node per visit with the leaf's
// triangles tested at once (kWalkStep); nodes i and i + 1 from one memory
// round trip (kWalkPaired); leaf tests postponed until the wave's lanes hold
// leaves together (kWalkPostponed); two rays per lane in lockstep (kWalkTwo);
// or the wave's rays as one packet (kWalkPacket).  All give the same closest
// hit.
enum { kWalkStep = 0, kWalkPaired = 1, kWalkPostponed = 2, kWalkTwo = 3, kWalkPacket = 4 };

template <int kWalk, bool kStats>
__device__ __forceinline__ void walk(pmd::Walker &w, const float4 *__restrict__ tris, uint32_t late,
                                     pmd::TraceStats &st) {
    if (kWalk == kWalkPostponed) {
        w.walk_postponed<kStats>(tris, late, st);
    } else {
        while (!w.done()) {
            if (kWalk == kWalkPaired) w.step2<kStats>(tris, st);
            else w.step<kStats>(tris, st);
        }
    }
}

// rays: [n][2] float4 = (o.xyz, tmin), (d.xyz, tmax).
// Rays are read once and results written once: non-temporal accesses keep
// them from displacing BVH nodes in L2 (measured: 4% off the traversal step;
// the bucketing's ray reads and (bucket, rank) pairs: a further 0.8%).  The
// ray order itself is read back at once by the walk and stays cached.
typedef float NtFloat4 __attribute__((ext_vector_type(4)));
typedef uint32_t NtUint2 __attribute__((ext_vector_type(2)));

__device__ __forceinline__ void start_walk(pmd::Walker &w, const pmd::Bvh &bvh, const float4 *__restrict__ rays,
                                           size_t r, int32_t force_set) {
    const NtFloat4 a0 = __builtin_nontemporal_load((const NtFloat4 *)(rays + 2 * r));
    const NtFloat4 a1 = __builtin_nontemporal_load((const NtFloat4 *)(rays + 2 * r + 1));
    const float4 r0 = make_float4(a0.x, a0.y, a0.z, a0.w), r1 = make_float4(a1.x, a1.y, a1.z, a1.w);
    pmd::V3 o = pmd::v3(r0.x, r0.y, r0.z), d = pmd::v3(r1.x, r1.y, r1.z);
    int set = force_set >= 0 ? force_set : pmd::link_set(d);
    w.init(bvh, set, o, d, r0.w, r1.w, -1);
}

template <bool kStats>
__device__ __forceinline__ void finish_walk(const pmd::Walker &w, const pmd::TraceStats &st, size_t r,
                                            int32_t *__restrict__ hit, float *__restrict__ tout,
                                            uint32_t *__restrict__ counters) {
    __builtin_nontemporal_store(w.best, hit + r);
    __builtin_nontemporal_store(w.t_hit(), tout + r);
    if (kStats) {
        counters[2 * r] = st.boxes;
        counters[2 * r + 1] = st.tris;
    }
}

// The rays of slot j: ray j (kPerm false) or perm[j]; two consecutive slots
// per lane for kWalkTwo.  With tile_w > 0 (kPerm false) the rays are the
// pixels of an image tile_w wide in row-major order and each wave takes an
// 8x8 tile.  Results go to each ray's own index.
template <bool kStats, int kWalk, bool kPerm>
__device__ __forceinline__ void trace_slot(const pmd::Bvh &bvh, const float4 *__restrict__ rays,
                                           const uint32_t *__restrict__ perm, uint64_t lane, uint64_t n,
                                           int32_t *__restrict__ hit, float *__restrict__ tout, int32_t force_set,
                                           uint32_t *__restrict__ counters, uint32_t late, uint32_t tile_w) {
    if (kWalk == kWalkTwo) {
        const uint64_t ja = 2 * lane, jb = ja + 1;
        if (ja >= n) return;
        const size_t ra = kPerm ? perm[ja] : ja;
        const bool has_b = jb < n;
        const size_t rb = has_b ? (kPerm ? perm[jb] : jb) : 0;
        pmd::Walker a, b;
        pmd::TraceStats sa{0u, 0u}, sb{0u, 0u};
        start_walk(a, bvh, rays, ra, force_set);
        if (has_b) {
            start_walk(b, bvh, rays, rb, force_set);
        } else {  // no second ray: a walker that is done from the start
            b = a;
            b.i = b.n = 0u;
        }
        pmd::walk_two<kStats>(a, b, bvh.tris, sa, sb);
        finish_walk<kStats>(a, sa, ra, hit, tout, counters);
        if (has_b) finish_walk<kStats>(b, sb, rb, hit, tout, counters);
    } else {
        size_t r;
        if (!kPerm && tile_w > 0) {
            const uint64_t wave = lane >> 6, l = lane & 63u, tiles_x = (tile_w + 7u) / 8u;
            const uint64_t x = (wave % tiles_x) * 8u + (l & 7u), y = (wave / tiles_x) * 8u + (l >> 3);
            if (x >= tile_w || y >= n / tile_w) return;
            r = (size_t)(y * tile_w + x);
        } else {
            if (lane >= n) return;
            r = kPerm ? __builtin_nontemporal_load(perm + lane) : lane;
        }
        pmd::Walker w;
        pmd::TraceStats st{0u, 0u};
        start_walk(w, bvh, rays, r, force_set);
        if (kWalk == kWalkPacket) {
            const int set = (int)((w.nodes - bvh.nodes) / bvh.n_nodes);
            const int set0 = __builtin_amdgcn_readfirstlane(set);
            if (__ballot(set != set0) == 0ull)  // one link set for the whole wave: its base is uniform
                pmd::walk_packet<kStats>(w, bvh.nodes + (size_t)(uint32_t)set0 * bvh.n_nodes, bvh.n_nodes, bvh.tris, st);
            else
                walk<kWalkStep, kStats>(w, bvh.tris, late, st);  // link sets differ within the wave
        } else {
            walk<kWalk, kStats>(w, bvh.tris, late, st);
        }
        finish_walk<kStats>(w, st, r, hit, tout, counters);
    }
}

// Postponed-leaf walk over one wavefront's slice of the ray order: rays
// begin .. end - 1 of perm (or of the input order without perm).  A lane
// whose ray has ended takes the next ray of the slice, so lanes do not idle
// while the wave's longest walk runs: the scheduling idea of the paper's
// photon path regeneration (Sec. 3.3), applied to rays.  A slice is a
// contiguous run of the bucketed order, so a wave's rays stay close in
// space.  The wave visits boxes until at most `late` lanes are still
// searching for a leaf hit and either some lane holds one or some lane can
// take a new ray; then the held leaves are tested, ended rays written and
// idle lanes refilled.  Each round advances a searching lane, tests a held
// leaf or starts a ray, so the walk ends (late < 64).  The closest hit of a
// ray does not depend on when it is walked.  Called by all lanes of a wave
// with wave-uniform begin and end.
template <bool kStats>
__device__ __forceinline__ void walk_slice(const pmd::Bvh &bvh, const float4 *__restrict__ rays,
                                           const uint32_t *__restrict__ perm, uint32_t begin, uint32_t end,
                                           int32_t *__restrict__ hit, float *__restrict__ tout, int32_t force_set,
                                           uint32_t *__restrict__ counters, uint32_t late) {
    pmd::Walker w;
    w.i = w.n = 0u;  // no ray yet
    pmd::TraceStats st{0u, 0u};
    size_t r = 0;
    bool active = false, halted = false;
    uint32_t held = 0u;
    uint32_t cursor = begin;  // next ray of the slice (wave-uniform)
    for (;;) {
        const bool idle = !active;
        const uint64_t idle_mask = __ballot(idle);
        if (idle_mask != 0ull && cursor < end) {
            const uint32_t rank = __builtin_amdgcn_mbcnt_hi((uint32_t)(idle_mask >> 32),
                                                            __builtin_amdgcn_mbcnt_lo((uint32_t)idle_mask, 0u));
            if (idle && rank < end - cursor) {
                r = perm ? perm[cursor + rank] : (size_t)(cursor + rank);
                start_walk(w, bvh, rays, r, force_set);
                st = pmd::TraceStats{0u, 0u};
                active = true;
            }
            const uint32_t taken = (uint32_t)__popcll(idle_mask);
            cursor = taken < end - cursor ? cursor + taken : end;
        }
        if (__ballot(active) == 0ull) break;
        for (;;) {
            const uint64_t searching = __ballot(w.i < w.n && held == 0u);
            if (searching == 0ull) break;
            if ((uint32_t)__popcll(searching) <= late &&
                (__ballot(held != 0u) != 0ull || (cursor < end && __ballot(w.i >= w.n && held == 0u) != 0ull)))
                break;
#pragma unroll
            for (int u = 0; u < pmd::Walker::kPostponedSteps; ++u) {
                if (w.i < w.n && !halted) {  // the box visits of Walker::walk_postponed
                    const uint4 q = w.nodes[w.i];
                    if (kStats) st.boxes++;
                    const bool leaf = (q.w >> 31) != 0u, hit = w.box_hit(q);
                    const bool leaf_hit = hit && leaf;
                    halted = leaf_hit && held != 0u;
                    held = (leaf_hit && held == 0u) ? q.w : held;
                    w.i = halted ? w.i : ((hit || leaf) ? w.i + 1 : q.w);
                }
            }
        }
        if (held != 0u) w.leaf_tris<kStats>(bvh.tris, held, st);
        held = 0u;
        halted = false;
        if (active && w.i >= w.n) {
            finish_walk<kStats>(w, st, r, hit, tout, counters);
            active = false;
        }
    }
}

// Rays in slices of `slice` consecutive entries of perm (or of the input
// order), one slice per wavefront.
template <bool kStats>
__global__ __launch_bounds__(kTraceBlock) void k_trace_slices(pmd::Bvh bvh, const float4 *__restrict__ rays,
                                                              const uint32_t *__restrict__ perm, uint32_t n,
                                                              int32_t *__restrict__ hit, float *__restrict__ tout,
                                                              int32_t force_set, uint32_t *__restrict__ counters,
                                                              uint32_t late, uint32_t slice) {
    const uint32_t wave = (pmd::xcd_block(blockIdx.x, gridDim.x) * blockDim.x + threadIdx.x) >> 6;
    const uint64_t begin = (uint64_t)wave * slice;
    if (begin >= n) return;
    const uint32_t end = (uint32_t)(begin + slice < n ? begin + slice : n);
    walk_slice<kStats>(bvh, rays, perm, (uint32_t)begin, end, hit, tout, force_set, counters, late);
}

// Rays in input order.
template <bool kStats, int kWalk>
__global__ __launch_bounds__(kTraceBlock) void k_trace(pmd::Bvh bvh, const float4 *__restrict__ rays, int64_t n,
                                                       int32_t *__restrict__ hit, float *__restrict__ tout,
                                                       int32_t force_set, uint32_t *__restrict__ counters,
                                                       uint32_t late, uint32_t tile_w) {
    const uint64_t lane = (uint64_t)pmd::xcd_block(blockIdx.x, gridDim.x) * blockDim.x + threadIdx.x;
    trace_slot<kStats, kWalk, false>(bvh, rays, nullptr, lane, (uint64_t)n, hit, tout, force_set, counters, late,
                                     tile_w);
}

// Persistent wavefronts with ray replacement (the scheduling idea of the
// paper's photon path regeneration, Sec. 3.3, applied to rays): every lane
// walks its ray one node per iteration; finished lanes publish their result
// and, once at least `refill` lanes of the wave are idle (or all are), the
// wave takes that many new ray indices from a global counter with one atomic.
// Every iteration advances each active ray to a strictly larger preorder
// index, so every wave exits once the counter passes n.
// With perm, the k-th ray taken is perm[k].
template <bool kStats>
__global__ __launch_bounds__(kTraceBlock) void k_trace_persistent(pmd::Bvh bvh, const float4 *__restrict__ rays,
                                                                  uint32_t n, int32_t *__restrict__ hit,
                                                                  float *__restrict__ tout, int32_t force_set,
                                                                  uint32_t *__restrict__ counters,
                                                                  uint32_t *__restrict__ next, uint32_t refill,
                                                                  const uint32_t *__restrict__ perm) {
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
                    if (perm) rr = perm[rr];
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

// Ray reordering: bucket = (Morton code of the origin cell in a grid over the
// scene box, link set[, signs of the two minor direction components]), so
// that the rays of a wave share a direction set and start near each other.
// The cell is the major key: consecutive buckets then lie near each other in
// space, and the contiguous share of the order that each XCD walks (see
// xcd_block) touches one region of the BVH (6.6% faster than link set first).
// Counting sort of ray indices: the count pass keeps each ray's bucket and its
// rank among that bucket's rays (the counter value its atomic returned), the
// scan turns counts into bucket starts, and the scatter places ray i at
// start + rank with no further atomics.  A wave whose rays all fall in one
// bucket uses one atomic and keeps its lanes in order.
constexpr uint32_t kOrderBucketsCoarse = 6 * 4096;        // 16^3 cells
constexpr uint32_t kOrderBucketsFine = 6 * 4 * 32768;      // minor signs x 32^3 cells

__device__ __forceinline__ uint32_t spread5(uint32_t v) {  // 5 bits -> every third bit
    return (v & 1u) | ((v & 2u) << 2) | ((v & 4u) << 4) | ((v & 8u) << 6) | ((v & 16u) << 8);
}

struct OrderBox {
    float lo[3], scale[3];  // cell = (o - lo) * scale, scale = cells / extent
    uint32_t cells;         // per axis: 16 (coarse) or 32 (fine)
    int32_t fine;
};

__device__ __forceinline__ uint32_t bucket_of(const float4 &r0, const float4 &r1, const OrderBox &ob,
                                              int32_t force_set) {
    int set = force_set >= 0 ? force_set : pmd::link_set(pmd::v3(r1.x, r1.y, r1.z));
    uint32_t c[3];
    float o[3] = {r0.x, r0.y, r0.z};
    const float cmax = (float)(ob.cells - 1);
    for (int a = 0; a < 3; ++a) {
        float f = (o[a] - ob.lo[a]) * ob.scale[a];
        c[a] = f >= cmax ? ob.cells - 1 : (f > 0.0f ? (uint32_t)f : 0u);  // NaN -> 0
    }
    uint32_t morton = spread5(c[0]) | (spread5(c[1]) << 1) | (spread5(c[2]) << 2);
    if (!ob.fine) return morton * 6u + (uint32_t)set;
    // signs of the two components other than the major axis
    int axis = set >> 1;
    float d[3] = {r1.x, r1.y, r1.z};
    uint32_t sg = (d[(axis + 1) % 3] < 0.0f ? 1u : 0u) | (d[(axis + 2) % 3] < 0.0f ? 2u : 0u);
    return morton * 24u + (uint32_t)set * 4u + sg;
}

// Ray i's two float4 words, read once (non-temporal).
__device__ __forceinline__ void load_ray_nt(const float4 *__restrict__ rays, uint32_t i, float4 &r0, float4 &r1) {
    const NtFloat4 a0 = __builtin_nontemporal_load((const NtFloat4 *)(rays + 2 * (size_t)i));
    const NtFloat4 a1 = __builtin_nontemporal_load((const NtFloat4 *)(rays + 2 * (size_t)i + 1));
    r0 = make_float4(a0.x, a0.y, a0.z, a0.w);
    r1 = make_float4(a1.x, a1.y, a1.z, a1.w);
}

// Wave-aggregated increment when every active lane has the same key.
__device__ __forceinline__ uint32_t bucket_add(uint32_t *counters, uint32_t key) {
    uint32_t k0 = __shfl(key, __ffsll((unsigned long long)__ballot(1)) - 1);
    if (__ballot(key != k0) == 0ull) return pmd::wave_fetch_add(&counters[key], __ballot(1), true);
    return atomicAdd(&counters[key], 1u);
}

// Each thread of the bucketing kernels takes kBucketRays rays (block-strided,
// so each step's loads stay coalesced) and issues their atomics back to back,
// so that their round trips overlap.
constexpr uint32_t kBucketRays = 4;

__global__ __launch_bounds__(kTraceBlock) void k_ray_count(const float4 *__restrict__ rays, uint32_t n, OrderBox ob,
                                                           int32_t force_set, uint32_t *__restrict__ counts,
                                                           uint2 *__restrict__ key_rank) {
    const uint32_t i0 = blockIdx.x * (kTraceBlock * kBucketRays) + threadIdx.x;
    uint32_t key[kBucketRays], rank[kBucketRays];
    if (i0 + (kBucketRays - 1) * kTraceBlock < n) {  // every ray of the thread exists (all but the last block)
        float4 r0[kBucketRays], r1[kBucketRays];
#pragma unroll
        for (uint32_t j = 0; j < kBucketRays; ++j) load_ray_nt(rays, i0 + j * kTraceBlock, r0[j], r1[j]);
        bool uniform = false;  // some step's keys are equal across the wave
#pragma unroll
        for (uint32_t j = 0; j < kBucketRays; ++j) {
            key[j] = bucket_of(r0[j], r1[j], ob, force_set);
            uniform |= __ballot(key[j] != __shfl(key[j], __ffsll((unsigned long long)__ballot(1)) - 1)) == 0ull;
        }
        if (uniform) {  // wave-uniform branch
#pragma unroll
            for (uint32_t j = 0; j < kBucketRays; ++j) rank[j] = bucket_add(counts, key[j]);
        } else {
#pragma unroll
            for (uint32_t j = 0; j < kBucketRays; ++j) rank[j] = atomicAdd(&counts[key[j]], 1u);
        }
#pragma unroll
        for (uint32_t j = 0; j < kBucketRays; ++j) {
            const NtUint2 kr = {key[j], rank[j]};
            __builtin_nontemporal_store(kr, (NtUint2 *)(key_rank + i0 + j * kTraceBlock));
        }
    } else {
#pragma unroll
        for (uint32_t j = 0; j < kBucketRays; ++j) {
            const uint32_t i = i0 + j * kTraceBlock;
            if (i < n) {
                float4 r0, r1;
                load_ray_nt(rays, i, r0, r1);
                const uint32_t k = bucket_of(r0, r1, ob, force_set);
                const NtUint2 kr = {k, bucket_add(counts, k)};
                __builtin_nontemporal_store(kr, (NtUint2 *)(key_rank + i));
            }
        }
    }
}

// rank < final count of the bucket, so start[key] + rank < n
__global__ __launch_bounds__(kTraceBlock) void k_ray_scatter(const uint2 *__restrict__ key_rank, uint32_t n,
                                                             const uint32_t *__restrict__ start,
                                                             uint32_t *__restrict__ perm) {
    const uint32_t i0 = blockIdx.x * (kTraceBlock * kBucketRays) + threadIdx.x;
    if (i0 + (kBucketRays - 1) * kTraceBlock < n) {  // every ray of the thread exists (all but the last block)
        NtUint2 kr[kBucketRays];
        uint32_t at[kBucketRays];
#pragma unroll
        for (uint32_t j = 0; j < kBucketRays; ++j)
            kr[j] = __builtin_nontemporal_load((const NtUint2 *)(key_rank + i0 + j * kTraceBlock));
#pragma unroll
        for (uint32_t j = 0; j < kBucketRays; ++j) at[j] = start[kr[j].x] + kr[j].y;
#pragma unroll
        for (uint32_t j = 0; j < kBucketRays; ++j) perm[at[j]] = i0 + j * kTraceBlock;
    } else {
#pragma unroll
        for (uint32_t j = 0; j < kBucketRays; ++j) {
            const uint32_t i = i0 + j * kTraceBlock;
            if (i < n) {
                const NtUint2 kr = __builtin_nontemporal_load((const NtUint2 *)(key_rank + i));
                perm[start[kr.x] + kr.y] = i;
            }
        }
    }
}

// Coarse bucketing without global atomics.  Each of up to kHistGroups
// workgroups counts one contiguous chunk of the rays in a histogram in LDS
// (the LDS atomic gives each ray its rank among the chunk's rays of its
// bucket) and writes it as one row of a [chunk][bucket] table.  A scan down
// each column turns the table into each chunk's offset within each bucket and
// gives the bucket totals; the bucket scan turns those into bucket starts; the
// scatter places ray i at start[bucket] + offset[chunk][bucket] + rank.  The
// (bucket, rank) pairs carry the chunk in the bucket word's upper bits.
constexpr uint32_t kHistGroups = 64;
constexpr uint32_t kHistBlock = 1024;
constexpr uint32_t kHistRays = 4;  // rays per thread whose loads go out together
constexpr uint32_t kHistChunkBits = 15;  // bucket < 2^15 in the packed word
static_assert(kOrderBucketsCoarse <= (1u << kHistChunkBits), "coarse bucket exceeds its packed field");

__global__ __launch_bounds__(kHistBlock) void k_hist_count(const float4 *__restrict__ rays, uint32_t n, uint32_t chunk,
                                                           OrderBox ob, int32_t force_set,
                                                           uint32_t *__restrict__ table, uint2 *__restrict__ key_rank) {
    __shared__ uint32_t h[kOrderBucketsCoarse];
    for (uint32_t b = threadIdx.x; b < kOrderBucketsCoarse; b += kHistBlock) h[b] = 0u;
    __syncthreads();
    const uint32_t i0 = blockIdx.x * chunk, i1 = min(n, i0 + chunk);
    const uint32_t tag = blockIdx.x << kHistChunkBits;
    for (uint32_t i = i0 + threadIdx.x; i < i1; i += kHistBlock * kHistRays) {
        float4 r0[kHistRays], r1[kHistRays];
#pragma unroll
        for (uint32_t j = 0; j < kHistRays; ++j)
            if (i + j * kHistBlock < i1) load_ray_nt(rays, i + j * kHistBlock, r0[j], r1[j]);
#pragma unroll
        for (uint32_t j = 0; j < kHistRays; ++j) {
            const uint32_t ij = i + j * kHistBlock;
            if (ij < i1) {
                const uint32_t key = bucket_of(r0[j], r1[j], ob, force_set);
                const NtUint2 kr = {key | tag, atomicAdd(&h[key], 1u)};
                __builtin_nontemporal_store(kr, (NtUint2 *)(key_rank + ij));
            }
        }
    }
    __syncthreads();
    uint32_t *row = table + (size_t)blockIdx.x * kOrderBucketsCoarse;
    for (uint32_t b = threadIdx.x; b < kOrderBucketsCoarse; b += kHistBlock) row[b] = h[b];
}

// Column b of the table: exclusive running sums over the chunks, in place,
// and the bucket's total in counts[b].
__global__ __launch_bounds__(kTraceBlock) void k_hist_columns(uint32_t *__restrict__ table, uint32_t groups,
                                                              uint32_t *__restrict__ counts) {
    const uint32_t b = blockIdx.x * kTraceBlock + threadIdx.x;
    if (b >= kOrderBucketsCoarse) return;
    uint32_t sum = 0u;
    for (uint32_t g0 = 0; g0 < groups; g0 += 8) {
        uint32_t v[8];
#pragma unroll
        for (uint32_t j = 0; j < 8; ++j)
            v[j] = g0 + j < groups ? table[(size_t)(g0 + j) * kOrderBucketsCoarse + b] : 0u;
#pragma unroll
        for (uint32_t j = 0; j < 8; ++j) {
            if (g0 + j < groups) table[(size_t)(g0 + j) * kOrderBucketsCoarse + b] = sum;
            sum += v[j];
        }
    }
    counts[b] = sum;
}

// start[bucket] + offset[chunk][bucket] + rank < n: the offsets of a bucket's
// chunks and the ranks within a chunk count the bucket's rays without gaps.
__global__ __launch_bounds__(kTraceBlock) void k_hist_scatter(const uint2 *__restrict__ key_rank, uint32_t n,
                                                              const uint32_t *__restrict__ start,
                                                              const uint32_t *__restrict__ table,
                                                              uint32_t *__restrict__ perm) {
    const uint32_t i0 = blockIdx.x * (kTraceBlock * kBucketRays) + threadIdx.x;
    NtUint2 kr[kBucketRays];
#pragma unroll
    for (uint32_t j = 0; j < kBucketRays; ++j)
        if (i0 + j * kTraceBlock < n) kr[j] = __builtin_nontemporal_load((const NtUint2 *)(key_rank + i0 + j * kTraceBlock));
#pragma unroll
    for (uint32_t j = 0; j < kBucketRays; ++j) {
        const uint32_t i = i0 + j * kTraceBlock;
        if (i < n) {
            const uint32_t key = kr[j].x & ((1u << kHistChunkBits) - 1u), g = kr[j].x >> kHistChunkBits;
            perm[start[key] + table[(size_t)g * kOrderBucketsCoarse + key] + kr[j].y] = i;
        }
    }
}

// Rays taken in the order of perm.
template <bool kStats, int kWalk>
__global__ __launch_bounds__(kTraceBlock) void k_trace_perm(pmd::Bvh bvh, const float4 *__restrict__ rays,
                                                            const uint32_t *__restrict__ perm, uint32_t n,
                                                            int32_t *__restrict__ hit, float *__restrict__ tout,
                                                            int32_t force_set, uint32_t *__restrict__ counters,
                                                            uint32_t late) {
    const uint64_t lane = (uint64_t)pmd::xcd_block(blockIdx.x, gridDim.x) * blockDim.x + threadIdx.x;
    trace_slot<kStats, kWalk, true>(bvh, rays, perm, lane, n, hit, tout, force_set, counters, late, 0u);
}

// Two batches in one launch: the first blocksA workgroups walk batch A in
// the order of perm (postponed leaf tests); the rest take batch B, an image
// tile_w wide, one 8x8 pixel tile per wavefront, as packets.  The dispatcher
// hands out B's workgroups once all of A's are running, so B fills the
// device as A's last wavefronts drain.
template <bool kStats>
__global__ __launch_bounds__(kTraceBlock) void k_trace_perm_then_tiles(
    pmd::Bvh bvh, uint32_t blocksA, const float4 *__restrict__ raysA, const uint32_t *__restrict__ perm, uint32_t nA,
    int32_t *__restrict__ hitA, float *__restrict__ tA, int32_t setA, uint32_t *__restrict__ countersA, uint32_t late,
    const float4 *__restrict__ raysB, int64_t nB, int32_t *__restrict__ hitB, float *__restrict__ tB, int32_t setB,
    uint32_t *__restrict__ countersB, uint32_t tile_w) {
    if (blockIdx.x < blocksA) {
        const uint64_t lane = (uint64_t)pmd::xcd_block(blockIdx.x, blocksA) * blockDim.x + threadIdx.x;
        trace_slot<kStats, kWalkPostponed, true>(bvh, raysA, perm, lane, nA, hitA, tA, setA, countersA, late, 0u);
    } else {
        const uint64_t lane =
            (uint64_t)pmd::xcd_block(blockIdx.x - blocksA, gridDim.x - blocksA) * blockDim.x + threadIdx.x;
        trace_slot<kStats, kWalkPacket, false>(bvh, raysB, nullptr, lane, (uint64_t)nB, hitB, tB, setB, countersB, 0u,
                                               tile_w);
    }
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
    b->n_refs = h.n_refs;
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
    b->pos_of.assign((size_t)h.n_tri, -1);
    for (int64_t k = 0; k < h.n_refs; ++k) {
        int32_t &p = b->pos_of[h.tris[(size_t)k * kTriWords + 9]];
        if (p < 0) p = (int32_t)k;
    }
    PM_HIP(hipGetDevice(&b->device));
    size_t nb = h.nodes.size() * sizeof(uint32_t), tb = h.tris.size() * sizeof(uint32_t);
    // zeroed pad nodes after the six arrays (a packet walk reads the node after the one it visits)
    PM_HIP(hipMalloc(&b->d_nodes, nb + sizeof(uint4) * pm::kPadNodes));
    PM_HIP(hipMemsetAsync((char *)b->d_nodes + nb, 0, sizeof(uint4) * pm::kPadNodes, s));
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
    if (b->d_perm) (void)hipFree(b->d_perm);
    if (b->d_order) (void)hipFree(b->d_order);
    for (int k = 0; k < PM_MAX_TRACE_BATCHES; ++k) {
        if (b->side[k]) (void)hipStreamDestroy(b->side[k]);
        if (b->ev_join[k]) (void)hipEventDestroy(b->ev_join[k]);
        b->side[k] = nullptr;
        b->ev_join[k] = nullptr;
    }
    if (b->ev_fork) (void)hipEventDestroy(b->ev_fork);
    b->ev_fork = nullptr;
    b->d_perm = nullptr;
    b->d_order = nullptr;
    b->perm_cap = 0;
    b->d_nodes = nullptr;
    b->d_tris = nullptr;
    b->d_next = nullptr;
}

// Workgroups of the persistent kernel that fill a device, cached per device
// (0: not computed yet); any host thread may call this.
constexpr int kMaxDevices = 64;
static std::atomic<uint32_t> g_persistent_grid[kMaxDevices];

static int persistent_grid(int device, uint32_t &grid) {
    if (device < 0 || device >= kMaxDevices) return set_error("device index out of range"), PM_ERR_ARG;
    grid = g_persistent_grid[device].load(std::memory_order_relaxed);
    if (grid != 0) return PM_OK;
    int cus = 0, per_cu = 0;
    PM_HIP(hipDeviceGetAttribute(&cus, hipDeviceAttributeMultiprocessorCount, device));
    PM_HIP(hipOccupancyMaxActiveBlocksPerMultiprocessor(&per_cu, k_trace_persistent<false>, kTraceBlock, 0));
    grid = (uint32_t)std::max(1, cus * std::max(1, per_cu));
    g_persistent_grid[device].store(grid, std::memory_order_relaxed);  // racing threads store the same value
    return PM_OK;
}

// Rays per wavefront of the slice kernel: the given count, else enough
// wavefronts for two per wavefront slot of the device (at least 64 rays).
static int slice_rays(int device, int64_t n, int slice, uint32_t &out) {
    if (slice > 0) {
        out = (uint32_t)slice;
        return PM_OK;
    }
    uint32_t grid = 0;
    int rc = persistent_grid(device, grid);
    if (rc) return rc;
    const uint64_t waves = 2ull * grid * (kTraceBlock / 64);
    uint64_t per = ((uint64_t)n + waves - 1) / waves;
    per = (per + 63) / 64 * 64;
    out = (uint32_t)std::max<uint64_t>(64, per);
    return PM_OK;
}

static int launch_slices(const pm_bvh *b, const pmd::Bvh &bvh, const float *rays, uint32_t n, int32_t *hit,
                         float *t, int link_set, uint32_t *counters, uint32_t late, int slice, uint32_t block,
                         const uint32_t *perm, hipStream_t s) {
    uint32_t per = 0;
    int rc = slice_rays(b->device, n, slice, per);
    if (rc) return rc;
    const uint64_t waves = ((uint64_t)n + per - 1) / per;
    const uint64_t blocks = (waves * 64 + block - 1) / block;
    if (blocks > 0x7fffffffull) return set_error("too many rays for one launch"), PM_ERR_ARG;
    hipLaunchKernelGGL(counters ? k_trace_slices<true> : k_trace_slices<false>, dim3((uint32_t)blocks), dim3(block),
                       0, s, bvh, (const float4 *)rays, perm, n, hit, t, link_set, counters, late, per);
    PM_HIP(hipGetLastError());
    return PM_OK;
}

static int walk_of(int kernel) {
    switch (kernel) {
    case PM_TRACE_PAIRED: return kWalkPaired;
    case PM_TRACE_POSTPONED: return kWalkPostponed;
    case PM_TRACE_TWO_RAYS: return kWalkTwo;
    case PM_TRACE_PACKET: return kWalkPacket;
    default: return kWalkStep;
    }
}

template <class K>
static K pick_walk(int wk, K step, K paired, K postponed, K two, K packet) {
    return wk == kWalkPaired       ? paired
           : wk == kWalkPostponed ? postponed
           : wk == kWalkTwo       ? two
           : wk == kWalkPacket    ? packet
                                  : step;
}

static int launch_persistent(const pm_bvh *b, const pmd::Bvh &bvh, const float *rays, uint32_t n, int32_t *hit,
                             float *t, int link_set, uint32_t *counters, int refill, const uint32_t *perm,
                             hipStream_t s) {
    uint32_t grid = 0;
    int rc = persistent_grid(b->device, grid);
    if (rc) return rc;
    uint32_t rf = refill > 0 ? (uint32_t)refill : 16u;
    hipLaunchKernelGGL(k_reset_counter, dim3(1), dim3(64), 0, s, b->d_next);
    auto kern = counters ? k_trace_persistent<true> : k_trace_persistent<false>;
    hipLaunchKernelGGL(kern, dim3(grid), dim3(kTraceBlock), 0, s, bvh, (const float4 *)rays, n, hit, t, link_set,
                       counters, b->d_next, rf, perm);
    PM_HIP(hipGetLastError());
    return PM_OK;
}

// Scratch of the bucketed trace: the ray order [perm_cap] followed, at an
// 8-byte aligned offset, by each ray's (bucket, rank) [perm_cap]; and the
// bucket arrays (counts, starts, fill cursors, scan block sums).
struct BucketScratch {
    uint32_t *perm;
    uint64_t perm_cap;
    uint32_t *order;
};
constexpr size_t kOrderWords = (3 * (size_t)kOrderBucketsFine + 1 + kOrderBucketsFine / 4096 + 1 + 63) & ~size_t(63);
// The coarse histogram table sits after the coarse bucket arrays (counts,
// starts, fill cursors, scan block sums), within the fine arrays' words.
constexpr size_t kOrderTableOffset = kOrderBucketsCoarse / 4096 + 1;
static_assert(3 * (size_t)kOrderBucketsCoarse + 1 + kOrderTableOffset + (size_t)kHistGroups * kOrderBucketsCoarse <=
                  kOrderWords,
              "coarse histogram table exceeds the bucket scratch");

constexpr size_t perm_words(uint64_t cap) { return 3 * (size_t)cap + 2; }

// The BVH handle's own scratch, grown (after the stream's work) for more rays.
static int bvh_scratch(pm_bvh *b, int64_t n, hipStream_t s, BucketScratch &sc) {
    if ((uint64_t)n > b->perm_cap) {
        if (b->d_perm) {
            PM_HIP(hipStreamSynchronize(s));
            PM_HIP(hipFree(b->d_perm));
            b->d_perm = nullptr;
        }
        PM_HIP(hipMalloc(&b->d_perm, sizeof(uint32_t) * perm_words((uint64_t)n)));
        b->perm_cap = (uint64_t)n;
    }
    if (!b->d_order) PM_HIP(hipMalloc(&b->d_order, sizeof(uint32_t) * kOrderWords));
    sc = BucketScratch{b->d_perm, b->perm_cap, b->d_order};
    return PM_OK;
}

// Bucket the rays (count, scan, scatter) into sc.perm: kernels only, no allocation.
static int bucket_rays(const pm_bvh *b, const BucketScratch &sc, const float *rays, int64_t n, int link_set,
                       int reorder, hipStream_t s) {
    const uint32_t nbk = reorder == 2 ? kOrderBucketsFine : kOrderBucketsCoarse;
    uint32_t *counts = sc.order, *start = counts + nbk, *fill = start + nbk + 1;
    uint32_t *bsum = fill + nbk;
    OrderBox ob;
    ob.cells = reorder == 2 ? 32u : 16u;
    ob.fine = reorder == 2;
    for (int a = 0; a < 3; ++a) {
        float ext = b->hi[a] - b->lo[a];
        ob.lo[a] = b->lo[a];
        ob.scale[a] = ext > 0.0f ? (float)ob.cells / ext : 0.0f;
    }
    const uint32_t nn = (uint32_t)n;
    const uint32_t blocks = (uint32_t)((n + kTraceBlock * kBucketRays - 1) / (kTraceBlock * kBucketRays));
    uint2 *key_rank = (uint2 *)(sc.perm + ((sc.perm_cap + 1) & ~uint64_t(1)));
    if (reorder != 2) {
        // histograms in LDS: one chunk of at least 4096 rays per workgroup, at most kHistGroups chunks
        uint32_t *table = bsum + kOrderTableOffset;
        const uint32_t groups = (uint32_t)std::min<int64_t>(kHistGroups, (n + 4095) / 4096);
        const uint32_t chunk = (uint32_t)((n + groups - 1) / groups);
        hipLaunchKernelGGL(k_hist_count, dim3(groups), dim3(kHistBlock), 0, s, (const float4 *)rays, nn, chunk, ob,
                           link_set, table, key_rank);
        hipLaunchKernelGGL(k_hist_columns, dim3((nbk + kTraceBlock - 1) / kTraceBlock), dim3(kTraceBlock), 0, s, table,
                           groups, counts);
        launch_bucket_scan(counts, start, fill, bsum, nbk, s);
        hipLaunchKernelGGL(k_hist_scatter, dim3(blocks), dim3(kTraceBlock), 0, s, (const uint2 *)key_rank, nn,
                           (const uint32_t *)start, (const uint32_t *)table, sc.perm);
    } else {
        hipLaunchKernelGGL(k_fill_u32, dim3((nbk + 255) / 256), dim3(256), 0, s, counts, nbk, 0u);
        hipLaunchKernelGGL(k_ray_count, dim3(blocks), dim3(kTraceBlock), 0, s, (const float4 *)rays, nn, ob, link_set,
                           counts, key_rank);
        launch_bucket_scan(counts, start, fill, bsum, nbk, s);
        hipLaunchKernelGGL(k_ray_scatter, dim3(blocks), dim3(kTraceBlock), 0, s, (const uint2 *)key_rank, nn,
                           (const uint32_t *)start, sc.perm);
    }
    PM_HIP(hipGetLastError());
    return PM_OK;
}

static int launch_trace_reordered(const pm_bvh *b, const BucketScratch &sc, const pmd::Bvh &bvh, const float *rays,
                                  int64_t n, int32_t *hit, float *t, int link_set, uint32_t *counters, int kernel,
                                  uint32_t late, int reorder, uint32_t block, int slice, hipStream_t s) {
    int rc = bucket_rays(b, sc, rays, n, link_set, reorder, s);
    if (rc) return rc;
    const uint32_t nn = (uint32_t)n;
    if (kernel == PM_TRACE_PERSISTENT)
        return launch_persistent(b, bvh, rays, nn, hit, t, link_set, counters, (int)late, sc.perm, s);
    if (kernel == PM_TRACE_SLICES)
        return launch_slices(b, bvh, rays, nn, hit, t, link_set, counters, late, slice, block, sc.perm, s);
    using Kern = void (*)(pmd::Bvh, const float4 *, const uint32_t *, uint32_t, int32_t *, float *, int32_t,
                          uint32_t *, uint32_t);
    const int wk = walk_of(kernel);
    Kern kern = counters ? pick_walk<Kern>(wk, k_trace_perm<true, kWalkStep>, k_trace_perm<true, kWalkPaired>,
                                           k_trace_perm<true, kWalkPostponed>, k_trace_perm<true, kWalkTwo>,
                                           k_trace_perm<true, kWalkPacket>)
                         : pick_walk<Kern>(wk, k_trace_perm<false, kWalkStep>, k_trace_perm<false, kWalkPaired>,
                                           k_trace_perm<false, kWalkPostponed>, k_trace_perm<false, kWalkTwo>,
                                           k_trace_perm<false, kWalkPacket>);
    const uint32_t lanes = wk == kWalkTwo ? (nn + 1) / 2 : nn;
    hipLaunchKernelGGL(kern, dim3((lanes + block - 1) / block), dim3(block), 0, s, bvh, (const float4 *)rays,
                       (const uint32_t *)sc.perm, nn, hit, t, link_set, counters, late);
    PM_HIP(hipGetLastError());
    return PM_OK;
}

// Scratch of the allocation-free bucketed trace: one array per device, set
// aside when the library's code is loaded on that device and kept until the
// process ends.  Host code must not pass `scratch` itself to a kernel (its
// host-side name is not a device address): it uses the address that
// hipGetSymbolAddress returns for the current device.
static __device__ __align__(256) uint32_t scratch[kOrderWords + perm_words(PM_NOALLOC_MAX_RAYS)];

static std::mutex g_scratch_mu;
static void *g_scratch_ptr[kMaxDevices];

static int noalloc_scratch(int device, BucketScratch &sc) {
    if (device < 0 || device >= kMaxDevices) return set_error("device index out of range"), PM_ERR_ARG;
    void *ptr = nullptr;
    {
        std::lock_guard<std::mutex> lock(g_scratch_mu);
        if (!g_scratch_ptr[device]) {
            // the first call on this device (which is current): look the array up once
            PM_HIP(hipGetSymbolAddress(&g_scratch_ptr[device], HIP_SYMBOL(scratch)));
            if (!g_scratch_ptr[device]) return set_error("scratch array has no device address"), PM_ERR_HIP;
        }
        ptr = g_scratch_ptr[device];
    }
    uint32_t *base = (uint32_t *)ptr;
    sc = BucketScratch{base + kOrderWords, (uint64_t)PM_NOALLOC_MAX_RAYS, base};
    return PM_OK;
}

int launch_trace(const pm_bvh *b, const TraceArgs &a, hipStream_t s) {
    const int64_t n = a.n;
    const int block = a.block == 0 ? kDefaultWalkBlock : a.block;
    int kernel = a.kernel;
    if (n == 0) return PM_OK;
    pmd::Bvh bvh = make_device_bvh(b);
    // the postponed and slice walks read their threshold from the refill
    // option (and the persistent one its refill count)
    const uint32_t late = kernel == PM_TRACE_POSTPONED || kernel == PM_TRACE_PERSISTENT || kernel == PM_TRACE_SLICES
                              ? (uint32_t)a.refill
                              : 0u;
    if (a.reorder) {
        BucketScratch sc;
        int rc = bvh_scratch(const_cast<pm_bvh *>(b), n, s, sc);
        if (rc) return rc;
        return launch_trace_reordered(b, sc, bvh, a.rays, n, a.hit, a.t, a.link_set, a.counters, kernel, late,
                                      a.reorder, (uint32_t)block, a.slice, s);
    }
    if (kernel == 0) kernel = PM_TRACE_PER_RAY;
    if (kernel == PM_TRACE_PERSISTENT || kernel == PM_TRACE_SLICES) {
        if (n >= (int64_t(1) << 31)) {
            set_error("too many rays for one launch");
            return PM_ERR_ARG;
        }
        if (kernel == PM_TRACE_SLICES)
            return launch_slices(b, bvh, a.rays, (uint32_t)n, a.hit, a.t, a.link_set, a.counters, late, a.slice,
                                 (uint32_t)block, nullptr, s);
        return launch_persistent(b, bvh, a.rays, (uint32_t)n, a.hit, a.t, a.link_set, a.counters, a.refill, nullptr,
                                 s);
    }
    const int wk = walk_of(kernel);
    int64_t lanes = wk == kWalkTwo ? (n + 1) / 2 : n;
    if (a.tile_w > 0) {  // one wave per 8x8 tile of a tile_w x (n / tile_w) image
        const int64_t tiles = ((a.tile_w + 7) / 8) * ((n / a.tile_w + 7) / 8);
        lanes = tiles * 64;
    }
    int64_t nblk = (lanes + block - 1) / block;
    if (nblk > 0x7fffffff) {
        set_error("too many rays for one launch");
        return PM_ERR_ARG;
    }
    using Kern = void (*)(pmd::Bvh, const float4 *, int64_t, int32_t *, float *, int32_t, uint32_t *, uint32_t,
                          uint32_t);
    Kern kern = a.counters ? pick_walk<Kern>(wk, k_trace<true, kWalkStep>, k_trace<true, kWalkPaired>,
                                             k_trace<true, kWalkPostponed>, k_trace<true, kWalkTwo>,
                                             k_trace<true, kWalkPacket>)
                           : pick_walk<Kern>(wk, k_trace<false, kWalkStep>, k_trace<false, kWalkPaired>,
                                             k_trace<false, kWalkPostponed>, k_trace<false, kWalkTwo>,
                                             k_trace<false, kWalkPacket>);
    hipLaunchKernelGGL(kern, dim3((uint32_t)nblk), dim3(block), 0, s, bvh, (const float4 *)a.rays, n, a.hit, a.t,
                       a.link_set, a.counters, late, (uint32_t)a.tile_w);
    PM_HIP(hipGetLastError());
    return PM_OK;
}

static int launch_perm_then_tiles(pm_bvh *b, const TraceArgs &A, const TraceArgs &B, int block, hipStream_t s) {
    BucketScratch sc;
    int rc = bvh_scratch(b, A.n, s, sc);
    if (rc) return rc;
    rc = bucket_rays(b, sc, A.rays, A.n, A.link_set, A.reorder, s);
    if (rc) return rc;
    const pmd::Bvh bvh = make_device_bvh(b);
    const uint32_t nA = (uint32_t)A.n;
    const uint64_t blocksA = ((uint64_t)nA + block - 1) / block;
    const int64_t tiles = (((int64_t)B.tile_w + 7) / 8) * ((B.n / B.tile_w + 7) / 8);
    const uint64_t blocksB = ((uint64_t)tiles * 64 + block - 1) / block;
    if (blocksA + blocksB > 0x7fffffffull) return set_error("too many rays for one launch"), PM_ERR_ARG;
    hipLaunchKernelGGL(A.counters ? k_trace_perm_then_tiles<true> : k_trace_perm_then_tiles<false>,
                       dim3((uint32_t)(blocksA + blocksB)), dim3(block), 0, s, bvh, (uint32_t)blocksA,
                       (const float4 *)A.rays, (const uint32_t *)sc.perm, nA, A.hit, A.t, A.link_set, A.counters,
                       (uint32_t)A.refill, (const float4 *)B.rays, B.n, B.hit, B.t, B.link_set, B.counters,
                       (uint32_t)B.tile_w);
    PM_HIP(hipGetLastError());
    return PM_OK;
}

int launch_trace_multi(pm_bvh *b, const TraceArgs *batches, int32_t n_batches, hipStream_t s) {
    auto one = [&](const TraceArgs &a, hipStream_t st) { return launch_trace(b, a, st); };
    if (n_batches == 1) return one(batches[0], s);
    if (n_batches == 2) {  // bucketed postponed walk + packets over image tiles: one launch for both
        for (int k = 0; k < 2; ++k) {
            const TraceArgs &A = batches[k], &B = batches[1 - k];
            const int blk = A.block ? A.block : kDefaultWalkBlock;
            if (A.reorder != 0 && A.kernel == PM_TRACE_POSTPONED && A.n > 0 && B.kernel == PM_TRACE_PACKET &&
                B.tile_w > 0 && B.reorder == 0 && B.n > 0 && (B.block ? B.block : kDefaultWalkBlock) == blk &&
                (A.counters == nullptr) == (B.counters == nullptr))
                return launch_perm_then_tiles(b, A, B, blk, s);
        }
    }
    if (!b->ev_fork) PM_HIP(hipEventCreateWithFlags(&b->ev_fork, hipEventDisableTiming));
    for (int32_t k = 1; k < n_batches; ++k) {
        if (!b->side[k]) PM_HIP(hipStreamCreateWithFlags(&b->side[k], hipStreamNonBlocking));
        if (!b->ev_join[k]) PM_HIP(hipEventCreateWithFlags(&b->ev_join[k], hipEventDisableTiming));
    }
    PM_HIP(hipEventRecord(b->ev_fork, s));
    for (int32_t k = 1; k < n_batches; ++k) PM_HIP(hipStreamWaitEvent(b->side[k], b->ev_fork, 0));
    int rc = PM_OK;
    for (int32_t k = 0; k < n_batches && rc == PM_OK; ++k) rc = one(batches[k], k == 0 ? s : b->side[k]);
    // join every side stream, also after a failed launch, so that s never runs ahead of them
    for (int32_t k = 1; k < n_batches; ++k) {
        PM_HIP(hipEventRecord(b->ev_join[k], b->side[k]));
        PM_HIP(hipStreamWaitEvent(s, b->ev_join[k], 0));
    }
    return rc;
}

int launch_trace_noalloc(const pm_bvh *b, const TraceArgs &a, hipStream_t s) {
    const int64_t n = a.n;
    if (n > (int64_t)PM_NOALLOC_MAX_RAYS) return set_error("n exceeds PM_NOALLOC_MAX_RAYS"), PM_ERR_ARG;
    if (a.reorder != 1 && a.reorder != 2)
        return set_error("the allocation-free trace buckets the rays: reorder 1 or 2"), PM_ERR_ARG;
    int dev = -1;
    PM_HIP(hipGetDevice(&dev));
    if (dev != b->device) return set_error("the BVH lives on another device than the current one"), PM_ERR_ARG;
    BucketScratch sc;
    int rc = noalloc_scratch(dev, sc);
    if (rc) return rc;
    if (n == 0) return PM_OK;
    const int block = a.block == 0 ? kDefaultWalkBlock : a.block;
    const int kernel = a.kernel;
    const uint32_t late = kernel == PM_TRACE_POSTPONED || kernel == PM_TRACE_PERSISTENT || kernel == PM_TRACE_SLICES
                              ? (uint32_t)a.refill
                              : 0u;
    return launch_trace_reordered(b, sc, make_device_bvh(b), a.rays, n, a.hit, a.t, a.link_set, a.counters, kernel,
                                  late, a.reorder, (uint32_t)block, a.slice, s);
}

}  // namespace pm
