// GPU construction of the multiple-threaded BVH (Sec. 3.1) from sorted Morton
// codes: a linear BVH (Karras 2012's radix tree over the sorted centroid
// codes), the GPU build the paper names as future work (Sec. 4.1).  It
// produces the same device layout as the host SAH build -- six preorder copies
// of 16-byte quantised nodes, one per link set, and 48-byte triangles in leaf
// order -- so every traversal kernel and the renderer use it unchanged.
//
// Steps (all on the device, on the caller's stream):
//   1. triangle boxes; scene and centroid bounds (block partials, one reduce)
//   2. 30-bit Morton code of each centroid; stable radix sort of the indices
//   3. radix tree: internal node i splits its key range at the highest
//      differing bit (keys made unique by their sorted position)
//   4. depth of every internal node; boxes, triangle counts and collapsed
//      subtree sizes level by level from the deepest (one launch per level, so
//      no kernel waits on another workgroup's writes)
//   5. subtrees of at most max_leaf triangles become leaves; each kept node's
//      index in the six preorders is the sum, over its ancestors, of 1 plus
//      the size of the earlier sibling when it is the later child (children
//      ordered by box centre along each set's direction, ties to the left)
//   6. quantised node records and triangle records
#include <hip/hip_runtime.h>
#include <hipcub/device/device_radix_sort.hpp>

#include <algorithm>
#include <chrono>
#include <cmath>
#include <vector>

#include "bvh_build.h"
#include "runtime.h"

namespace {

constexpr int kLb = 256;

inline uint32_t lb_blocks(int64_t n) { return (uint32_t)((n + kLb - 1) / kLb); }

// Per triangle: box [lo.xyz, hi.xyz]; per block: partial bounds of the
// vertices (vlo, vhi) and of the box centres (clo, chi).
__global__ __launch_bounds__(kLb) void k_lb_boxes(const float *__restrict__ verts, uint32_t n,
                                                  float *__restrict__ tbox, float *__restrict__ part) {
    __shared__ float red[kLb / 64][12];
    const uint32_t i = blockIdx.x * kLb + threadIdx.x;
    float v[12];
    for (int a = 0; a < 3; ++a) {
        v[a] = INFINITY;       // vertex lo
        v[3 + a] = -INFINITY;  // vertex hi
        v[6 + a] = INFINITY;   // centre lo
        v[9 + a] = -INFINITY;  // centre hi
    }
    if (i < n) {
        float lo[3], hi[3];
        for (int a = 0; a < 3; ++a) {
            float x0 = verts[9 * (size_t)i + a], x1 = verts[9 * (size_t)i + 3 + a], x2 = verts[9 * (size_t)i + 6 + a];
            lo[a] = fminf(fminf(x0, x1), x2);
            hi[a] = fmaxf(fmaxf(x0, x1), x2);
            tbox[6 * (size_t)i + a] = lo[a];
            tbox[6 * (size_t)i + 3 + a] = hi[a];
            float c = 0.5f * (lo[a] + hi[a]);
            v[a] = lo[a];
            v[3 + a] = hi[a];
            v[6 + a] = c;
            v[9 + a] = c;
        }
    }
    for (int off = 32; off > 0; off >>= 1)
        for (int a = 0; a < 3; ++a) {
            v[a] = fminf(v[a], __shfl_xor(v[a], off));
            v[3 + a] = fmaxf(v[3 + a], __shfl_xor(v[3 + a], off));
            v[6 + a] = fminf(v[6 + a], __shfl_xor(v[6 + a], off));
            v[9 + a] = fmaxf(v[9 + a], __shfl_xor(v[9 + a], off));
        }
    if ((threadIdx.x & 63) == 0)
        for (int c = 0; c < 12; ++c) red[threadIdx.x >> 6][c] = v[c];
    __syncthreads();
    if (threadIdx.x < 12) {
        const int c = threadIdx.x;
        const bool is_min = (c / 3) % 2 == 0;
        float r = red[0][c];
        for (int w = 1; w < kLb / 64; ++w) r = is_min ? fminf(r, red[w][c]) : fmaxf(r, red[w][c]);
        part[12 * (size_t)blockIdx.x + c] = r;
    }
}

__global__ __launch_bounds__(kLb) void k_lb_reduce(const float *__restrict__ part, uint32_t nblk,
                                                   float *__restrict__ out) {
    if (threadIdx.x >= 12) return;
    const int c = threadIdx.x;
    const bool is_min = (c / 3) % 2 == 0;
    float r = part[c];
    for (uint32_t b = 1; b < nblk; ++b) r = is_min ? fminf(r, part[12 * (size_t)b + c]) : fmaxf(r, part[12 * (size_t)b + c]);
    out[c] = r;
}

__device__ __forceinline__ uint32_t spread10(uint32_t v) {  // 10 bits -> every third bit
    v &= 0x3ffu;
    v = (v | (v << 16)) & 0x030000ffu;
    v = (v | (v << 8)) & 0x0300f00fu;
    v = (v | (v << 4)) & 0x030c30c3u;
    v = (v | (v << 2)) & 0x09249249u;
    return v;
}

struct CentreMap {
    float lo[3], scale[3];  // cell = (c - lo) * scale, scale = 1024 / extent (0 for a flat axis)
};

__global__ __launch_bounds__(kLb) void k_lb_morton(const float *__restrict__ tbox, uint32_t n, CentreMap cm,
                                                   uint32_t *__restrict__ code, uint32_t *__restrict__ idx) {
    const uint32_t i = blockIdx.x * kLb + threadIdx.x;
    if (i >= n) return;
    uint32_t q[3];
    for (int a = 0; a < 3; ++a) {
        float c = 0.5f * (tbox[6 * (size_t)i + a] + tbox[6 * (size_t)i + 3 + a]);
        float f = (c - cm.lo[a]) * cm.scale[a];
        q[a] = f >= 1023.0f ? 1023u : (f > 0.0f ? (uint32_t)f : 0u);
    }
    code[i] = spread10(q[0]) | (spread10(q[1]) << 1) | (spread10(q[2]) << 2);
    idx[i] = i;
}

// Length of the common prefix of sorted keys i and j, the key being the Morton
// code followed by the sorted position (so keys are unique); -1 outside.
__device__ __forceinline__ int lb_delta(const uint32_t *__restrict__ code, int n, int i, int j) {
    if (j < 0 || j >= n) return -1;
    uint32_t a = code[i], b = code[j];
    if (a != b) return __clz(a ^ b);
    return 32 + __clz((uint32_t)i ^ (uint32_t)j);
}

// Node numbering: internal nodes 0 .. n-2 (0 is the root), leaf k (sorted
// position k) is node n-1+k.  For n = 1 the single leaf is node 0.
__global__ __launch_bounds__(kLb) void k_lb_tree(const uint32_t *__restrict__ code, int n, int32_t *__restrict__ left,
                                                 int32_t *__restrict__ right, int32_t *__restrict__ parent,
                                                 int32_t *__restrict__ rlo, int32_t *__restrict__ rhi) {
    const int i = (int)(blockIdx.x * kLb + threadIdx.x);
    if (i >= n - 1) return;
    const int d = lb_delta(code, n, i, i + 1) > lb_delta(code, n, i, i - 1) ? 1 : -1;
    const int dmin = lb_delta(code, n, i, i - d);
    int lmax = 2;
    while (lb_delta(code, n, i, i + lmax * d) > dmin) lmax *= 2;
    int l = 0;
    for (int t = lmax / 2; t >= 1; t /= 2)
        if (lb_delta(code, n, i, i + (l + t) * d) > dmin) l += t;
    const int j = i + l * d;
    const int dnode = lb_delta(code, n, i, j);
    int s = 0, t = l;
    do {
        t = (t + 1) / 2;
        if (lb_delta(code, n, i, i + (s + t) * d) > dnode) s += t;
    } while (t > 1);
    const int gamma = i + s * d + min(d, 0);
    const int lo = min(i, j), hi = max(i, j);
    const int lc = lo == gamma ? n - 1 + gamma : gamma;
    const int rc = hi == gamma + 1 ? n - 1 + gamma + 1 : gamma + 1;
    left[i] = lc;
    right[i] = rc;
    parent[lc] = i;
    parent[rc] = i;
    rlo[i] = lo;
    rhi[i] = hi;
    if (i == 0) parent[0] = -1;
}

// A radix tree over unique keys of at most 62 bits is at most 62 deep; the
// walks up the tree stop at kMaxWalk steps and flag an error instead.
constexpr int kMaxWalk = 128;

__global__ __launch_bounds__(kLb) void k_lb_depth(const int32_t *__restrict__ parent, int n_internal,
                                                  int32_t *__restrict__ depth, uint32_t *__restrict__ max_depth,
                                                  uint32_t *__restrict__ bad) {
    const int i = (int)(blockIdx.x * kLb + threadIdx.x);
    if (i >= n_internal) return;
    int dep = 0;
    for (int v = i; v > 0 && dep < kMaxWalk; v = parent[v]) dep++;
    if (dep >= kMaxWalk) atomicOr(bad, 1u);
    depth[i] = dep;
    atomicMax(max_depth, (uint32_t)dep);
}

// Leaves: box of their triangle, one triangle, collapsed size 1.
__global__ __launch_bounds__(kLb) void k_lb_leaves(const float *__restrict__ tbox, const uint32_t *__restrict__ order,
                                                   int n, float *__restrict__ nbox, int32_t *__restrict__ cnt,
                                                   int32_t *__restrict__ sz, int32_t *__restrict__ rlo,
                                                   int32_t *__restrict__ rhi) {
    const int k = (int)(blockIdx.x * kLb + threadIdx.x);
    if (k >= n) return;
    const int v = n - 1 + k;
    const uint32_t t = order[k];
    for (int c = 0; c < 6; ++c) nbox[6 * (size_t)v + c] = tbox[6 * (size_t)t + c];
    cnt[v] = 1;
    sz[v] = 1;
    rlo[v] = k;
    rhi[v] = k;
}

// Internal nodes at one depth: box union, triangle count and size in the
// collapsed tree (a node of at most max_leaf triangles is one leaf).
__global__ __launch_bounds__(kLb) void k_lb_level(const int32_t *__restrict__ depth, int n_internal, int level,
                                                  const int32_t *__restrict__ left, const int32_t *__restrict__ right,
                                                  int max_leaf, float *__restrict__ nbox, int32_t *__restrict__ cnt,
                                                  int32_t *__restrict__ sz) {
    const int i = (int)(blockIdx.x * kLb + threadIdx.x);
    if (i >= n_internal || depth[i] != level) return;
    const int l = left[i], r = right[i];
    for (int a = 0; a < 3; ++a) {
        nbox[6 * (size_t)i + a] = fminf(nbox[6 * (size_t)l + a], nbox[6 * (size_t)r + a]);
        nbox[6 * (size_t)i + 3 + a] = fmaxf(nbox[6 * (size_t)l + 3 + a], nbox[6 * (size_t)r + 3 + a]);
    }
    const int c = cnt[l] + cnt[r];
    cnt[i] = c;
    sz[i] = c <= max_leaf ? 1 : 1 + sz[l] + sz[r];
}

struct QuantGrid {
    double qlo[3], qstep[3], pad;
};

__device__ __forceinline__ uint32_t lb_q_down(const QuantGrid &g, int a, double x) {
    double q = floor((x - g.qlo[a]) / g.qstep[a]);
    q = fmin(fmax(q, 0.0), 65535.0);
    while (q > 0.0 && g.qlo[a] + q * g.qstep[a] > x) q -= 1.0;
    return (uint32_t)q;
}

__device__ __forceinline__ uint32_t lb_q_up(const QuantGrid &g, int a, double x) {
    double q = ceil((x - g.qlo[a]) / g.qstep[a]);
    q = fmin(fmax(q, 0.0), 65535.0);
    while (q < 65535.0 && g.qlo[a] + q * g.qstep[a] < x) q += 1.0;
    return (uint32_t)q;
}

// Per internal node, bit s set when its right child comes first in link set s
// (s = 2 axis + negative): box centres compared along the axis, ties to the left.
__global__ __launch_bounds__(kLb) void k_lb_order(const int32_t *__restrict__ left, const int32_t *__restrict__ right,
                                                  int n_internal, const float *__restrict__ nbox,
                                                  uint8_t *__restrict__ rfirst) {
    const int i = (int)(blockIdx.x * kLb + threadIdx.x);
    if (i >= n_internal) return;
    const int l = left[i], r = right[i];
    uint32_t m = 0;
    for (int a = 0; a < 3; ++a) {
        float kl = nbox[6 * (size_t)l + a] + nbox[6 * (size_t)l + 3 + a];
        float kr = nbox[6 * (size_t)r + a] + nbox[6 * (size_t)r + 3 + a];
        if (kr < kl) m |= 1u << (2 * a);
        if (kr > kl) m |= 1u << (2 * a + 1);
    }
    rfirst[i] = (uint8_t)m;
}

struct TreeStats {
    unsigned long long leaves;
    uint32_t depth;
    uint32_t bad;  // a walk too long or a preorder index out of range
    double sah;
};

// Every kept node writes its record into each of the six preorders.
__global__ __launch_bounds__(kLb) void k_lb_thread(int n, int max_leaf, const int32_t *__restrict__ parent,
                                                   const int32_t *__restrict__ left, const int32_t *__restrict__ right,
                                                   const uint8_t *__restrict__ rfirst, const float *__restrict__ nbox,
                                                   const int32_t *__restrict__ cnt, const int32_t *__restrict__ sz,
                                                   const int32_t *__restrict__ rlo, QuantGrid g, uint32_t n_nodes,
                                                   double trav_cost, uint4 *__restrict__ nodes,
                                                   TreeStats *__restrict__ stats) {
    const int v = (int)(blockIdx.x * kLb + threadIdx.x);
    if (v >= 2 * n - 1) return;
    const bool leaf = cnt[v] <= max_leaf;
    const int pv = parent[v];
    if (v != 0 && pv < 0) {  // every node but the root has a parent
        atomicOr(&stats->bad, 1u);
        return;
    }
    if (leaf && v != 0 && cnt[pv] <= max_leaf) return;  // inside a collapsed leaf
    uint32_t idx[6] = {0, 0, 0, 0, 0, 0};
    uint32_t dep = 0;
    for (int c = v; c > 0 && dep < (uint32_t)kMaxWalk; c = parent[c]) {
        const int u = parent[c];
        if (u < 0 || u >= n - 1) {  // parents are internal nodes
            atomicOr(&stats->bad, 1u);
            return;
        }
        const uint32_t m = rfirst[u];
        const bool is_right = right[u] == c;
        for (int s = 0; s < 6; ++s) {
            const bool rf = (m >> s) & 1u;
            const int first = rf ? right[u] : left[u];
            idx[s] += (is_right == rf) ? 1u : 1u + (uint32_t)sz[first];
        }
        dep++;
    }
    uint32_t lo3[3], hi3[3];
    for (int a = 0; a < 3; ++a) {
        lo3[a] = lb_q_down(g, a, (double)nbox[6 * (size_t)v + a] - g.pad);
        hi3[a] = lb_q_up(g, a, (double)nbox[6 * (size_t)v + 3 + a] + g.pad);
    }
    uint4 rec;
    rec.x = lo3[0] | (hi3[0] << 16);
    rec.y = lo3[1] | (hi3[1] << 16);
    rec.z = lo3[2] | (hi3[2] << 16);
    if (dep >= (uint32_t)kMaxWalk) {
        atomicOr(&stats->bad, 1u);
        return;
    }
    for (int s = 0; s < 6; ++s) {
        rec.w = leaf ? (0x80000000u | ((uint32_t)rlo[v] << 3) | (uint32_t)cnt[v]) : idx[s] + (uint32_t)sz[v];
        if (idx[s] < n_nodes) nodes[(size_t)s * n_nodes + idx[s]] = rec;
        else atomicOr(&stats->bad, 1u);
    }
    // statistics: SAH cost with C_isect = 1, normalised by the root's area
    double e[3], r[3];
    for (int a = 0; a < 3; ++a) {
        e[a] = (double)nbox[6 * (size_t)v + 3 + a] - (double)nbox[6 * (size_t)v + a];
        r[a] = (double)nbox[3 + a] - (double)nbox[a];
    }
    const double area = e[0] * e[1] + e[1] * e[2] + e[2] * e[0];
    const double root = r[0] * r[1] + r[1] * r[2] + r[2] * r[0];
    const double rel = root > 0.0 ? area / root : 1.0;
    unsafeAtomicAdd(&stats->sah, rel * (leaf ? (double)cnt[v] : trav_cost));
    atomicMax(&stats->depth, dep);
    if (leaf) atomicAdd(&stats->leaves, 1ull);
}

// Triangle records in leaf (sorted) order: v0, v1, v2, original index,
// material.
__global__ __launch_bounds__(kLb) void k_lb_tris(const float *__restrict__ verts, const uint32_t *__restrict__ mats,
                                                 const uint32_t *__restrict__ order, int n, float4 *__restrict__ tris) {
    const int k = (int)(blockIdx.x * kLb + threadIdx.x);
    if (k >= n) return;
    const uint32_t t = order[k];
    const float *p = verts + 9 * (size_t)t;
    tris[3 * (size_t)k] = make_float4(p[0], p[1], p[2], p[3]);
    tris[3 * (size_t)k + 1] = make_float4(p[4], p[5], p[6], p[7]);
    tris[3 * (size_t)k + 2] = make_float4(p[8], __uint_as_float(t), __uint_as_float(mats ? mats[t] : 0u), 0.0f);
}

struct Scratch {
    std::vector<void *> bufs;
    ~Scratch() {
        for (void *b : bufs) (void)hipFree(b);
    }
    template <class T>
    hipError_t alloc(T **p, size_t count) {
        hipError_t e = hipMalloc((void **)p, sizeof(T) * std::max<size_t>(count, 1));
        if (e == hipSuccess) bufs.push_back((void *)*p);
        return e;
    }
};

}  // namespace

namespace pm {

int build_bvh_gpu(const float *verts_h, const uint32_t *mats_h, int64_t n_tri, int max_leaf, double trav_cost,
                  hipStream_t s, pm_bvh *b) {
    const auto t0 = std::chrono::steady_clock::now();
    const int n = (int)n_tri;
    Scratch sc;
    float *verts = nullptr, *tbox = nullptr, *part = nullptr, *bounds = nullptr, *nbox = nullptr;
    uint32_t *mats = nullptr, *code = nullptr, *code_s = nullptr, *idx = nullptr, *order = nullptr,
             *max_depth = nullptr;
    int32_t *left = nullptr, *right = nullptr, *parent = nullptr, *rlo = nullptr, *rhi = nullptr, *depth = nullptr,
            *cnt = nullptr, *sz = nullptr;
    uint8_t *rfirst = nullptr;
    TreeStats *stats = nullptr;
    const int n_int = std::max(n - 1, 0), n_all = 2 * n - 1;
    const uint32_t nblk = lb_blocks(n);
    PM_HIP(sc.alloc(&verts, 9 * (size_t)n));
    PM_HIP(sc.alloc(&mats, (size_t)n));
    PM_HIP(sc.alloc(&tbox, 6 * (size_t)n));
    PM_HIP(sc.alloc(&part, 12 * (size_t)nblk));
    PM_HIP(sc.alloc(&bounds, 12));
    PM_HIP(sc.alloc(&code, (size_t)n));
    PM_HIP(sc.alloc(&code_s, (size_t)n));
    PM_HIP(sc.alloc(&idx, (size_t)n));
    PM_HIP(sc.alloc(&order, (size_t)n));
    PM_HIP(sc.alloc(&left, (size_t)n_int));
    PM_HIP(sc.alloc(&right, (size_t)n_int));
    PM_HIP(sc.alloc(&depth, (size_t)n_int));
    PM_HIP(sc.alloc(&rfirst, (size_t)n_int));
    PM_HIP(sc.alloc(&parent, (size_t)n_all));
    PM_HIP(sc.alloc(&rlo, (size_t)n_all));
    PM_HIP(sc.alloc(&rhi, (size_t)n_all));
    PM_HIP(sc.alloc(&cnt, (size_t)n_all));
    PM_HIP(sc.alloc(&sz, (size_t)n_all));
    PM_HIP(sc.alloc(&nbox, 6 * (size_t)n_all));
    PM_HIP(sc.alloc(&max_depth, 2));  // [0] depth, [1] error flag
    PM_HIP(sc.alloc(&stats, 1));
    PM_HIP(hipMemcpyAsync(verts, verts_h, sizeof(float) * 9 * (size_t)n, hipMemcpyHostToDevice, s));
    if (mats_h) PM_HIP(hipMemcpyAsync(mats, mats_h, sizeof(uint32_t) * (size_t)n, hipMemcpyHostToDevice, s));
    else PM_HIP(hipMemsetAsync(mats, 0, sizeof(uint32_t) * (size_t)n, s));

    // 1. boxes and bounds
    hipLaunchKernelGGL(k_lb_boxes, dim3(nblk), dim3(kLb), 0, s, (const float *)verts, (uint32_t)n, tbox, part);
    hipLaunchKernelGGL(k_lb_reduce, dim3(1), dim3(64), 0, s, (const float *)part, nblk, bounds);
    float bh[12];
    PM_HIP(hipMemcpyAsync(bh, bounds, sizeof(bh), hipMemcpyDeviceToHost, s));
    PM_HIP(hipStreamSynchronize(s));

    // the quantisation grid of the host build: padded scene box, 16-bit steps
    float ext = 0.0f, mag = 0.0f;
    for (int a = 0; a < 3; ++a) {
        ext = std::max(ext, bh[3 + a] - bh[a]);
        mag = std::max(mag, std::max(std::fabs(bh[a]), std::fabs(bh[3 + a])));
    }
    QuantGrid g;
    g.pad = std::max((double)ext * 0x1p-15, (double)mag * 0x1p-20) + 1e-30;
    for (int a = 0; a < 3; ++a) {
        double lo = (double)bh[a] - g.pad, hi = (double)bh[3 + a] + g.pad;
        float l = (float)lo;
        if ((double)l > lo) l = std::nextafter(l, -INFINITY);
        float sf = (float)((hi - (double)l) / 65535.0);
        while ((double)l + 65535.0 * (double)sf < hi) sf = std::nextafter(sf, INFINITY);
        g.qlo[a] = (double)l;
        g.qstep[a] = (double)sf;
        b->lo[a] = bh[a];
        b->hi[a] = bh[3 + a];
        b->qlo[a] = l;
        b->qstep[a] = sf;
    }

    // 2. Morton codes and a stable sort by code
    CentreMap cm;
    for (int a = 0; a < 3; ++a) {
        float e = bh[9 + a] - bh[6 + a];
        cm.lo[a] = bh[6 + a];
        cm.scale[a] = e > 0.0f ? 1024.0f / e : 0.0f;
    }
    hipLaunchKernelGGL(k_lb_morton, dim3(nblk), dim3(kLb), 0, s, (const float *)tbox, (uint32_t)n, cm, code, idx);
    size_t tmp_bytes = 0;
    PM_HIP(hipcub::DeviceRadixSort::SortPairs(nullptr, tmp_bytes, code, code_s, idx, order, n, 0, 30, s));
    void *tmp = nullptr;
    PM_HIP(sc.alloc((uint8_t **)&tmp, tmp_bytes));
    PM_HIP(hipcub::DeviceRadixSort::SortPairs(tmp, tmp_bytes, code, code_s, idx, order, n, 0, 30, s));

    // 3-4. radix tree, depths, boxes level by level
    uint32_t maxd = 0;
    PM_HIP(hipMemsetAsync(parent, 0xff, sizeof(int32_t) * (size_t)n_all, s));  // -1: no parent yet
    if (n_int > 0) {
        hipLaunchKernelGGL(k_lb_tree, dim3(lb_blocks(n_int)), dim3(kLb), 0, s, (const uint32_t *)code_s, n, left,
                           right, parent, rlo, rhi);
        PM_HIP(hipMemsetAsync(max_depth, 0, 2 * sizeof(uint32_t), s));
        hipLaunchKernelGGL(k_lb_depth, dim3(lb_blocks(n_int)), dim3(kLb), 0, s, (const int32_t *)parent, n_int, depth,
                           max_depth, max_depth + 1);
        uint32_t dh[2];
        PM_HIP(hipMemcpyAsync(dh, max_depth, sizeof(dh), hipMemcpyDeviceToHost, s));
        PM_HIP(hipStreamSynchronize(s));
        if (dh[1]) return set_error("GPU BVH build: radix tree walk did not end"), PM_ERR_STATE;
        maxd = dh[0];
    }
    hipLaunchKernelGGL(k_lb_leaves, dim3(nblk), dim3(kLb), 0, s, (const float *)tbox, (const uint32_t *)order, n,
                       nbox, cnt, sz, rlo, rhi);
    PM_HIP(hipStreamSynchronize(s));
    if (n_int > 0) {
        for (int lev = (int)maxd; lev >= 0; --lev)
            hipLaunchKernelGGL(k_lb_level, dim3(lb_blocks(n_int)), dim3(kLb), 0, s, (const int32_t *)depth, n_int, lev,
                               (const int32_t *)left, (const int32_t *)right, max_leaf, nbox, cnt, sz);
        hipLaunchKernelGGL(k_lb_order, dim3(lb_blocks(n_int)), dim3(kLb), 0, s, (const int32_t *)left,
                           (const int32_t *)right, n_int, (const float *)nbox, rfirst);
    }
    int32_t root_sz = 1;
    PM_HIP(hipMemcpyAsync(&root_sz, sz, sizeof(int32_t), hipMemcpyDeviceToHost, s));
    PM_HIP(hipStreamSynchronize(s));

    // 5-6. records
    const uint32_t n_nodes = (uint32_t)root_sz;
    PM_HIP(hipGetDevice(&b->device));
    // zeroed pad nodes after the six arrays (a packet walk reads the node after the one it visits)
    PM_HIP(hipMalloc(&b->d_nodes, sizeof(uint4) * (kLinkSets * (size_t)n_nodes + pm::kPadNodes)));
    PM_HIP(hipMemsetAsync(b->d_nodes + kLinkSets * (size_t)n_nodes, 0, sizeof(uint4) * pm::kPadNodes, s));
    PM_HIP(hipMalloc(&b->d_tris, sizeof(float4) * 3 * (size_t)n));
    PM_HIP(hipMalloc(&b->d_next, 64));
    PM_HIP(hipMemsetAsync(stats, 0, sizeof(TreeStats), s));
    hipLaunchKernelGGL(k_lb_thread, dim3(lb_blocks(n_all)), dim3(kLb), 0, s, n, max_leaf, (const int32_t *)parent,
                       (const int32_t *)left, (const int32_t *)right, (const uint8_t *)rfirst, (const float *)nbox,
                       (const int32_t *)cnt, (const int32_t *)sz, (const int32_t *)rlo, g, n_nodes, trav_cost,
                       b->d_nodes, stats);
    hipLaunchKernelGGL(k_lb_tris, dim3(nblk), dim3(kLb), 0, s, (const float *)verts, (const uint32_t *)mats,
                       (const uint32_t *)order, n, b->d_tris);
    PM_HIP(hipGetLastError());
    TreeStats st;
    std::vector<uint32_t> order_h((size_t)n);
    PM_HIP(hipMemcpyAsync(&st, stats, sizeof(st), hipMemcpyDeviceToHost, s));
    PM_HIP(hipMemcpyAsync(order_h.data(), order, sizeof(uint32_t) * (size_t)n, hipMemcpyDeviceToHost, s));
    PM_HIP(hipStreamSynchronize(s));
    if (st.bad) return set_error("GPU BVH build: inconsistent tree"), PM_ERR_STATE;
    b->n_tri = n_tri;
    b->n_refs = n_tri;
    b->n_nodes = n_nodes;
    b->n_leaves = (int64_t)st.leaves;
    b->depth = (int32_t)st.depth;
    b->max_leaf = max_leaf;
    b->sah_cost = st.sah;
    b->pos_of.assign((size_t)n, 0);
    for (int k = 0; k < n; ++k) b->pos_of[order_h[(size_t)k]] = k;
    b->build_ms = std::chrono::duration<double, std::milli>(std::chrono::steady_clock::now() - t0).count();
    return PM_OK;
}

}  // namespace pm
