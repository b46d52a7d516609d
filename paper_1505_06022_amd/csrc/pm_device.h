// Device building blocks of the photon-mapping hot path (gfx950 / CDNA4).
//
// Floating-point rules (the same rules the method is specified with):
// float32 geometry, no contraction of a*b+c into FMA (explicit fmaf only in
// the conservative box test), correctly rounded division and square root,
// fixed evaluation order for dot/cross/normalize, no transcendental calls.
#pragma once
#include <hip/hip_runtime.h>
#include <stdint.h>

#pragma clang fp contract(off)

namespace pmd {

// ---------------------------------------------------------------------------
// Random numbers (Sec. 3.2): four multiplicative LCGs s <- a*s mod m, each
// evaluated with Schrage's decomposition (q = m div a, r = m mod a) exactly
// as the paper's float code does, but in 32-bit integers; output is the
// fractional part of s0/m0 - s1/m1 + s2/m2 - s3/m3 of the advanced state.
// ---------------------------------------------------------------------------
struct Rng {
    int32_t s0, s1, s2, s3;
};

enum : uint32_t { kKindEye = 1u, kKindPhoton = 2u };

__device__ __forceinline__ int32_t lcg_step(int32_t s, int32_t a, int32_t q, int32_t r, int32_t m) {
    int32_t hi = s / q;
    int32_t lo = s - hi * q;
    int32_t t = a * lo - r * hi;
    return t < 0 ? t + m : t;
}

// s / m rounded to nearest float, for a state 0 < s < m of one of the four
// generators: the product with the rounded reciprocal, corrected once by its
// exact fma residual (Markstein's division, IBM J. Res. Dev. 1990). For these
// four moduli it equals the IEEE quotient for every state (checked
// exhaustively on the host), in 3 instructions instead of the ~10 of a full
// division.
__device__ __forceinline__ float div_by_modulus(int32_t s, float m, float inv_m) {
    float x = (float)s;
    float q0 = x * inv_m;
    float r = __builtin_fmaf(-q0, m, x);
    return __builtin_fmaf(r, inv_m, q0);
}

__device__ __forceinline__ float rng_next(Rng &g) {
    g.s0 = lcg_step(g.s0, 3423, 1225, 1112, 4194287);
    g.s1 = lcg_step(g.s1, 2646, 1585, 367, 4194277);
    g.s2 = lcg_step(g.s2, 1707, 2457, 92, 4194191);
    g.s3 = lcg_step(g.s3, 1999, 2098, 265, 4194167);
    float f0 = div_by_modulus(g.s0, 4194287.0f, 1.0f / 4194287.0f);
    float f1 = div_by_modulus(g.s1, 4194277.0f, 1.0f / 4194277.0f);
    float f2 = div_by_modulus(g.s2, 4194191.0f, 1.0f / 4194191.0f);
    float f3 = div_by_modulus(g.s3, 4194167.0f, 1.0f / 4194167.0f);
    float x = ((f0 - f1) + f2) - f3;
    float u = x - floorf(x);
    return u >= 1.0f ? 0x1.fffffep-1f : u;
}

// splitmix64 (Steele, Lea, Flood 2014)
__device__ __forceinline__ uint64_t splitmix64(uint64_t &st) {
    uint64_t z = (st += 0x9E3779B97F4A7C15ull);
    z = (z ^ (z >> 30)) * 0xBF58476D1CE4E5B9ull;
    z = (z ^ (z >> 27)) * 0x94D049BB133111EBull;
    return z ^ (z >> 31);
}

// Per-stream state from a counter key: splitmix64 mixes (seed, kind,
// iteration, index) into a Marsaglia xorshift128 seed (the generator the
// paper seeds its per-thread states with), whose outputs 9..12 are reduced
// into [1, m_j - 1].
__device__ __forceinline__ Rng rng_seed(uint64_t seed, uint32_t kind, uint32_t k, uint64_t index) {
    uint64_t st = seed;
    uint64_t h = splitmix64(st);
    st = h ^ (((uint64_t)kind << 32) | (uint64_t)k);
    h = splitmix64(st);
    st = h ^ index;
    uint64_t w01 = splitmix64(st);
    uint64_t w23 = splitmix64(st);
    uint32_t x = (uint32_t)w01, y = (uint32_t)(w01 >> 32), z = (uint32_t)w23, w = (uint32_t)(w23 >> 32);
    if ((x | y | z | w) == 0u) x = 1u;
    uint32_t o[4];
#pragma unroll
    for (int i = 0; i < 12; ++i) {
        uint32_t t = x ^ (x << 11);
        x = y;
        y = z;
        z = w;
        w = (w ^ (w >> 19)) ^ (t ^ (t >> 8));
        if (i >= 8) o[i - 8] = w;
    }
    Rng g;
    g.s0 = (int32_t)(1u + o[0] % 4194286u);
    g.s1 = (int32_t)(1u + o[1] % 4194276u);
    g.s2 = (int32_t)(1u + o[2] % 4194190u);
    g.s3 = (int32_t)(1u + o[3] % 4194166u);
    return g;
}

// ---------------------------------------------------------------------------
// float3 arithmetic with a fixed evaluation order
// ---------------------------------------------------------------------------
struct V3 {
    float x, y, z;
};
__device__ __forceinline__ V3 v3(float x, float y, float z) { return V3{x, y, z}; }
__device__ __forceinline__ V3 vsub(V3 a, V3 b) { return v3(a.x - b.x, a.y - b.y, a.z - b.z); }
__device__ __forceinline__ float vdot(V3 a, V3 b) { return (a.x * b.x + a.y * b.y) + a.z * b.z; }
__device__ __forceinline__ V3 vcross(V3 a, V3 b) {
    return v3(a.y * b.z - a.z * b.y, a.z * b.x - a.x * b.z, a.x * b.y - a.y * b.x);
}
__device__ __forceinline__ V3 vnorm(V3 v) {
    float l = sqrtf(vdot(v, v));
    return v3(v.x / l, v.y / l, v.z / l);
}
__device__ __forceinline__ V3 vneg(V3 a) { return v3(-a.x, -a.y, -a.z); }
__device__ __forceinline__ V3 vray(V3 o, float t, V3 d) { return v3(o.x + t * d.x, o.y + t * d.y, o.z + t * d.z); }

// ---------------------------------------------------------------------------
// Scene layout on the device
// ---------------------------------------------------------------------------
struct Tri {
    V3 v0, v1, v2;
    int32_t id;
    uint32_t mat;
};

// 48-byte triangle record: v0.xyz v1.x | v1.yz v2.xy | v2.z id mat 0
__device__ __forceinline__ Tri load_tri(const float4 *__restrict__ tris, uint32_t k) {
    const float4 *p = tris + 3 * (size_t)k;
    float4 a = p[0], b = p[1], c = p[2];
    Tri t;
    t.v0 = v3(a.x, a.y, a.z);
    t.v1 = v3(a.w, b.x, b.y);
    t.v2 = v3(b.z, b.w, c.x);
    t.id = __float_as_int(c.y);
    t.mat = __float_as_uint(c.z);
    return t;
}

// Edge vectors v1 - v0 and v2 - v0 (for the normal and for points on the
// triangle), rounded once per component.
__device__ __forceinline__ V3 tri_e1(const Tri &t) { return vsub(t.v1, t.v0); }
__device__ __forceinline__ V3 tri_e2(const Tri &t) { return vsub(t.v2, t.v0); }
__device__ __forceinline__ V3 tri_normal(const Tri &t) { return vnorm(vcross(tri_e1(t), tri_e2(t))); }

// Per-ray constants of the watertight triangle test: kz = the major axis of d
// (ties x, y, z, as for the link set), kx = kz + 1 and ky = kz + 2 (mod 3),
// and the shear that maps d onto the kz axis: sx = d_kx / d_kz,
// sy = d_ky / d_kz, sz = 1 / d_kz.
struct Shear {
    float sx, sy, sz;
    uint32_t kz;
};

__device__ __forceinline__ Shear ray_shear(V3 d) {
    const float ax = fabsf(d.x), ay = fabsf(d.y), az = fabsf(d.z);
    Shear h;
    h.kz = (ax >= ay && ax >= az) ? 0u : (ay >= az ? 1u : 2u);
    const float dz = h.kz == 0u ? d.x : (h.kz == 1u ? d.y : d.z);
    const float dx = h.kz == 0u ? d.y : (h.kz == 1u ? d.z : d.x);
    const float dy = h.kz == 0u ? d.z : (h.kz == 1u ? d.x : d.y);
    h.sx = dx / dz;
    h.sy = dy / dz;
    h.sz = 1.0f / dz;
    return h;
}

// a b - c d with a relative error of at most 2u (u = 2^-24; Kahan's 2x2
// determinant with one fused multiply-add for the rounding error of c d), so
// its sign is the exact value's sign.
__device__ __forceinline__ float det2(float a, float b, float c, float d) {
    const float w = c * d;
    const float e = fmaf(-c, d, w);
    const float f = fmaf(a, b, -w);
    return f + e;
}

// Vertex v seen from the ray: (x, y) its position in the plane sheared along
// d (the ray passes through (0, 0)) and z its distance along the kz axis.
__device__ __forceinline__ void shear_vertex(V3 v, V3 o, const Shear &h, float &x, float &y, float &z) {
    const V3 a = vsub(v, o);
    const float az = h.kz == 0u ? a.x : (h.kz == 1u ? a.y : a.z);
    const float ax = h.kz == 0u ? a.y : (h.kz == 1u ? a.z : a.x);
    const float ay = h.kz == 0u ? a.z : (h.kz == 1u ? a.x : a.y);
    x = fmaf(-h.sx, az, ax);
    y = fmaf(-h.sy, az, ay);
    z = az;
}

// Watertight ray/triangle test (two-sided; Woop, Benthin and Wald 2013, with
// the edge functions taken by det2).  The edge functions U, V, W are the
// doubled signed areas that the ray's point spans with each edge of the
// sheared triangle; their signs are exact for the sheared vertices, so the
// ray hits when all three agree, and an edge shared by two triangles has
// the same vertices and the opposite sign in both (no ray slips between
// them).  t = (U z0 + V z1 + W z2) / (U + V + W) (z scaled by sz), the
// depth of the point with those barycentric weights.
//
// Error bound (used by the traversal's box test): the point o + t d lies
// within 22u (t |d_a| + L) of a point of the triangle along every axis a
// (L its longest edge): the weights are the exact non-negative barycentric
// coordinates of the ray in the sheared, rounded vertices (relative error of
// U, V, W at most 2u), each sheared coordinate is within 3u (|t d_a| + L) of
// the exact one, and t within 16u (|t| + L / |d_kz|).
__device__ __forceinline__ bool wt_hit(V3 o, const Shear &h, const Tri &tr, float &t_out) {
    float ax, ay, az, bx, by, bz, cx, cy, cz;
    shear_vertex(tr.v0, o, h, ax, ay, az);
    shear_vertex(tr.v1, o, h, bx, by, bz);
    shear_vertex(tr.v2, o, h, cx, cy, cz);
    const float U = det2(cx, by, cy, bx);
    const float V = det2(ax, cy, ay, cx);
    const float W = det2(bx, ay, by, ax);
    if ((U < 0.0f || V < 0.0f || W < 0.0f) && (U > 0.0f || V > 0.0f || W > 0.0f)) return false;
    const float det = (U + V) + W;
    if (det == 0.0f) return false;
    const float T = fmaf(W, h.sz * cz, fmaf(V, h.sz * bz, U * (h.sz * az)));
    t_out = T / det;
    return true;
}

// Closest-hit acceptance: inside (tmin, tbest), ties in t to the lower index.
__device__ __forceinline__ bool accept_hit(float t, int32_t id, float tmin, float tbest, int32_t best) {
    if (!(t > tmin)) return false;
    if (t < tbest) return true;
    return t == tbest && best >= 0 && id < best;
}

// Link set of a ray: the principal direction = major axis of d (ties x, y,
// z), signed by that component (the cube-map lookup of Fig. "mtbvh").
__device__ __forceinline__ int link_set(V3 d) {
    float ax = fabsf(d.x), ay = fabsf(d.y), az = fabsf(d.z);
    if (ax >= ay && ax >= az) return d.x < 0.0f ? 1 : 0;
    if (ay >= az) return d.y < 0.0f ? 3 : 2;
    return d.z < 0.0f ? 5 : 4;
}

struct Bvh {
    const uint4 *nodes;   // [6][n_nodes] 16-byte nodes, then a pad node
    const float4 *tris;   // [n_tri][3] float4
    uint32_t n_nodes;
    float qlo[3], qstep[3];  // node box grid: coordinate = qlo + q * qstep
};

struct TraceStats {
    uint32_t boxes, tris;
};

// Stackless closest-hit traversal of one link set (Sec. 3.1, Fig. "mtbvh"):
// follow the hit link (next node) when the ray meets the node's box, else the
// miss (skip) link; at a leaf test its triangles and continue with the miss
// link.  The box test is conservative (padded boxes, a relative slack on the
// exit distance; the bound is at box_hit) so the result equals the
// brute-force closest hit.  Walker holds one lane's traversal state so that a persistent kernel
// can interleave node steps of different rays.  kPairTris: a leaf's triangle
// records are requested two at a time (more registers; it pays where leaves
// are full and the kernel's occupancy is already register-bound).
template <bool kPairTris>
struct WalkerT {
    const uint4 *nodes;
    uint32_t n, i;
    V3 o, d;
    Shear sh;                      // the triangle test's shear
    float sx, sy, sz, bx, by, bz;  // slab planes: t = q * s + b per axis
    uint32_t rx, ry, rz;           // 16 where the axis is walked backwards (near plane = hi), else 0
    float tmin, tbest;
    int32_t best, exclude;
    uint32_t best_k;

    __device__ __forceinline__ void init(const Bvh &bvh, int set, V3 o_, V3 d_, float tmin_, float tmax_,
                                         int32_t exclude_) {
        nodes = bvh.nodes + (size_t)set * bvh.n_nodes;
        n = bvh.n_nodes;
        i = 0;
        o = o_;
        d = d_;
        sh = ray_shear(d_);
        // reciprocal direction; zero components replaced by a tiny signed value
        float dx = fabsf(d.x) > 1e-30f ? d.x : copysignf(1e-30f, d.x);
        float dy = fabsf(d.y) > 1e-30f ? d.y : copysignf(1e-30f, d.y);
        float dz = fabsf(d.z) > 1e-30f ? d.z : copysignf(1e-30f, d.z);
        float ix = 1.0f / dx, iy = 1.0f / dy, iz = 1.0f / dz;
        sx = bvh.qstep[0] * ix;
        sy = bvh.qstep[1] * iy;
        sz = bvh.qstep[2] * iz;
        bx = (bvh.qlo[0] - o.x) * ix;
        by = (bvh.qlo[1] - o.y) * iy;
        bz = (bvh.qlo[2] - o.z) * iz;
        rx = sx < 0.0f ? 16u : 0u;
        ry = sy < 0.0f ? 16u : 0u;
        rz = sz < 0.0f ? 16u : 0u;
        tmin = tmin_;
        tbest = tmax_;
        best = -1;
        best_k = 0;
        exclude = exclude_;
    }

    __device__ __forceinline__ bool done() const { return i >= n; }

    // One node visit (and, at a leaf, its triangles).  Requires !done().
    // Next node: i + 1 after an inner-node hit or any leaf, else the skip link.
    template <bool kStats>
    __device__ __forceinline__ void step(const float4 *__restrict__ tris, TraceStats &st) {
        visit<kStats>(nodes[i], tris, st);
    }

    // The visit of node i once its record q has been loaded.
    template <bool kStats>
    __device__ __forceinline__ void visit(const uint4 &q, const float4 *__restrict__ tris, TraceStats &st) {
        const bool leaf = (q.w >> 31) != 0u;
        const bool hit = box_hit(q);
        if (kStats) st.boxes++;
        if (hit && leaf) leaf_tris<kStats>(tris, q.w, st);
        i = (hit || leaf) ? i + 1 : q.w;
    }

    // Slab test of a quantised node box against [tmin, tbest].  Each word
    // holds one axis as lo | hi << 16; rotating it by 16 where the ray runs
    // towards -axis puts that axis's entry plane in the low half, so the
    // entry and exit distances need no min/max per axis (the values equal
    // min/max of the two plane distances).
    //
    // Conservative: a plane distance fma(q, s, b), with s and b rounded once
    // each, is within 4u |t| + 2u ext / |d_a| of the exact one (u = 2^-24,
    // ext the scene extent, for any ray origin).  An accepted triangle hit at
    // t puts o + t d within 22u (|t d_a| + L) of a point of the triangle along
    // each axis (see wt_hit), so inside the triangle's box grown by that
    // much.  The absolute parts (2u ext, 22u L) are covered many times over by
    // the padding of every box (at least 2^-15 ext), and the relative parts,
    // at most 52u |t| in all, by the slack kBoxSlack = 256u on the exit
    // distance: every box that holds a triangle with an accepted hit at a t
    // in (tmin, tbest] passes, so the walk finds the brute-force closest hit.
    static constexpr float kBoxSlack = 0x1p-16f;
    __device__ __forceinline__ bool box_hit(const uint4 &q) const {
        const uint32_t ax = __builtin_rotateright32(q.x, rx), ay = __builtin_rotateright32(q.y, ry),
                       az = __builtin_rotateright32(q.z, rz);
        const float nx = fmaf((float)(ax & 0xffffu), sx, bx), fx = fmaf((float)(ax >> 16), sx, bx);
        const float ny = fmaf((float)(ay & 0xffffu), sy, by), fy = fmaf((float)(ay >> 16), sy, by);
        const float nz = fmaf((float)(az & 0xffffu), sz, bz), fz = fmaf((float)(az >> 16), sz, bz);
        const float tn = fmaxf(fmaxf(nx, ny), fmaxf(nz, tmin));
        const float tf = fminf(fminf(fx, fy), fminf(fz, tbest));
        return tn <= fmaf(fabsf(tf), kBoxSlack, tf);
    }

    template <bool kStats>
    __device__ __forceinline__ void leaf_tris(const float4 *__restrict__ tris, uint32_t w, TraceStats &st) {
        uint32_t first = (w >> 3) & 0x0fffffffu, cnt = w & 7u;
        // the excluded triangle is checked after the test, so that a record's
        // words arrive in one round trip (a branch on the index first would
        // wait for it before loading the vertices)
        if constexpr (kPairTris) {
            for (uint32_t k = 0; k < cnt; k += 2) {
                const bool two = k + 1 < cnt;
                const Tri ta = load_tri(tris, first + k);
                const Tri tb = load_tri(tris, first + k + (two ? 1u : 0u));
                if (kStats) st.tris += two ? 2u : 1u;
                tri_test(ta, first + k);
                if (two) tri_test(tb, first + k + 1);
            }
        } else {
            for (uint32_t k = 0; k < cnt; ++k) {
                const Tri tr = load_tri(tris, first + k);
                if (kStats) st.tris++;
                tri_test(tr, first + k);
            }
        }
    }

    // Triangle record rec against the ray: the closest hit so far, ties in t
    // to the lower original index, the excluded triangle skipped.
    __device__ __forceinline__ void tri_test(const Tri &tr, uint32_t rec) {
        float t;
        if (wt_hit(o, sh, tr, t) && tr.id != exclude && accept_hit(t, tr.id, tmin, tbest, best)) {
            tbest = t;
            best = tr.id;
            best_k = rec;
        }
    }

    // Up to two node visits per memory round trip: nodes i and i + 1 are
    // loaded together; when the walk continues at i + 1 (an inner-node hit or
    // any leaf) that node is tested without waiting for another load.
    template <bool kStats>
    __device__ __forceinline__ void step2(const float4 *__restrict__ tris, TraceStats &st) {
        uint4 q0 = nodes[i];
        uint4 q1 = nodes[i + 1 < n ? i + 1 : i];
        if (kStats) st.boxes++;
        bool leaf = (q0.w >> 31) != 0u, hit = box_hit(q0);
        if (hit && leaf) leaf_tris<kStats>(tris, q0.w, st);
        if (!(hit || leaf)) {
            i = q0.w;
            return;
        }
        i = i + 1;
        if (i >= n) return;
        if (kStats) st.boxes++;
        leaf = (q1.w >> 31) != 0u;
        hit = box_hit(q1);
        if (hit && leaf) leaf_tris<kStats>(tris, q1.w, st);
        i = (hit || leaf) ? i + 1 : q1.w;
    }

    // The whole walk with postponed leaf tests.  The wave visits boxes until
    // at most `late` of its lanes are still looking for a leaf hit (and at
    // least one lane holds one); then every lane that holds a leaf tests its
    // triangles, all lanes together.  A lane that holds a leaf keeps visiting
    // boxes while others search and halts in front of its next leaf hit, which
    // it visits again after the tests.  The wave votes once per
    // kPostponedSteps box visits (fewer ballots and branches per visit; an
    // idle lane just waits a few steps longer).  Each round of visits advances
    // every searching lane, so the walk ends.  The closest hit under the
    // lower-index tie rule does not depend on the order of the visits: the
    // result is the one of step().
#ifndef PM_POSTPONED_STEPS
#define PM_POSTPONED_STEPS 8
#endif
    static constexpr int kPostponedSteps = PM_POSTPONED_STEPS;

    template <bool kStats>
    __device__ __forceinline__ void walk_postponed(const float4 *__restrict__ tris, uint32_t late, TraceStats &st) {
        uint32_t held = 0u;  // link word of a leaf hit not yet tested, or 0
        bool halted = false;
        for (;;) {
            for (;;) {
                const uint64_t searching = __ballot(i < n && held == 0u);
                if (searching == 0ull) break;
                if ((uint32_t)__popcll(searching) <= late && __ballot(held != 0u) != 0ull) break;
#pragma unroll
                for (int u = 0; u < kPostponedSteps; ++u) {
                    if (i < n && !halted) {
                        const uint4 q = nodes[i];
                        if (kStats) st.boxes++;
                        const bool leaf = (q.w >> 31) != 0u, hit = box_hit(q);
                        const bool leaf_hit = hit && leaf;
                        halted = leaf_hit && held != 0u;
                        held = (leaf_hit && held == 0u) ? q.w : held;
                        i = halted ? i : ((hit || leaf) ? i + 1 : q.w);
                    }
                }
            }
            if (__ballot(held != 0u) == 0ull) break;  // no lane searching and none holding: all done
            if (held != 0u) leaf_tris<kStats>(tris, held, st);
            held = 0u;
            halted = false;
        }
    }

    __device__ __forceinline__ float t_hit() const { return best >= 0 ? tbest : __builtin_inff(); }
};
using Walker = WalkerT<false>;

// Packet walk, for a wave whose lanes all walk one link set (nodes = that
// set's node array, the same on every lane): the wave follows one node index,
// taking the hit link when any lane's box test passes and the skip link
// otherwise; at a leaf each lane whose own box test passes tests the
// triangles.  The nodes a lane meets are a superset of those of its own walk
// and its box tests use its own t_best, so its closest hit is unchanged.  The
// node index, the link words and so every branch are uniform across the wave,
// and all lanes read the same node and triangle records.
template <bool kStats>
__device__ __forceinline__ uint32_t packet_visit(Walker &w, const uint4 &q, uint32_t i,
                                                 const float4 *__restrict__ tris, TraceStats &st) {
    const uint32_t link = (uint32_t)__builtin_amdgcn_readfirstlane((int)q.w);
    const bool hit = w.box_hit(q);
    if (kStats) st.boxes++;
    if ((link >> 31) != 0u) {
        if (hit) w.leaf_tris<kStats>(tris, link, st);
        return i + 1;
    }
    return __ballot(hit) != 0ull ? i + 1 : link;
}

// Nodes a packet walk requests at once (measured: 2 beats 1, 3, 4 and 5).
constexpr int kPacketRun = 2;

template <bool kStats>
__device__ __forceinline__ void walk_packet(Walker &w, const uint4 *__restrict__ nodes, uint32_t n,
                                            const float4 *__restrict__ tris, TraceStats &st) {
    constexpr int kRun = kPacketRun;
    uint32_t i = 0;
    while (i < n) {
        // nodes i .. i + kRun - 1 come in one request: each is the next node
        // after a hit or a leaf, which then costs no further round trip
        const uint4 *p = nodes + i;  // in bounds: the node arrays end with kRun - 1 pad nodes
        uint4 q[kRun];
#pragma unroll
        for (int k = 0; k < kRun; ++k) q[k] = p[k];
        uint32_t cur = packet_visit<kStats>(w, q[0], i, tris, st);
#pragma unroll
        for (int k = 1; k < kRun; ++k)
            if (cur == i + (uint32_t)k && cur < n) cur = packet_visit<kStats>(w, q[k], cur, tris, st);
        i = cur;
    }
    w.i = n;
}

// Two rays per lane walked in lockstep: both node records are requested
// before either box is tested, so each lane keeps two loads in flight.  A
// walker that has finished re-reads node 0 of its link set (an in-bounds,
// cached address) and is left unchanged until the other one finishes.
template <bool kStats>
__device__ __forceinline__ void walk_two(Walker &a, Walker &b, const float4 *__restrict__ tris, TraceStats &sa,
                                         TraceStats &sb) {
    for (;;) {
        const bool da = a.done(), db = b.done();
        if (da && db) break;
        const uint4 qa = a.nodes[da ? 0u : a.i];
        const uint4 qb = b.nodes[db ? 0u : b.i];
        if (!da) a.visit<kStats>(qa, tris, sa);
        if (!db) b.visit<kStats>(qb, tris, sb);
    }
}

// Returns the original index of the closest triangle (-1: none); t_out gets
// its distance (+inf on a miss) and k_out its position in the triangle array.
// paired: the walk requests nodes i and i + 1 together (step2); kPairTris:
// a leaf's triangle records two at a time.
template <bool kStats, bool kPairTris = false>
__device__ __forceinline__ int32_t closest_hit(const Bvh &bvh, int set, V3 o, V3 d, float tmin, float tmax,
                                               int32_t exclude, float &t_out, uint32_t &k_out, TraceStats &st,
                                               bool paired = false) {
    WalkerT<kPairTris> w;
    w.init(bvh, set, o, d, tmin, tmax, exclude);
    if (paired) {
        while (!w.done()) w.template step2<kStats>(bvh.tris, st);
    } else {
        while (!w.done()) w.template step<kStats>(bvh.tris, st);
    }
    t_out = w.t_hit();
    k_out = w.best_k;
    return w.best;
}

// Wave-aggregated counter increment for the lanes in `mask` (uniform across
// the wave): returns base + rank of this lane within mask.
__device__ __forceinline__ uint32_t wave_fetch_add(uint32_t *counter, uint64_t mask, bool member) {
    uint32_t rank = __builtin_amdgcn_mbcnt_hi((uint32_t)(mask >> 32), __builtin_amdgcn_mbcnt_lo((uint32_t)mask, 0u));
    int leader = __ffsll((unsigned long long)mask) - 1;
    uint32_t base = 0;
    if (member && rank == 0) base = atomicAdd(counter, (uint32_t)__popcll(mask));
    base = __shfl(base, leader);
    return base + rank;
}

// ---------------------------------------------------------------------------
// Sampling (only + - * / sqrt; the same rules as the method's definition)
// ---------------------------------------------------------------------------
// Orthonormal basis about unit n (Duff et al. 2017).
__device__ __forceinline__ void onb(V3 n, V3 &b1, V3 &b2) {
    float sign = copysignf(1.0f, n.z);
    float a = -1.0f / (sign + n.z);
    float b = n.x * n.y * a;
    b1 = v3(1.0f + sign * n.x * n.x * a, sign * b, -sign * n.x);
    b2 = v3(b, sign + n.y * n.y * a, -n.y);
}

// Cosine-weighted direction about unit n: disk point by rejection from the
// square (at most 64 tries), lifted to the hemisphere (Malley's method).
__device__ __forceinline__ V3 cosine_dir(V3 n, Rng &g) {
    float a = 0.0f, b = 0.0f, r2 = 0.0f;
    bool ok = false;
    for (int tries = 0; tries < 64; ++tries) {
        a = 2.0f * rng_next(g) - 1.0f;
        b = 2.0f * rng_next(g) - 1.0f;
        r2 = a * a + b * b;
        if (r2 < 1.0f) {
            ok = true;
            break;
        }
    }
    if (!ok) {
        a = 0.0f;
        b = 0.0f;
        r2 = 0.0f;
    }
    float z = sqrtf(1.0f - r2);
    V3 t1, t2;
    onb(n, t1, t2);
    V3 w = v3((a * t1.x + b * t2.x) + z * n.x, (a * t1.y + b * t2.y) + z * n.y, (a * t1.z + b * t2.z) + z * n.z);
    return vnorm(w);
}

__device__ __forceinline__ V3 reflect(V3 d, V3 n) {
    float c = 2.0f * vdot(d, n);
    return v3(d.x - c * n.x, d.y - c * n.y, d.z - c * n.z);
}

// Smooth dielectric: unpolarised Fresnel reflectance picks reflection or
// refraction with one draw (also drawn under total internal reflection).
__device__ __forceinline__ V3 glass_dir(V3 d, V3 n, float ior, Rng &g) {
    float cosi = -vdot(d, n);
    float eta, ci;
    V3 nn;
    if (cosi > 0.0f) {
        eta = 1.0f / ior;
        nn = n;
        ci = cosi;
    } else {
        eta = ior;
        nn = vneg(n);
        ci = -cosi;
    }
    float sin2t = (eta * eta) * (1.0f - ci * ci);
    float k = 1.0f - sin2t;
    float F = 1.0f, ct = 0.0f;
    if (k >= 0.0f) {
        ct = sqrtf(k);
        float rs = (eta * ci - ct) / (eta * ci + ct);
        float rp = (ci - eta * ct) / (ci + eta * ct);
        F = 0.5f * (rs * rs + rp * rp);
    }
    float u = rng_next(g);
    if (u < F) return reflect(d, n);
    float c = eta * ci - ct;
    return vnorm(v3(eta * d.x + c * nn.x, eta * d.y + c * nn.y, eta * d.z + c * nn.z));
}

constexpr float kInvPiF = 0.318309886183790671538f;
constexpr double kPiD = 3.14159265358979323846;

// XCD-aware block order: hardware hands consecutive workgroups to the 8 XCDs
// round robin; remap so each XCD (and its L2) owns a contiguous range.
__device__ __forceinline__ uint32_t xcd_block(uint32_t bid, uint32_t nblk) {
    uint32_t per = nblk >> 3, rem = nblk & 7u;
    uint32_t x = bid & 7u, k = bid >> 3;
    return x * per + (x < rem ? x : rem) + k;
}

}  // namespace pmd
