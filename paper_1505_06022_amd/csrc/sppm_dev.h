// Device side of one SPPM iteration (Sec. 2), written per element so that the
// single-scene kernels and the batched persistent kernels share it.
#pragma once
#include "pm.h"
#include "pm_device.h"

namespace pmd {

constexpr int kBlock = 256;
constexpr int kScanItems = 16;                  // per thread
constexpr int kScanTile = kBlock * kScanItems;  // buckets per scan tile
constexpr int kMaxAdjMat = 256;
// markers of the adjoint's per-path material table (entries are uint16)
constexpr uint16_t kMatNone = 0xffffu;  // no photon stored at this bounce
constexpr uint16_t kMatEnd = 0xfffeu;   // the path ended before this bounce

struct SceneDev {
    Bvh bvh;
    const int32_t *mat_type;
    const float *mat_rho, *mat_q, *mat_Le, *mat_ior;
    const uint32_t *emit_pos;  // triangle-array position of each emitter (original order)
    const double *emit_cdf;
    int32_t n_emit;
    double power;
    float eps;
    float lo[3];
    float ext;  // largest extent of the scene box
    V3 cpos, cf, cr, cu;
    float tanh_fov, aspect;
    int32_t W, H;
};

// One scene's parameters and device buffers.  Bucket arrays may be shared by
// several scenes: this scene owns buckets [table_off, table_off + mask + 1).
struct SppmDev {
    SceneDev sc;
    uint64_t seed;
    int32_t max_depth, max_bounces;
    uint32_t n_paths, cap;
    float phi0;
    double alpha, scale, inv_scale;
    int64_t P;
    uint32_t mask, table_off;
    int32_t photon_kernel;    // PM_PHOTON_* (resolved: per path or regenerating)
    uint32_t refill;          // regeneration: idle lanes that trigger a refill
    int32_t force_set;        // -1: link set by ray direction; 0..5: that set for every ray
    int32_t paired_walk;      // 1: walks request nodes i and i + 1 together (single-scene handles)
    int32_t gather_mode;      // PM_GATHER_EXACT or PM_GATHER_STOCHASTIC
    unsigned long long *sh_key;  // stochastic hashing: smallest (depth, photon id) per entry
    uint32_t *sh_surv;           // stochastic hashing: store index of each entry's survivor
    float4 *hp_pos, *hp_nrm;  // (x, W*rho/pi), (n toward the eye, material bits | -1)
    double *N, *R2, *tau, *D;
    float4 *store;            // [cap][2]: (x, phi), (w, path << 5 | bounce)
    uint2 *key_rank;          // [cap] exact gather: each stored photon's bucket and its rank in the bucket
    uint32_t *counters;       // [0] photons stored, [1] sticky flags (1: store overflow, 2: flux overflow), [2] next path
    unsigned long long *r2max;
    uint32_t *M;
    unsigned long long *Phi;
    unsigned long long *stats;  // [kStatCount] profiling counts (PM_PROFILE_COUNT), else unused
};

// Profiling counts (accumulated by the kStats variants of the kernels).
enum {
    kStatEyePaths = 0, kStatEyeRays, kStatEyeBoxes, kStatEyeTris,
    kStatPhotonPaths, kStatPhotonRays, kStatPhotonBoxes, kStatPhotonTris,
    kStatGatherHits, kStatGatherBuckets, kStatGatherExamined, kStatGatherAccepted,
    kStatPhotonStored,
    kStatCount = 16
};

// Per-lane counts of a traced path (or of all paths a persistent lane traced).
struct LaneStats {
    uint64_t paths = 0, rays = 0, boxes = 0, tris = 0, stored = 0;
};

// Adds v summed over the wavefront to *dst; every lane of the wave must call it.
__device__ __forceinline__ void wave_stat_add(unsigned long long *dst, uint64_t v) {
    for (int off = 32; off > 0; off >>= 1) v += __shfl_xor(v, off);
    if ((threadIdx.x & 63) == 0 && v) atomicAdd(dst, (unsigned long long)v);
}

__device__ __forceinline__ void wave_stats_flush(unsigned long long *dst, const LaneStats &ls) {
    wave_stat_add(dst + 0, ls.paths);
    wave_stat_add(dst + 1, ls.rays);
    wave_stat_add(dst + 2, ls.boxes);
    wave_stat_add(dst + 3, ls.tris);
}

// Link set of a ray: by its direction (MTBVH), or one set for every ray.
__device__ __forceinline__ int ray_set(const SppmDev &d, V3 dir) {
    return d.force_set >= 0 ? d.force_set : link_set(dir);
}

// ---------------------------------------------------------------------------
// Eye pass: a jittered pinhole ray followed through mirror and glass to the
// first diffuse (rho > 0) surface, which becomes the pixel's hit point;
// directly seen emission is accumulated into D (skipped when replaying).
// ---------------------------------------------------------------------------
template <bool kStats = false>
__device__ __forceinline__ void eye_elem(const SppmDev &d, uint32_t k, int64_t p, bool accumulate_D,
                                        LaneStats *ls = nullptr) {
    const SceneDev &sc = d.sc;
    int32_t px = (int32_t)(p % sc.W), py = (int32_t)(p / sc.W);
    Rng g = rng_seed(d.seed, kKindEye, k, (uint64_t)p);
    float j0 = rng_next(g), j1 = rng_next(g);
    float fx = ((float)px + j0) / (float)sc.W;
    float fy = ((float)py + j1) / (float)sc.H;
    float sx = (2.0f * fx - 1.0f) * (sc.tanh_fov * sc.aspect);
    float sy = (1.0f - 2.0f * fy) * sc.tanh_fov;
    V3 dir = vnorm(v3((sc.cf.x + sx * sc.cr.x) + sy * sc.cu.x, (sc.cf.y + sx * sc.cr.y) + sy * sc.cu.y,
                      (sc.cf.z + sx * sc.cr.z) + sy * sc.cu.z));
    V3 org = sc.cpos;
    float tmin = 0.0f, thr = 1.0f;
    int32_t excl = -1;
    double dadd = 0.0;
    float4 pos = make_float4(0.0f, 0.0f, 0.0f, 0.0f);
    float4 nrm = make_float4(0.0f, 0.0f, 0.0f, __int_as_float(-1));
    TraceStats st{0u, 0u};
    for (int depth = 0; depth < d.max_depth; ++depth) {
        float t;
        uint32_t kp;
        int32_t h = closest_hit<kStats>(sc.bvh, ray_set(d, dir), org, dir, tmin, __builtin_inff(), excl, t, kp, st,
                                        d.paired_walk != 0);
        if (kStats) ls->rays++;
        if (h < 0) break;
        V3 x = vray(org, t, dir);
        Tri tr = load_tri(sc.bvh.tris, kp);
        V3 n = tri_normal(tr);
        uint32_t m = tr.mat;
        bool front = vdot(dir, n) < 0.0f;
        float Le = sc.mat_Le[m];
        if (Le > 0.0f && front) dadd += (double)(thr * Le);
        int type = sc.mat_type[m];
        if (type == PM_MAT_DIFFUSE) {
            float rho = sc.mat_rho[m];
            if (rho > 0.0f) {
                V3 nh = front ? n : vneg(n);
                pos = make_float4(x.x, x.y, x.z, (thr * rho) * kInvPiF);
                nrm = make_float4(nh.x, nh.y, nh.z, __uint_as_float(m));
            }
            break;
        } else if (type == PM_MAT_MIRROR) {
            dir = reflect(dir, n);
        } else {
            dir = glass_dir(dir, n, sc.mat_ior[m], g);
        }
        org = x;
        tmin = sc.eps;
        excl = h;
    }
    d.hp_pos[p] = pos;
    d.hp_nrm[p] = nrm;
    if (accumulate_D) d.D[p] += dadd;
    if (kStats) {
        ls->paths++;
        ls->boxes += st.boxes;
        ls->tris += st.tris;
    }
}

// Wave-aggregated append: one atomic per wavefront for all lanes currently
// active at this call site (they must share `counter`).  Returns the slot.
__device__ __forceinline__ uint32_t wave_append(uint32_t *counter) {
    uint64_t mask = __ballot(1);
    uint32_t lane_rank = __builtin_amdgcn_mbcnt_hi((uint32_t)(mask >> 32), __builtin_amdgcn_mbcnt_lo((uint32_t)mask, 0u));
    int leader = __ffsll((unsigned long long)mask) - 1;
    uint32_t base = 0;
    if (lane_rank == 0) base = atomicAdd(counter, (uint32_t)__popcll(mask));
    base = __shfl(base, leader);
    return base + lane_rank;
}

// ---------------------------------------------------------------------------
// Photon path n (Sec. 2, Sec. 3.3): emitter by power, point by folding,
// cosine direction, then bounces until a miss, an absorbing surface, Russian
// roulette or the cap; a photon is stored at every diffuse hit.  The path is
// split into emission and single bounces so that a lane can switch to a new
// path as soon as its path ends (regeneration).
// ---------------------------------------------------------------------------
struct PhotonPath {
    Rng g;
    V3 org, dir;
    float phi;
    int32_t excl;
    uint32_t n;
    int32_t b;     // next bounce index
    int32_t last;  // last bounce written to the adjoint row (recording only)
};

// Returns false when the scene has no emitter (the path is empty).
__device__ __forceinline__ bool photon_emit(const SppmDev &d, uint32_t k, uint32_t n, PhotonPath &P) {
    const SceneDev &sc = d.sc;
    P.n = n;
    P.b = 0;
    P.last = -1;
    if (sc.n_emit == 0) return false;
    P.g = rng_seed(d.seed, kKindPhoton, k, (uint64_t)n);
    float u0 = rng_next(P.g);
    double target = (double)u0 * sc.power;
    // first emitter whose cumulative power exceeds the target
    int32_t lo = 0, hi = sc.n_emit - 1;
    while (lo < hi) {
        int32_t mid = (lo + hi) >> 1;
        if (target < sc.emit_cdf[mid]) hi = mid;
        else lo = mid + 1;
    }
    Tri et = load_tri(sc.bvh.tris, sc.emit_pos[lo]);
    float u1 = rng_next(P.g), u2 = rng_next(P.g);
    if (u1 + u2 > 1.0f) {
        u1 = 1.0f - u1;
        u2 = 1.0f - u2;
    }
    const V3 e1 = tri_e1(et), e2 = tri_e2(et);
    P.org = v3((et.v0.x + u1 * e1.x) + u2 * e2.x, (et.v0.y + u1 * e1.y) + u2 * e2.y,
               (et.v0.z + u1 * e1.z) + u2 * e2.z);
    P.dir = cosine_dir(tri_normal(et), P.g);
    P.phi = d.phi0;
    P.excl = et.id;
    return true;
}

// One bounce of a live path; returns true while the path continues.
// kRecord (adjoint replay): row n of mat_tab gets, per bounce, the material of
// a stored photon (kMatNone: none at that bounce), and the matching entries of
// adj_tab are cleared for the adjoint gather; photon_finish marks the end
// (kMatEnd).  Material ids are below kMaxAdjMat, so neither marker is a material.
template <bool kRecord, bool kStats>
__device__ __forceinline__ bool photon_shade(const SppmDev &d, PhotonPath &P, int32_t h, float t, uint32_t kp,
                                             uint16_t *__restrict__ mat_tab, long long *__restrict__ adj_tab,
                                             LaneStats *ls);

template <bool kRecord, bool kStats = false>
__device__ __forceinline__ bool photon_bounce(const SppmDev &d, PhotonPath &P, uint16_t *__restrict__ mat_tab,
                                              long long *__restrict__ adj_tab, LaneStats *ls = nullptr) {
    const SceneDev &sc = d.sc;
    float t;
    uint32_t kp;
    TraceStats st{0u, 0u};
    int32_t h = closest_hit<kStats, true>(sc.bvh, ray_set(d, P.dir), P.org, P.dir, sc.eps, __builtin_inff(), P.excl,
                                          t, kp, st, d.paired_walk != 0);
    if (kStats) {
        ls->rays++;
        ls->boxes += st.boxes;
        ls->tris += st.tris;
    }
    return photon_shade<kRecord, kStats>(d, P, h, t, kp, mat_tab, adj_tab, ls);
}

// The rest of a bounce once the closest hit (h, t, kp) of the ray from P.org
// along P.dir is known: store a photon at a diffuse hit, Russian roulette and
// a new cosine direction, or a specular direction; returns true while the
// path continues.
template <bool kRecord, bool kStats>
__device__ __forceinline__ bool photon_shade(const SppmDev &d, PhotonPath &P, int32_t h, float t, uint32_t kp,
                                             uint16_t *__restrict__ mat_tab, long long *__restrict__ adj_tab,
                                             LaneStats *ls) {
    const SceneDev &sc = d.sc;
    const int32_t mb = d.max_bounces;
    const int b = P.b;
    if (h < 0) return false;
    V3 x = vray(P.org, t, P.dir);
    Tri tr = load_tri(sc.bvh.tris, kp);
    V3 nrm = tri_normal(tr);
    uint32_t m = tr.mat;
    int type = sc.mat_type[m];
    uint16_t *row = kRecord ? mat_tab + (size_t)P.n * mb : nullptr;
    if (kRecord) {
        row[b] = kMatNone;
        P.last = b;
    }
    if (type == PM_MAT_DIFFUSE) {
        float rho = sc.mat_rho[m];
        if (!(rho > 0.0f)) return false;
        if (kRecord) {
            row[b] = (uint16_t)m;
            adj_tab[(size_t)P.n * mb + b] = 0;
        }
        if (kStats) ls->stored++;
        uint32_t slot = wave_append(&d.counters[0]);
        if (slot < d.cap) {
            d.store[2 * (size_t)slot] = make_float4(x.x, x.y, x.z, P.phi);
            d.store[2 * (size_t)slot + 1] = make_float4(P.dir.x, P.dir.y, P.dir.z, __uint_as_float((P.n << 5) | (uint32_t)b));
        } else {
            atomicOr(&d.counters[1], 1u);
        }
        float u = rng_next(P.g);
        float q = sc.mat_q[m];
        if (!(u < q)) return false;
        P.phi = (P.phi * rho) / q;
        V3 ns = vdot(P.dir, nrm) < 0.0f ? nrm : vneg(nrm);
        P.dir = cosine_dir(ns, P.g);
    } else if (type == PM_MAT_MIRROR) {
        P.dir = reflect(P.dir, nrm);
    } else {
        P.dir = glass_dir(P.dir, nrm, sc.mat_ior[m], P.g);
    }
    P.org = x;
    P.excl = h;
    P.b = b + 1;
    return P.b < mb;
}

template <bool kRecord>
__device__ __forceinline__ void photon_finish(const SppmDev &d, const PhotonPath &P, uint16_t *__restrict__ mat_tab) {
    if (kRecord && P.last + 1 < d.max_bounces) mat_tab[(size_t)P.n * d.max_bounces + P.last + 1] = kMatEnd;
}

// Photon path n traced to its end by one lane.
template <bool kRecord>
__device__ __forceinline__ void photon_elem(const SppmDev &d, uint32_t k, uint32_t n, uint16_t *__restrict__ mat_tab,
                                            long long *__restrict__ adj_tab) {
    PhotonPath P;
    if (photon_emit(d, k, n, P))
        while (photon_bounce<kRecord>(d, P, mat_tab, adj_tab)) {
        }
    photon_finish<kRecord>(d, P, mat_tab);
}

// Path state in device memory (56 B per slot, structure of arrays), used by
// the one-bounce-per-pass schedule and by the two-phase photon pass.
constexpr uint32_t kSlotIdle = 0xffffffffu;

struct PassSlots {
    int4 *g;     // [S] random stream state
    float4 *o;   // [S] origin, flux
    float4 *w;   // [S] direction, excluded triangle (int bits)
    uint2 *nb;   // [S] path index (kSlotIdle: none), next bounce
    uint32_t S;
};

__device__ __forceinline__ bool slot_load(const PassSlots &ps, uint32_t s, PhotonPath &P) {
    const uint2 nb = ps.nb[s];
    if (nb.x == kSlotIdle) return false;
    const int4 g = ps.g[s];
    const float4 o = ps.o[s], w = ps.w[s];
    P.g = Rng{g.x, g.y, g.z, g.w};
    P.org = v3(o.x, o.y, o.z);
    P.phi = o.w;
    P.dir = v3(w.x, w.y, w.z);
    P.excl = __float_as_int(w.w);
    P.n = nb.x;
    P.b = (int32_t)nb.y;
    P.last = -1;
    return true;
}

__device__ __forceinline__ void slot_store(const PassSlots &ps, uint32_t s, const PhotonPath &P, bool live) {
    if (live) {
        ps.g[s] = make_int4(P.g.s0, P.g.s1, P.g.s2, P.g.s3);
        ps.o[s] = make_float4(P.org.x, P.org.y, P.org.z, P.phi);
        ps.w[s] = make_float4(P.dir.x, P.dir.y, P.dir.z, __int_as_float(P.excl));
        ps.nb[s] = make_uint2(P.n, (uint32_t)P.b);
    } else {
        ps.nb[s] = make_uint2(kSlotIdle, 0u);
    }
}

// Two-phase photon pass (PM_PHOTON_TWO_PHASE).  A path can reflect inside a
// glass object up to the bounce limit, so the pass ends with a few long paths
// on an almost idle device.  The first launch (regeneration) stops once the
// path counter has run out and at most kParkLive lanes of a wavefront still
// hold a path: those paths go to a queue in device memory and the wavefront
// exits.  A second launch, on a stream of its own, continues the queued
// paths, so the first launch of the next iteration can start beside it.
// Each path consumes its random stream as in photon_elem, so the photons are
// the same.
#ifndef PM_PARK_LIVE
#define PM_PARK_LIVE 32
#endif
constexpr uint32_t kParkLive = PM_PARK_LIVE;

struct PathQueue {
    PassSlots s;    // s.S slots: at least the first launch's lanes
    uint32_t *cnt;  // [0] paths queued, [1] queued paths taken by the second launch
};

// Photon paths with regeneration (Sec. 3.3): persistent lanes trace one bounce
// per step; a lane whose path ended takes the next path index from the
// counter d.counters[2] once at least `refill` lanes of its wave are idle (or
// all are).  Every step advances each live path by one bounce and paths are
// bounded by max_bounces, so every wave exits once the counter passes n_paths.
// Called by every lane of a wave; the wave's lanes must share one scene.
// kRecord (adjoint replay): paths also write their rows of mat_tab / adj_tab
// as in photon_elem.  kPark (first launch of the two-phase pass): once the
// path counter has run out and at most kParkLive lanes hold a path, those
// paths go to the queue and the wave stops.  kQueue (second launch): the
// lanes take the queued paths (counted by queue.cnt[1]) instead of starting
// new ones.
template <bool kRecord = false, bool kStats = false, bool kPark = false, bool kQueue = false>
__device__ __forceinline__ void photon_regen_loop(const SppmDev &d, uint32_t k, uint32_t refill,
                                                  uint16_t *__restrict__ mat_tab = nullptr,
                                                  long long *__restrict__ adj_tab = nullptr,
                                                  PathQueue queue = PathQueue{}) {
    PhotonPath P;
    LaneStats ls;
    bool live = false, exhausted = false;
    uint32_t n_queued = 0u;
    if constexpr (kQueue) n_queued = queue.cnt[0];
    for (;;) {
        bool idle = !live && !exhausted;
        uint64_t idle_mask = __ballot(idle);
        uint64_t live_mask = __ballot(live);
        if (idle_mask != 0ull && (live_mask == 0ull || (uint32_t)__popcll(idle_mask) >= refill)) {
            uint32_t n = wave_fetch_add(kQueue ? &queue.cnt[1] : &d.counters[2], idle_mask, idle);
            if (idle) {
                if constexpr (kQueue) {
                    if (n < n_queued) {
                        live = slot_load(queue.s, n, P);
                        // recording: a live path's last written bounce is the one before its next
                        if (kRecord) P.last = P.b - 1;
                    } else {
                        exhausted = true;
                    }
                } else if (n < d.n_paths) {
                    live = photon_emit(d, k, n, P);
                    if (kStats) ls.paths++;
                    if (kRecord && !live) photon_finish<true>(d, P, mat_tab);
                } else {
                    exhausted = true;
                }
            }
            live_mask = __ballot(live);
        }
        if (live_mask == 0ull && __ballot(!exhausted) == 0ull) break;
        if constexpr (kPark) {
            if (__ballot(exhausted) != 0ull && (uint32_t)__popcll(live_mask) <= kParkLive) {
                if (live_mask != 0ull) {
                    const uint32_t v = wave_fetch_add(&queue.cnt[0], live_mask, live);
                    if (live) slot_store(queue.s, v, P, true);
                }
                break;
            }
        }
        if (live) {
            live = photon_bounce<kRecord, kStats>(d, P, mat_tab, adj_tab, &ls);
            if (kRecord && !live) photon_finish<true>(d, P, mat_tab);
        }
    }
    if (kStats) {
        wave_stats_flush(d.stats + kStatPhotonPaths, ls);
        wave_stat_add(d.stats + kStatPhotonStored, ls.stored);
    }
}

// Photon paths from a wavefront's queue in LDS (PM_PHOTON_POOL).  Each
// wavefront keeps up to kPoolSlots started paths in its own slice of LDS.
// Once some lanes are idle and the queue holds fewer paths than that, the
// whole wavefront starts 64 new paths at once (every lane emits one, so the
// emission runs at full width) and appends them to the queue, compacted by
// ballot rank.  Then every idle lane takes a queued path, so the lanes of a
// bounce step are full until the path counter runs out.  Each path consumes
// its random stream as in photon_elem, so the photons are the same.  Every
// step advances each live path by one bounce, and a wavefront starts new
// paths only while the counter is below n_paths, so every wavefront exits.
// Called by every lane of a wavefront; pool is the wavefront's slice
// (kPoolWords x kPoolSlots words), used by that wavefront only.
constexpr int kPoolSlots = 128;  // >= 63 queued + 64 new
constexpr int kPoolWords = 14;   // Rng (4), org (3), dir (3), phi, excl, n, b

__device__ __forceinline__ void pool_put(uint32_t *pool, uint32_t slot, const PhotonPath &P) {
    const uint32_t w[kPoolWords] = {(uint32_t)P.g.s0, (uint32_t)P.g.s1, (uint32_t)P.g.s2, (uint32_t)P.g.s3,
                                    __float_as_uint(P.org.x), __float_as_uint(P.org.y), __float_as_uint(P.org.z),
                                    __float_as_uint(P.dir.x), __float_as_uint(P.dir.y), __float_as_uint(P.dir.z),
                                    __float_as_uint(P.phi), (uint32_t)P.excl, P.n, (uint32_t)P.b};
#pragma unroll
    for (int i = 0; i < kPoolWords; ++i) pool[i * kPoolSlots + slot] = w[i];
}

__device__ __forceinline__ void pool_get(const uint32_t *pool, uint32_t slot, PhotonPath &P) {
    uint32_t w[kPoolWords];
#pragma unroll
    for (int i = 0; i < kPoolWords; ++i) w[i] = pool[i * kPoolSlots + slot];
    P.g.s0 = (int32_t)w[0];
    P.g.s1 = (int32_t)w[1];
    P.g.s2 = (int32_t)w[2];
    P.g.s3 = (int32_t)w[3];
    P.org = v3(__uint_as_float(w[4]), __uint_as_float(w[5]), __uint_as_float(w[6]));
    P.dir = v3(__uint_as_float(w[7]), __uint_as_float(w[8]), __uint_as_float(w[9]));
    P.phi = __uint_as_float(w[10]);
    P.excl = (int32_t)w[11];
    P.n = w[12];
    P.b = (int32_t)w[13];
    P.last = -1;
}

template <bool kStats = false>
__device__ __forceinline__ void photon_pool_loop(const SppmDev &d, uint32_t k, uint32_t *__restrict__ pool) {
    PhotonPath P;
    LaneStats ls;
    bool live = false, exhausted = false;
    uint32_t queued = 0;  // paths in the queue (wave-uniform)
    for (;;) {
        const uint64_t idle_mask = __ballot(!live);
        const uint32_t n_idle = (uint32_t)__popcll(idle_mask);
        if (n_idle != 0u && queued < n_idle && !exhausted) {
            // every lane starts a path; the started ones join the queue
            const uint32_t n = wave_fetch_add(&d.counters[2], __ballot(1), true);
            PhotonPath Q;
            bool ok = false;
            if (n < d.n_paths) {
                ok = photon_emit(d, k, n, Q);
                if (kStats) ls.paths++;
            }
            exhausted = __ballot(n >= d.n_paths) != 0ull;
            const uint64_t ok_mask = __ballot(ok);
            if (ok) {
                const uint32_t rank = __builtin_amdgcn_mbcnt_hi((uint32_t)(ok_mask >> 32),
                                                                __builtin_amdgcn_mbcnt_lo((uint32_t)ok_mask, 0u));
                pool_put(pool, queued + rank, Q);
            }
            queued += (uint32_t)__popcll(ok_mask);
            // the queue is shared by the wavefront's lanes: order the writes before the reads below
            __builtin_amdgcn_fence(__ATOMIC_SEQ_CST, "wavefront");
            __builtin_amdgcn_wave_barrier();
        }
        // idle lanes take queued paths, the last ones first
        const uint32_t take = n_idle < queued ? n_idle : queued;
        if (!live) {
            const uint32_t rank = __builtin_amdgcn_mbcnt_hi((uint32_t)(idle_mask >> 32),
                                                            __builtin_amdgcn_mbcnt_lo((uint32_t)idle_mask, 0u));
            if (rank < take) {
                pool_get(pool, queued - 1u - rank, P);
                live = true;
            }
        }
        queued -= take;
        // the slots just read may be written by the next refill
        __builtin_amdgcn_fence(__ATOMIC_SEQ_CST, "wavefront");
        __builtin_amdgcn_wave_barrier();
        if (__ballot(live) == 0ull && exhausted && queued == 0u) break;
        if (live) live = photon_bounce<false, kStats>(d, P, nullptr, nullptr, &ls);
    }
    if (kStats) {
        wave_stats_flush(d.stats + kStatPhotonPaths, ls);
        wave_stat_add(d.stats + kStatPhotonStored, ls.stored);
    }
}

// Photon paths with regeneration at ray granularity: each lane walks its own
// ray; once at least `refill` lanes of the wave wait (their ray has ended, or
// they have no path and paths remain), those lanes shade their hits and start
// the next ray of their path, or take a new path from the counter
// d.counters[2], while the other lanes keep walking.  A wave therefore does
// not wait for its longest walk at every bounce.  Every path consumes its
// random stream exactly as in photon_elem, so the photons are the same.
// Each round of walk steps advances every walking lane and each shading round
// serves every waiting lane, so every wave exits once the counter passes
// n_paths.  Called by every lane of a wave.
constexpr int kStreamVoteSteps = 4;  // walk steps between two votes of the wave

template <bool kStats = false>
__device__ __forceinline__ void photon_stream_loop(const SppmDev &d, uint32_t k, uint32_t refill) {
    const SceneDev &sc = d.sc;
    PhotonPath P;
    Walker w;
    TraceStats st{0u, 0u};
    LaneStats ls;
    bool live = false, walking = false, exhausted = false;
    const bool paired = d.paired_walk != 0;
    for (;;) {
        if (live && !walking) {  // this lane's ray has ended: the rest of its bounce
            if (kStats) ls.rays++;
            // the walker holds the ray (P's copies need not stay live during the walk)
            P.org = w.o;
            P.dir = w.d;
            P.excl = w.exclude;
            live = photon_shade<false, kStats>(d, P, w.best, w.t_hit(), w.best_k, nullptr, nullptr, &ls);
            if (live) {
                w.init(sc.bvh, ray_set(d, P.dir), P.org, P.dir, sc.eps, __builtin_inff(), P.excl);
                walking = true;
            }
        }
        const bool idle = !live && !exhausted;
        const uint64_t idle_mask = __ballot(idle);
        if (idle_mask != 0ull) {
            const uint32_t n = wave_fetch_add(&d.counters[2], idle_mask, idle);
            if (idle) {
                if (n < d.n_paths) {
                    live = photon_emit(d, k, n, P);
                    if (kStats) ls.paths++;
                    if (live) {
                        w.init(sc.bvh, ray_set(d, P.dir), P.org, P.dir, sc.eps, __builtin_inff(), P.excl);
                        walking = true;
                    }
                } else {
                    exhausted = true;
                }
            }
        }
        if (__ballot(live) == 0ull && __ballot(!exhausted) == 0ull) break;
        for (;;) {
            const uint64_t walk_mask = __ballot(walking);
            if (walk_mask == 0ull) break;
            // waiting lanes: a finished ray to shade, or no path while paths remain
            if ((uint32_t)__popcll(__ballot(!walking && (live || !exhausted))) >= refill) break;
#pragma unroll
            for (int u = 0; u < kStreamVoteSteps; ++u) {
                if (walking) {
                    if (paired)
                        w.step2<kStats>(sc.bvh.tris, st);
                    else
                        w.step<kStats>(sc.bvh.tris, st);
                    walking = !w.done();
                }
            }
        }
    }
    if (kStats) {
        ls.boxes = st.boxes;
        ls.tris = st.tris;
        wave_stats_flush(d.stats + kStatPhotonPaths, ls);
        wave_stat_add(d.stats + kStatPhotonStored, ls.stored);
    }
}

// Regeneration over the paths [n0, n1) of one wavefront (batched photon
// stage): the path cursor is a wave-uniform register, so lanes take new paths
// without atomics.  Called by every lane of a wave; the loop ends once the
// range is handed out and no path is live.
__device__ __forceinline__ void photon_regen_range(const SppmDev &d, uint32_t k, uint32_t n0, uint32_t n1,
                                                   uint32_t refill) {
    PhotonPath P;
    bool live = false;
    uint32_t next = n0;
    for (;;) {
        const bool idle = !live;
        const uint64_t idle_mask = __ballot(idle);
        uint64_t live_mask = __ballot(live);
        if (next < n1 && idle_mask != 0ull && (live_mask == 0ull || (uint32_t)__popcll(idle_mask) >= refill)) {
            const uint32_t rank =
                __builtin_amdgcn_mbcnt_hi((uint32_t)(idle_mask >> 32), __builtin_amdgcn_mbcnt_lo((uint32_t)idle_mask, 0u));
            if (idle && next + rank < n1) live = photon_emit(d, k, next + rank, P);
            next += (uint32_t)__popcll(idle_mask);
            live_mask = __ballot(live);
        }
        if (live_mask == 0ull && next >= n1) break;
        if (live) live = photon_bounce<false>(d, P, nullptr, nullptr);
    }
}

// ---------------------------------------------------------------------------
// Photon paths one bounce per pass (Sec. 3.3 as the paper schedules it): a
// fixed pool of threads, each owning one slot; every launch (a pass) moves the
// path of each slot by exactly one bounce, so no thread deposits more than
// a single photon in a pass.  A slot whose path was killed or left the scene takes the
// next path index in the following pass and traces that path's first segment
// there.  A slot's path state lives in memory between passes.
// ---------------------------------------------------------------------------
// The path counter as one value for the whole wave (it only grows).
__device__ __forceinline__ uint32_t paths_handed_out(const SppmDev &d) {
    const uint32_t c = __hip_atomic_load(&d.counters[2], __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
    return (uint32_t)__builtin_amdgcn_readfirstlane((int)c);
}

// One pass of slot s.  Called by every lane of a wave; lanes with s >= S
// only take part in the wave's votes.
__device__ __forceinline__ void photon_pass_elem(const SppmDev &d, uint32_t k, const PassSlots &ps, uint32_t s) {
    const bool in = s < ps.S;
    PhotonPath P;
    const bool was_live = in && slot_load(ps, s, P);
    bool live = was_live;
    const bool want = in && !was_live;
    const uint64_t want_mask = __ballot(want);
    if (want_mask != 0ull && paths_handed_out(d) < d.n_paths) {
        const uint32_t n = wave_fetch_add(&d.counters[2], want_mask, want);
        if (want && n < d.n_paths) live = photon_emit(d, k, n, P);
    }
    if (live) live = photon_bounce<false>(d, P, nullptr, nullptr);
    if (in && (live || was_live)) slot_store(ps, s, P, live);
}

// After the last pass: the paths still in flight are traced to their end and
// the paths no pass started are taken by regenerating lanes.  Called by every
// lane of a wave.
__device__ __forceinline__ void photon_drain_elem(const SppmDev &d, uint32_t k, const PassSlots &ps, uint32_t s) {
    PhotonPath P;
    bool live = s < ps.S && slot_load(ps, s, P);
    if (live) wave_append(&d.counters[3]);
    while (live) live = photon_bounce<false>(d, P, nullptr, nullptr);
    if (paths_handed_out(d) < d.n_paths) photon_regen_loop(d, k, d.refill);
}

// ---------------------------------------------------------------------------
// Hashed grid: cell edge h = 2 R_max (1 + 2^-10), so the 2x2x2 cells around a
// hit point cover its disc; cells hash (Teschner et al. 2003) into a
// power-of-two table; photons are counting-sorted by bucket.  The exact
// gather uses fine cells instead, h = R_max (1 + 2^-5): a disc then touches
// at most 3 cells per axis, and a hit point examines the photons of a smaller
// region.
// ---------------------------------------------------------------------------
struct Grid {
    float lo[3];
    float inv_h;
    uint32_t mask;
    uint32_t fine;
};

__device__ __forceinline__ uint32_t cell_hash(int32_t ix, int32_t iy, int32_t iz, uint32_t mask) {
    return (((uint32_t)ix * 73856093u) ^ ((uint32_t)iy * 19349663u) ^ ((uint32_t)iz * 83492791u)) & mask;
}

// Fine cells only while the scene spans at most 4096 of them, which bounds the
// rounding slack of the cell coordinates (see disc_cells).
constexpr double kFineMaxCells = 4096.0;

// The exact gather uses fine cells wherever they are allowed: on the box and
// procedural scenes they cost the same as 2 R_max cells when discs hold tens
// of photons and save 11-14% of the iteration when they hold thousands.  The
// stochastic estimator is defined on the 2 R_max grid.
__device__ __forceinline__ Grid make_grid(const SppmDev &d) {
    double r2 = __longlong_as_double((long long)*d.r2max);
    double h = 2.0 * sqrt(r2) * (1.0 + 1.0 / 1024.0);
    Grid gr;
    gr.fine = 0u;
    if (d.gather_mode == PM_GATHER_EXACT) {
        const double hf = sqrt(r2) * (1.0 + 1.0 / 32.0);
        if (hf > 0.0 && (double)d.sc.ext <= kFineMaxCells * hf) {
            h = hf;
            gr.fine = 1u;
        }
    }
    gr.lo[0] = d.sc.lo[0];
    gr.lo[1] = d.sc.lo[1];
    gr.lo[2] = d.sc.lo[2];
    gr.inv_h = h > 0.0 ? (float)(1.0 / h) : 0.0f;
    gr.mask = d.mask;
    return gr;
}

__device__ __forceinline__ uint32_t photon_bucket(const Grid &gr, float x, float y, float z) {
    int32_t ix = (int32_t)floorf((x - gr.lo[0]) * gr.inv_h);
    int32_t iy = (int32_t)floorf((y - gr.lo[1]) * gr.inv_h);
    int32_t iz = (int32_t)floorf((z - gr.lo[2]) * gr.inv_h);
    return cell_hash(ix, iy, iz, gr.mask);
}

__device__ __forceinline__ uint32_t stored_photons(const SppmDev &d) { return min(d.counters[0], d.cap); }

// Largest squared radius among valid hit points (positive doubles order like
// their bit patterns): rmax_lane gives one pixel's candidate, rmax_flush
// reduces a wave's candidates and folds them into the result with one atomic.
// rmax_flush is called by every lane of a wave; its lanes must belong to one
// scene.
__device__ __forceinline__ unsigned long long rmax_lane(const SppmDev &d, const double *__restrict__ R2src, int64_t p) {
    if (__float_as_int(d.hp_nrm[p].w) < 0) return 0ull;
    return (unsigned long long)__double_as_longlong(R2src[p]);
}

__device__ __forceinline__ void rmax_flush(const SppmDev &d, unsigned long long v) {
    for (int off = 32; off > 0; off >>= 1) {
        unsigned long long o = __shfl_xor(v, off);
        v = o > v ? o : v;
    }
    if ((threadIdx.x & 63) == 0 && v) atomicMax(d.r2max, v);
}

// Counting sort of the stored photons by bucket: the count pass keeps each
// photon's bucket and its rank in the bucket (the value its atomic returned);
// after the scan the scatter places it at the bucket's start + rank, which
// is below the next bucket's start, with no further atomics.
__device__ __forceinline__ void count_elem(const SppmDev &d, const Grid &gr, uint32_t j, uint32_t *__restrict__ cell_count) {
    float4 a = d.store[2 * (size_t)j];
    const uint32_t hb = photon_bucket(gr, a.x, a.y, a.z);
    d.key_rank[j] = make_uint2(hb, atomicAdd(&cell_count[d.table_off + hb], 1u));
}

__device__ __forceinline__ void scatter_elem(const SppmDev &d, uint32_t j, const uint32_t *__restrict__ start,
                                             float4 *__restrict__ sorted) {
    float4 a = d.store[2 * (size_t)j];
    float4 b = d.store[2 * (size_t)j + 1];
    const uint2 kr = d.key_rank[j];
    const uint32_t pos = start[d.table_off + kr.x] + kr.y;
    sorted[2 * (size_t)pos] = a;
    sorted[2 * (size_t)pos + 1] = b;
}

// The photons of one bucket inside the disc (squared distance < R^2, float32
// distance compared in double) that arrived from the eye's side.
template <typename F>
__device__ __forceinline__ void photons_of_bucket(const SppmDev &d, uint32_t hb, float4 hx, float4 hn, double r2,
                                                  const uint32_t *__restrict__ start, const float4 *__restrict__ sorted,
                                                  F &f) {
    uint32_t q0 = start[d.table_off + hb], q1 = start[d.table_off + hb + 1];
    for (uint32_t q = q0; q < q1; ++q) {
        float4 a = sorted[2 * (size_t)q];
        float dx = a.x - hx.x, dy = a.y - hx.y, dz = a.z - hx.z;
        float d2 = (dx * dx + dy * dy) + dz * dz;
        if ((double)d2 < r2) {
            float4 b = sorted[2 * (size_t)q + 1];
            float c2 = (b.x * hn.x + b.y * hn.y) + b.z * hn.z;
            if (c2 < 0.0f) f(a, b);
        }
    }
}

// The cells a hit point's disc can reach, as a block of at most 3x3x3 cells
// from c0; bit t of `uniq` marks cell c0 + (t % 3, t / 3 % 3, t / 9) as the
// first of the block's cells in its bucket (hash collisions are visited once).
struct DiscCells {
    int32_t c0[3];
    uint32_t uniq;
};

__device__ __forceinline__ uint32_t disc_cell_bucket(const Grid &gr, const int32_t c0[3], int t) {
    return cell_hash(c0[0] + t % 3, c0[1] + (t / 3) % 3, c0[2] + t / 9, gr.mask);
}

// In cell units the disc spans cc -/+ rr per axis, rr widened by 2^-8
// relative and by (|cc| + 1) 2^-s absolute, far above the rounding of the cell
// coordinates, so no cell holding a photon of the disc is left out.
// * Fine cells (edge R_max (1 + 2^-5), at most 4096 across the scene, s = 20):
//   rr < 0.98, so floor(cc - rr) .. floor(cc + rr) are at most 3 cells.
// * Cells of edge 2 R_max (1 + 2^-10) (s = 16): the cells b and b + 1 with
//   b = floor(cc - 1/2) contain the disc; one of them is dropped when the
//   widened disc does not reach it.
__device__ __forceinline__ DiscCells disc_cells(const Grid &gr, float4 hx, double r2) {
    const float cc[3] = {(hx.x - gr.lo[0]) * gr.inv_h, (hx.y - gr.lo[1]) * gr.inv_h, (hx.z - gr.lo[2]) * gr.inv_h};
    const float rc = (float)sqrt(r2) * gr.inv_h;
    DiscCells dc;
    uint32_t nc[3];
    for (int a = 0; a < 3; ++a) {
        if (gr.fine) {
            const float rr = rc * (1.0f + 0x1p-8f) + (fabsf(cc[a]) + 1.0f) * 0x1p-20f;
            dc.c0[a] = (int32_t)floorf(cc[a] - rr);
            nc[a] = (uint32_t)min((int32_t)floorf(cc[a] + rr) - dc.c0[a] + 1, 3);
        } else {
            const float rr = rc * (1.0f + 0x1p-8f) + (fabsf(cc[a]) + 1.0f) * 0x1p-16f;
            const int32_t bb = (int32_t)floorf(cc[a] - 0.5f);
            const float mid = (float)(bb + 1);
            const bool lower = cc[a] - rr < mid, upper = cc[a] + rr >= mid;
            dc.c0[a] = lower ? bb : bb + 1;
            nc[a] = (lower ? 1u : 0u) + (upper ? 1u : 0u);
        }
    }
    uint32_t hs[27];
    dc.uniq = 0u;
#pragma unroll
    for (int t = 0; t < 27; ++t) {
        const bool used = (uint32_t)(t % 3) < nc[0] && (uint32_t)((t / 3) % 3) < nc[1] && (uint32_t)(t / 9) < nc[2];
        const uint32_t hb = used ? disc_cell_bucket(gr, dc.c0, t) : 0xffffffffu;
        hs[t] = hb;
        bool dup = false;
#pragma unroll
        for (int e = 0; e < t; ++e) dup |= (hs[e] == hb);
        if (used && !dup) dc.uniq |= 1u << t;
    }
    return dc;
}

// Visit every photon inside a hit point's disc that arrived from the eye's
// side, through the distinct buckets of the cells its disc can reach.
template <typename F>
__device__ __forceinline__ void for_each_photon_in_disc(const SppmDev &d, const Grid &gr, float4 hx, float4 hn, double r2,
                                                       const uint32_t *__restrict__ start,
                                                       const float4 *__restrict__ sorted, F &&f) {
    const DiscCells dc = disc_cells(gr, hx, r2);
    for (uint32_t m = dc.uniq; m != 0u; m &= m - 1u)
        photons_of_bucket(d, disc_cell_bucket(gr, dc.c0, __builtin_ctz(m)), hx, hn, r2, start, sorted, f);
}

// Adds n fixed-point flux terms rint(v) to F; `bad` is set when a term or the
// sum leaves the range of u64 (the sum itself stays the sum modulo 2^64).
__device__ __forceinline__ void flux_add(unsigned long long &F, double v, uint32_t n, bool &bad) {
    const double t = rint(v);
    const bool ok = t < 0x1p63;  // v >= 0; false for NaN too
    const unsigned long long u = ok ? (unsigned long long)t : 0ull;
    const unsigned long long un = u * (unsigned long long)n;
    bad |= !ok || __umul64hi(u, (unsigned long long)n) != 0ull;
    const unsigned long long s = F + un;
    bad |= s < F;
    F = s;
}

// ---------------------------------------------------------------------------
// Stochastic spatial hashing (Sec. 3.4): every photon is hashed to the entry
// of its cell (the same grid and table as above); the entry keeps one photon,
// the smallest (random depth, photon id) -- a z-buffer test with a depth drawn
// per photon from stream (seed, DEPTH, k, path * 32 + bounce), independent of
// the path's properties -- and counts the photons it received.  A hit point
// counts each surviving photon inside its disc once per photon of its entry.
// The smallest key wins whatever the order of the atomics, so the estimate is
// deterministic.
// ---------------------------------------------------------------------------
constexpr uint32_t kKindDepth = 3u;

__device__ __forceinline__ unsigned long long photon_key(const SppmDev &d, uint32_t k, uint32_t id) {
    Rng g = rng_seed(d.seed, kKindDepth, k, (uint64_t)id);
    float depth = rng_next(g);
    return ((unsigned long long)__float_as_uint(depth) << 32) | (unsigned long long)id;
}

__device__ __forceinline__ void sh_insert_elem(const SppmDev &d, const Grid &gr, uint32_t k, uint32_t j,
                                               uint32_t *__restrict__ count) {
    float4 a = d.store[2 * (size_t)j];
    uint32_t id = __float_as_uint(d.store[2 * (size_t)j + 1].w);
    uint32_t e = d.table_off + photon_bucket(gr, a.x, a.y, a.z);
    atomicAdd(&count[e], 1u);
    atomicMin(&d.sh_key[e], photon_key(d, k, id));
}

__device__ __forceinline__ void sh_pick_elem(const SppmDev &d, const Grid &gr, uint32_t k, uint32_t j) {
    float4 a = d.store[2 * (size_t)j];
    uint32_t id = __float_as_uint(d.store[2 * (size_t)j + 1].w);
    uint32_t e = d.table_off + photon_bucket(gr, a.x, a.y, a.z);
    if (d.sh_key[e] == photon_key(d, k, id)) d.sh_surv[e] = j;
}

__device__ __forceinline__ void sh_gather_elem(const SppmDev &d, const Grid &gr, int64_t p,
                                               const uint32_t *__restrict__ count) {
    float4 hn = d.hp_nrm[p];
    uint32_t M = 0;
    unsigned long long F = 0ull;
    bool bad = false;
    if (__float_as_int(hn.w) >= 0) {
        float4 hx = d.hp_pos[p];
        const double wk = (double)hx.w, r2 = d.R2[p];
        int32_t bx = (int32_t)floorf((hx.x - gr.lo[0]) * gr.inv_h - 0.5f);
        int32_t by = (int32_t)floorf((hx.y - gr.lo[1]) * gr.inv_h - 0.5f);
        int32_t bz = (int32_t)floorf((hx.z - gr.lo[2]) * gr.inv_h - 0.5f);
        uint32_t seen[8];
        for (int c = 0; c < 8; ++c) {
            uint32_t hb = cell_hash(bx + (c & 1), by + ((c >> 1) & 1), bz + (c >> 2), gr.mask);
            bool dup = false;
            for (int e = 0; e < c; ++e) dup |= (seen[e] == hb);
            seen[c] = hb;
            if (dup) continue;
            const uint32_t n = count[d.table_off + hb];
            if (n == 0) continue;
            const uint32_t j = d.sh_surv[d.table_off + hb];
            float4 a = d.store[2 * (size_t)j];
            float dx = a.x - hx.x, dy = a.y - hx.y, dz = a.z - hx.z;
            float d2 = (dx * dx + dy * dy) + dz * dz;
            if (!((double)d2 < r2)) continue;
            float4 b = d.store[2 * (size_t)j + 1];
            float c2 = (b.x * hn.x + b.y * hn.y) + b.z * hn.z;
            if (!(c2 < 0.0f)) continue;
            M += n;
            flux_add(F, (wk * (double)a.w) * d.scale, n, bad);
        }
    }
    if (bad) atomicOr(&d.counters[1], 2u);
    d.M[p] = M;
    d.Phi[p] = F;
}

// Range query: per hit point, M photons and their flux, each term rounded to
// 2^-shift fixed point and summed as integers (order independent).  Called
// by every lane of a wave, one pixel per lane (p >= P: no pixel).  A hit
// point whose buckets hold at least kCoopMin photons is scanned by the whole
// wave, 64 consecutive photons per step, and the lanes' partial counts and
// sums are added up; the others are scanned by their own lane.  Both give the
// same M and flux.
constexpr uint32_t kCoopMin = 256;

__device__ __forceinline__ uint32_t lane_id() {
    return __builtin_amdgcn_mbcnt_hi(0xffffffffu, __builtin_amdgcn_mbcnt_lo(0xffffffffu, 0u));
}

__device__ __forceinline__ float readlane_f(float v, int l) {
    return __int_as_float(__builtin_amdgcn_readlane(__float_as_int(v), l));
}

template <bool kStats = false>
__device__ __forceinline__ void gather_wave(const SppmDev &d, const Grid &gr, int64_t p,
                                            const uint32_t *__restrict__ start, const float4 *__restrict__ sorted) {
    const bool in = p < d.P;
    const float4 hn = in ? d.hp_nrm[p] : make_float4(0.0f, 0.0f, 0.0f, __int_as_float(-1));
    const bool valid = in && __float_as_int(hn.w) >= 0;
    float4 hx = make_float4(0.0f, 0.0f, 0.0f, 0.0f);
    double r2 = 0.0;
    DiscCells dc{};
    uint32_t load = 0u;
    if (valid) {
        hx = d.hp_pos[p];
        r2 = d.R2[p];
        dc = disc_cells(gr, hx, r2);
        for (uint32_t m = dc.uniq; m != 0u; m &= m - 1u) {
            const uint32_t hb = d.table_off + disc_cell_bucket(gr, dc.c0, __builtin_ctz(m));
            load += start[hb + 1] - start[hb];
        }
    }
    const double scale = d.scale;
    uint32_t M = 0u;
    unsigned long long F = 0ull;
    bool bad = false;
    const bool coop = load >= kCoopMin;
    if (valid && !coop) {
        const double wk = (double)hx.w;
        auto add = [&](const float4 &a, const float4 &) {
            M++;
            flux_add(F, (wk * (double)a.w) * scale, 1u, bad);
        };
        for (uint32_t m = dc.uniq; m != 0u; m &= m - 1u)
            photons_of_bucket(d, disc_cell_bucket(gr, dc.c0, __builtin_ctz(m)), hx, hn, r2, start, sorted, add);
    }
    const uint32_t lane = lane_id();
    for (uint64_t todo = __ballot(coop); todo != 0ull; todo &= todo - 1ull) {
        const int L = __ffsll((unsigned long long)todo) - 1;
        const float4 xl = make_float4(readlane_f(hx.x, L), readlane_f(hx.y, L), readlane_f(hx.z, L), readlane_f(hx.w, L));
        const float4 nl = make_float4(readlane_f(hn.x, L), readlane_f(hn.y, L), readlane_f(hn.z, L), 0.0f);
        const unsigned long long r2b = (unsigned long long)__double_as_longlong(r2);
        const double r2l = __longlong_as_double(
            (long long)(((unsigned long long)(uint32_t)__builtin_amdgcn_readlane((int)(uint32_t)(r2b >> 32), L) << 32) |
                        (uint32_t)__builtin_amdgcn_readlane((int)(uint32_t)r2b, L)));
        const int32_t c0l[3] = {__builtin_amdgcn_readlane(dc.c0[0], L), __builtin_amdgcn_readlane(dc.c0[1], L),
                                __builtin_amdgcn_readlane(dc.c0[2], L)};
        const uint32_t uniql = (uint32_t)__builtin_amdgcn_readlane((int)dc.uniq, L);
        const double wk = (double)xl.w;
        uint32_t m = 0u;
        unsigned long long f = 0ull;
        bool fbad = false;
        for (uint32_t bits = uniql; bits != 0u; bits &= bits - 1u) {
            const uint32_t hb = d.table_off + disc_cell_bucket(gr, c0l, __builtin_ctz(bits));
            const uint32_t q1 = start[hb + 1];
            for (uint32_t q = start[hb] + lane; q < q1; q += 64u) {
                const float4 a = sorted[2 * (size_t)q];
                const float dx = a.x - xl.x, dy = a.y - xl.y, dz = a.z - xl.z;
                const float d2 = (dx * dx + dy * dy) + dz * dz;
                if ((double)d2 < r2l) {
                    const float4 b = sorted[2 * (size_t)q + 1];
                    const float c2 = (b.x * nl.x + b.y * nl.y) + b.z * nl.z;
                    if (c2 < 0.0f) {
                        m++;
                        flux_add(f, (wk * (double)a.w) * scale, 1u, fbad);
                    }
                }
            }
        }
        for (int off = 32; off > 0; off >>= 1) {
            m += __shfl_xor(m, off);
            const unsigned long long s = f + __shfl_xor(f, off);
            fbad |= s < f;  // a partial sum passing 2^64 wraps in some lane
            f = s;
        }
        const bool any_bad = __ballot(fbad) != 0ull;
        if ((int)lane == L) {
            M = m;
            F = f;
            bad = any_bad;
        }
    }
    if (in) {
        if (bad) atomicOr(&d.counters[1], 2u);
        d.M[p] = M;
        d.Phi[p] = F;
    }
    if (kStats) {  // hit points, distinct buckets visited, photons in them, photons accepted
        wave_stat_add(d.stats + kStatGatherHits, valid ? 1u : 0u);
        wave_stat_add(d.stats + kStatGatherBuckets, valid ? (uint64_t)__popc(dc.uniq) : 0u);
        wave_stat_add(d.stats + kStatGatherExamined, load);
        wave_stat_add(d.stats + kStatGatherAccepted, M);
    }
}

// Progressive update (radius reduction and flux rescaling of SPPM); hist
// (optional) receives the radius used in this iteration.
__device__ __forceinline__ void update_elem(const SppmDev &d, int64_t p, double *__restrict__ hist) {
    if (hist) hist[p] = d.R2[p];
    uint32_t Mi = d.M[p];
    if (__float_as_int(d.hp_nrm[p].w) < 0 || Mi == 0) return;
    double m = (double)Mi;
    double n0 = d.N[p];
    double nn = n0 + d.alpha * m;
    double ratio = nn / (n0 + m);
    d.R2[p] = d.R2[p] * ratio;
    d.tau[p] = (d.tau[p] + (double)d.Phi[p] * d.inv_scale) * ratio;
    d.N[p] = nn;
}

__device__ __forceinline__ float resolve_elem(const SppmDev &d, int64_t p, int32_t K) {
    double L = d.tau[p] / ((kPiD * d.R2[p]) * (double)K) + d.D[p] / (double)K;
    return (float)L;
}

// Block-wide exclusive scan of one value per thread (kBlock threads).
__device__ __forceinline__ uint32_t block_exscan(uint32_t v, uint32_t *lds_wave, uint32_t &total) {
    int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
    uint32_t x = v;
    for (int off = 1; off < 64; off <<= 1) {
        uint32_t y = __shfl_up(x, off);
        if (lane >= off) x += y;
    }
    if (lane == 63) lds_wave[wave] = x;
    __syncthreads();
    uint32_t before = 0;
    total = 0;
    for (int w = 0; w < kBlock / 64; ++w) {
        uint32_t s = lds_wave[w];
        if (w < wave) before += s;
        total += s;
    }
    __syncthreads();
    return before + x - v;
}

}  // namespace pmd
