// Stochastic progressive photon mapping on the device (Sec. 2): eye pass,
// photon pass, hashed-grid build, range query, progressive update, resolve.
#include <algorithm>
#include <cmath>
#include <cstring>
#include <vector>

#include "pm_device.h"
#include "runtime.h"
#include "sppm.h"

namespace {

using pmd::V3;

constexpr int kBlock = 256;
constexpr int kScanItems = 16;                      // per thread
constexpr int kScanTile = kBlock * kScanItems;      // 4096 buckets per block

struct SceneDev {
    pmd::Bvh bvh;
    const int32_t *mat_type;
    const float *mat_rho, *mat_q, *mat_Le, *mat_ior;
    const uint32_t *emit_pos;  // triangle-array position of each emitter (original order)
    const double *emit_cdf;
    int32_t n_emit;
    double power;
    float eps;
    float lo[3];
    V3 cpos, cf, cr, cu;
    float tanh_fov, aspect;
    int32_t W, H;
};

// ---------------------------------------------------------------------------
// Eye pass: per pixel, a jittered pinhole ray followed through mirror and
// glass to the first diffuse (rho > 0) surface, which becomes the pixel's hit
// point; directly seen emission is accumulated into D.
// hp_pos = (x, W*rho/pi), hp_nrm = (n toward the eye, material bits | -1).
// ---------------------------------------------------------------------------
__global__ __launch_bounds__(kBlock) void k_eye(SceneDev sc, uint64_t seed, uint32_t k, int32_t max_depth,
                                                float4 *__restrict__ hp_pos, float4 *__restrict__ hp_nrm,
                                                double *__restrict__ D) {
    // D == nullptr: replay (adjoint) -- hit points only
    int64_t p = (int64_t)pmd::xcd_block(blockIdx.x, gridDim.x) * kBlock + threadIdx.x;
    int64_t P = (int64_t)sc.W * sc.H;
    if (p >= P) return;
    int32_t px = (int32_t)(p % sc.W), py = (int32_t)(p / sc.W);
    pmd::Rng g = pmd::rng_seed(seed, pmd::kKindEye, k, (uint64_t)p);
    float j0 = pmd::rng_next(g), j1 = pmd::rng_next(g);
    float fx = ((float)px + j0) / (float)sc.W;
    float fy = ((float)py + j1) / (float)sc.H;
    float sx = (2.0f * fx - 1.0f) * (sc.tanh_fov * sc.aspect);
    float sy = (1.0f - 2.0f * fy) * sc.tanh_fov;
    V3 dir = pmd::vnorm(pmd::v3((sc.cf.x + sx * sc.cr.x) + sy * sc.cu.x, (sc.cf.y + sx * sc.cr.y) + sy * sc.cu.y,
                                (sc.cf.z + sx * sc.cr.z) + sy * sc.cu.z));
    V3 org = sc.cpos;
    float tmin = 0.0f, thr = 1.0f;
    int32_t excl = -1;
    double dadd = 0.0;
    float4 pos = make_float4(0.0f, 0.0f, 0.0f, 0.0f);
    float4 nrm = make_float4(0.0f, 0.0f, 0.0f, __int_as_float(-1));
    pmd::TraceStats st;
    for (int depth = 0; depth < max_depth; ++depth) {
        float t;
        uint32_t kp;
        int32_t h = pmd::closest_hit<false>(sc.bvh, pmd::link_set(dir), org, dir, tmin, __builtin_inff(), excl, t,
                                            kp, st);
        if (h < 0) break;
        V3 x = pmd::vray(org, t, dir);
        pmd::Tri tr = pmd::load_tri(sc.bvh.tris, kp);
        V3 n = pmd::tri_normal(tr);
        uint32_t m = tr.mat;
        bool front = pmd::vdot(dir, n) < 0.0f;
        float Le = sc.mat_Le[m];
        if (Le > 0.0f && front) dadd += (double)(thr * Le);
        int type = sc.mat_type[m];
        if (type == PM_MAT_DIFFUSE) {
            float rho = sc.mat_rho[m];
            if (rho > 0.0f) {
                V3 nh = front ? n : pmd::vneg(n);
                pos = make_float4(x.x, x.y, x.z, (thr * rho) * pmd::kInvPiF);
                nrm = make_float4(nh.x, nh.y, nh.z, __uint_as_float(m));
            }
            break;
        } else if (type == PM_MAT_MIRROR) {
            dir = pmd::reflect(dir, n);
        } else {
            dir = pmd::glass_dir(dir, n, sc.mat_ior[m], g);
        }
        org = x;
        tmin = sc.eps;
        excl = h;
    }
    hp_pos[p] = pos;
    hp_nrm[p] = nrm;
    if (D) D[p] += dadd;
}

// Wave-aggregated append: one atomic per wavefront for all lanes currently
// active at this call site.  Returns this lane's slot.
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
// Photon pass: one lane per photon path (Sec. 2, Sec. 3.3).  Emission point
// and direction from the emitters (by power), then bounces until a miss, an
// absorbing surface, Russian roulette or the bounce cap.  A photon is stored
// at every diffuse hit.  Record: (x, phi), (w, path << 5 | bounce).
// ---------------------------------------------------------------------------
// kRecord (adjoint replay): row n of mat_tab gets, per bounce, the material
// of a stored photon (0xff: no photon at that bounce; 0xfe: the path ended),
// and the matching entries of adj_tab are cleared for the adjoint gather.
template <bool kRecord>
__global__ __launch_bounds__(kBlock) void k_photon(SceneDev sc, uint64_t seed, uint32_t k, uint32_t n_paths,
                                                   float phi0, int32_t max_bounces, float4 *__restrict__ store,
                                                   uint32_t cap, uint32_t *__restrict__ counters,
                                                   uint8_t *__restrict__ mat_tab, double *__restrict__ adj_tab) {
    uint32_t n = pmd::xcd_block(blockIdx.x, gridDim.x) * kBlock + threadIdx.x;
    if (n >= n_paths) return;
    if (sc.n_emit == 0) {
        if (kRecord) mat_tab[(size_t)n * max_bounces] = 0xfeu;
        return;
    }
    pmd::Rng g = pmd::rng_seed(seed, pmd::kKindPhoton, k, (uint64_t)n);
    float u0 = pmd::rng_next(g);
    double target = (double)u0 * sc.power;
    // first emitter whose cumulative power exceeds the target
    int32_t lo = 0, hi = sc.n_emit - 1;
    while (lo < hi) {
        int32_t mid = (lo + hi) >> 1;
        if (target < sc.emit_cdf[mid]) hi = mid;
        else lo = mid + 1;
    }
    pmd::Tri et = pmd::load_tri(sc.bvh.tris, sc.emit_pos[lo]);
    float u1 = pmd::rng_next(g), u2 = pmd::rng_next(g);
    if (u1 + u2 > 1.0f) {
        u1 = 1.0f - u1;
        u2 = 1.0f - u2;
    }
    V3 org = pmd::v3((et.v0.x + u1 * et.e1.x) + u2 * et.e2.x, (et.v0.y + u1 * et.e1.y) + u2 * et.e2.y,
                     (et.v0.z + u1 * et.e1.z) + u2 * et.e2.z);
    V3 dir = pmd::cosine_dir(pmd::tri_normal(et), g);
    float phi = phi0;
    int32_t excl = et.id;
    pmd::TraceStats st;
    uint8_t *row = kRecord ? mat_tab + (size_t)n * max_bounces : nullptr;
    int last = -1;  // last bounce written to the row
    for (int b = 0; b < max_bounces; ++b) {
        float t;
        uint32_t kp;
        int32_t h = pmd::closest_hit<false>(sc.bvh, pmd::link_set(dir), org, dir, sc.eps, __builtin_inff(), excl, t,
                                            kp, st);
        if (h < 0) break;
        V3 x = pmd::vray(org, t, dir);
        pmd::Tri tr = pmd::load_tri(sc.bvh.tris, kp);
        V3 nrm = pmd::tri_normal(tr);
        uint32_t m = tr.mat;
        int type = sc.mat_type[m];
        if (kRecord) {
            row[b] = 0xffu;
            last = b;
        }
        if (type == PM_MAT_DIFFUSE) {
            float rho = sc.mat_rho[m];
            if (!(rho > 0.0f)) break;
            if (kRecord) {
                row[b] = (uint8_t)m;
                adj_tab[(size_t)n * max_bounces + b] = 0.0;
            }
            uint32_t slot = wave_append(&counters[0]);
            if (slot < cap) {
                store[2 * (size_t)slot] = make_float4(x.x, x.y, x.z, phi);
                store[2 * (size_t)slot + 1] = make_float4(dir.x, dir.y, dir.z, __uint_as_float((n << 5) | (uint32_t)b));
            } else {
                atomicOr(&counters[1], 1u);
            }
            float u = pmd::rng_next(g);
            float q = sc.mat_q[m];
            if (!(u < q)) break;
            phi = (phi * rho) / q;
            V3 ns = pmd::vdot(dir, nrm) < 0.0f ? nrm : pmd::vneg(nrm);
            dir = pmd::cosine_dir(ns, g);
        } else if (type == PM_MAT_MIRROR) {
            dir = pmd::reflect(dir, nrm);
        } else {
            dir = pmd::glass_dir(dir, nrm, sc.mat_ior[m], g);
        }
        org = x;
        excl = h;
    }
    if (kRecord && last + 1 < max_bounces) row[last + 1] = 0xfeu;
}

// ---------------------------------------------------------------------------
// Hashed grid (exact): cell edge h = 2 R_max (1 + 2^-10) so the 2x2x2 cells
// around a hit point cover its disc; cells hash (Teschner et al. 2003) into a
// power-of-two table; photons are counting-sorted by bucket.
// ---------------------------------------------------------------------------
struct Grid {
    float lo[3];
    float inv_h;
    uint32_t mask;
};

__device__ __forceinline__ uint32_t cell_hash(int32_t ix, int32_t iy, int32_t iz, uint32_t mask) {
    return (((uint32_t)ix * 73856093u) ^ ((uint32_t)iy * 19349663u) ^ ((uint32_t)iz * 83492791u)) & mask;
}

__device__ __forceinline__ Grid make_grid(const SceneDev &sc, const unsigned long long *r2max_bits, uint32_t mask) {
    double r2 = __longlong_as_double((long long)*r2max_bits);
    double h = 2.0 * sqrt(r2) * (1.0 + 1.0 / 1024.0);
    Grid gr;
    gr.lo[0] = sc.lo[0];
    gr.lo[1] = sc.lo[1];
    gr.lo[2] = sc.lo[2];
    gr.inv_h = h > 0.0 ? (float)(1.0 / h) : 0.0f;
    gr.mask = mask;
    return gr;
}

__device__ __forceinline__ uint32_t photon_bucket(const Grid &gr, float x, float y, float z) {
    int32_t ix = (int32_t)floorf((x - gr.lo[0]) * gr.inv_h);
    int32_t iy = (int32_t)floorf((y - gr.lo[1]) * gr.inv_h);
    int32_t iz = (int32_t)floorf((z - gr.lo[2]) * gr.inv_h);
    return cell_hash(ix, iy, iz, gr.mask);
}

// Frame setup: clear the photon counter and the R_max accumulator.
__global__ void k_begin(uint32_t *counters, unsigned long long *r2max_bits) {
    if (threadIdx.x == 0) {
        counters[0] = 0u;
        *r2max_bits = 0ull;
    }
}

__global__ __launch_bounds__(kBlock) void k_fill_u32(uint32_t *__restrict__ p, uint32_t n, uint32_t v) {
    uint32_t i = blockIdx.x * kBlock + threadIdx.x;
    if (i < n) p[i] = v;
}

// Largest squared radius among valid hit points (positive doubles order like
// their bit patterns).
__global__ __launch_bounds__(kBlock) void k_rmax(const float4 *__restrict__ hp_nrm, const double *__restrict__ R2,
                                                 int64_t P, unsigned long long *r2max_bits) {
    int64_t p = (int64_t)blockIdx.x * kBlock + threadIdx.x;
    unsigned long long v = 0ull;
    if (p < P && __float_as_int(hp_nrm[p].w) >= 0) v = (unsigned long long)__double_as_longlong(R2[p]);
    for (int off = 32; off > 0; off >>= 1) {
        unsigned long long o = __shfl_xor(v, off);
        v = o > v ? o : v;
    }
    if ((threadIdx.x & 63) == 0 && v) atomicMax(r2max_bits, v);
}

__global__ __launch_bounds__(kBlock) void k_count(const float4 *__restrict__ store, const uint32_t *__restrict__ counters,
                                                  uint32_t cap, SceneDev sc, const unsigned long long *r2max_bits,
                                                  uint32_t mask, uint32_t *__restrict__ cell_count) {
    uint32_t n_ph = min(counters[0], cap);
    Grid gr = make_grid(sc, r2max_bits, mask);
    for (uint32_t j = blockIdx.x * kBlock + threadIdx.x; j < n_ph; j += gridDim.x * kBlock) {
        float4 a = store[2 * (size_t)j];
        atomicAdd(&cell_count[photon_bucket(gr, a.x, a.y, a.z)], 1u);
    }
}

// Block-wide exclusive scan of one value per thread (4 waves of 64).
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

// Pass 1: per-tile exclusive scan into start[], tile totals into bsum[].
__global__ __launch_bounds__(kBlock) void k_scan_tiles(const uint32_t *__restrict__ in, uint32_t *__restrict__ out,
                                                       uint32_t *__restrict__ bsum) {
    __shared__ uint32_t lds[kBlock / 64];
    const uint32_t *src = in + (size_t)blockIdx.x * kScanTile + threadIdx.x * kScanItems;
    uint32_t vals[kScanItems];
    uint32_t s = 0;
#pragma unroll
    for (int i = 0; i < kScanItems; ++i) {
        vals[i] = src[i];
        s += vals[i];
    }
    uint32_t total;
    uint32_t ex = block_exscan(s, lds, total);
    uint32_t *dst = out + (size_t)blockIdx.x * kScanTile + threadIdx.x * kScanItems;
#pragma unroll
    for (int i = 0; i < kScanItems; ++i) {
        dst[i] = ex;
        ex += vals[i];
    }
    if (threadIdx.x == 0) bsum[blockIdx.x] = total;
}

// Pass 2: exclusive scan of up to kScanTile tile totals in one block.
__global__ __launch_bounds__(kBlock) void k_scan_sums(uint32_t *__restrict__ bsum, uint32_t nb) {
    __shared__ uint32_t lds[kBlock / 64];
    uint32_t vals[kScanItems];
    uint32_t s = 0;
#pragma unroll
    for (int i = 0; i < kScanItems; ++i) {
        uint32_t j = threadIdx.x * kScanItems + i;
        vals[i] = j < nb ? bsum[j] : 0u;
        s += vals[i];
    }
    uint32_t total;
    uint32_t ex = block_exscan(s, lds, total);
#pragma unroll
    for (int i = 0; i < kScanItems; ++i) {
        uint32_t j = threadIdx.x * kScanItems + i;
        if (j < nb) bsum[j] = ex;
        ex += vals[i];
    }
    if (threadIdx.x == 0) bsum[nb] = total;
}

// Pass 3: add tile offsets; write start[] and the scatter cursors fill[].
__global__ __launch_bounds__(kBlock) void k_scan_add(uint32_t *__restrict__ start, uint32_t *__restrict__ fill,
                                                     const uint32_t *__restrict__ bsum, uint32_t nb) {
    uint32_t off = bsum[blockIdx.x];
    size_t base = (size_t)blockIdx.x * kScanTile;
    for (int i = threadIdx.x; i < kScanTile; i += kBlock) {
        uint32_t v = start[base + i] + off;
        start[base + i] = v;
        fill[base + i] = v;
    }
    if (blockIdx.x == 0 && threadIdx.x == 0) start[(size_t)nb * kScanTile] = bsum[nb];
}

__global__ __launch_bounds__(kBlock) void k_scatter(const float4 *__restrict__ store, const uint32_t *__restrict__ counters,
                                                    uint32_t cap, SceneDev sc, const unsigned long long *r2max_bits,
                                                    uint32_t mask, uint32_t *__restrict__ fill,
                                                    float4 *__restrict__ sorted) {
    uint32_t n_ph = min(counters[0], cap);
    Grid gr = make_grid(sc, r2max_bits, mask);
    for (uint32_t j = blockIdx.x * kBlock + threadIdx.x; j < n_ph; j += gridDim.x * kBlock) {
        float4 a = store[2 * (size_t)j];
        float4 b = store[2 * (size_t)j + 1];
        uint32_t pos = atomicAdd(&fill[photon_bucket(gr, a.x, a.y, a.z)], 1u);
        sorted[2 * (size_t)pos] = a;
        sorted[2 * (size_t)pos + 1] = b;
    }
}

// ---------------------------------------------------------------------------
// Range query (exact): photons of the (deduplicated) buckets of the 8 cells
// around the hit point, accepted if squared distance < R^2 and arriving from
// the eye's side.  Flux terms are rounded one by one to 2^-shift fixed point
// and summed as integers, so the result does not depend on photon order.
// ---------------------------------------------------------------------------
__global__ __launch_bounds__(kBlock) void k_gather(const float4 *__restrict__ hp_pos, const float4 *__restrict__ hp_nrm,
                                                   const double *__restrict__ R2, int64_t P, SceneDev sc,
                                                   const unsigned long long *r2max_bits, uint32_t mask,
                                                   const uint32_t *__restrict__ start, const float4 *__restrict__ sorted,
                                                   double scale, uint32_t *__restrict__ M_out,
                                                   unsigned long long *__restrict__ Phi_out) {
    int64_t p = (int64_t)pmd::xcd_block(blockIdx.x, gridDim.x) * kBlock + threadIdx.x;
    if (p >= P) return;
    float4 hn = hp_nrm[p];
    uint32_t M = 0;
    unsigned long long F = 0ull;
    if (__float_as_int(hn.w) >= 0) {
        float4 hx = hp_pos[p];
        double r2 = R2[p];
        Grid gr = make_grid(sc, r2max_bits, mask);
        int32_t bx = (int32_t)floorf((hx.x - gr.lo[0]) * gr.inv_h - 0.5f);
        int32_t by = (int32_t)floorf((hx.y - gr.lo[1]) * gr.inv_h - 0.5f);
        int32_t bz = (int32_t)floorf((hx.z - gr.lo[2]) * gr.inv_h - 0.5f);
        uint32_t seen[8];
        double wk = (double)hx.w;
        for (int c = 0; c < 8; ++c) {
            uint32_t hb = cell_hash(bx + (c & 1), by + ((c >> 1) & 1), bz + (c >> 2), mask);
            bool dup = false;
            for (int e = 0; e < c; ++e) dup |= (seen[e] == hb);
            seen[c] = hb;
            if (dup) continue;
            uint32_t q0 = start[hb], q1 = start[hb + 1];
            for (uint32_t q = q0; q < q1; ++q) {
                float4 a = sorted[2 * (size_t)q];
                float dx = a.x - hx.x, dy = a.y - hx.y, dz = a.z - hx.z;
                float d2 = (dx * dx + dy * dy) + dz * dz;
                if ((double)d2 < r2) {
                    float4 b = sorted[2 * (size_t)q + 1];
                    float c2 = (b.x * hn.x + b.y * hn.y) + b.z * hn.z;
                    if (c2 < 0.0f) {
                        M++;
                        F += (unsigned long long)rint((wk * (double)a.w) * scale);
                    }
                }
            }
        }
    }
    M_out[p] = M;
    Phi_out[p] = F;
}

// Progressive update (radius reduction and flux rescaling of SPPM).
// hist (optional) receives the radius used in this iteration, for the adjoint.
__global__ __launch_bounds__(kBlock) void k_update(const float4 *__restrict__ hp_nrm, const uint32_t *__restrict__ M_in,
                                                   const unsigned long long *__restrict__ Phi_in, int64_t P,
                                                   double alpha, double inv_scale, double *__restrict__ N,
                                                   double *__restrict__ R2, double *__restrict__ tau,
                                                   double *__restrict__ hist) {
    int64_t p = (int64_t)blockIdx.x * kBlock + threadIdx.x;
    if (p >= P) return;
    if (hist) hist[p] = R2[p];
    uint32_t Mi = M_in[p];
    if (__float_as_int(hp_nrm[p].w) < 0 || Mi == 0) return;
    double m = (double)Mi;
    double n0 = N[p];
    double nn = n0 + alpha * m;
    double ratio = nn / (n0 + m);
    R2[p] = R2[p] * ratio;
    tau[p] = (tau[p] + (double)Phi_in[p] * inv_scale) * ratio;
    N[p] = nn;
}

// ---------------------------------------------------------------------------
// Adjoint (gradient of an image loss by replay).  With sampling held fixed the
// radiance of pixel p is sum_k sum_c c / (pi R2_{p,k} K) + D_p / K, each
// contribution c = W rho_h / pi * phi_j, where phi_j carries rho_m / q_m for
// every earlier diffuse bounce on m.  Per iteration the replayed gather adds
// G_h = g_h / (pi R2_{h,k} K) times c to the photon's (path, bounce) entry and
// the hit point's own albedo term G_h * sum c / rho_h; a per-path suffix sum
// then gives the earlier-bounce terms.  Material sums are reduced in LDS.
// ---------------------------------------------------------------------------
constexpr int kMaxAdjMat = 256;

__device__ __forceinline__ void lds_flush(double *lds, int n_mat, double *__restrict__ grad_mat) {
    __syncthreads();
    for (int m = threadIdx.x; m < n_mat; m += kBlock)
        if (lds[m] != 0.0) unsafeAtomicAdd(&grad_mat[m], lds[m]);
}

__global__ __launch_bounds__(kBlock) void k_gather_adj(const float4 *__restrict__ hp_pos, const float4 *__restrict__ hp_nrm,
                                                       const double *__restrict__ R2k, int64_t P, SceneDev sc,
                                                       const unsigned long long *r2max_bits, uint32_t mask,
                                                       const uint32_t *__restrict__ start,
                                                       const float4 *__restrict__ sorted, const float *__restrict__ g,
                                                       double K, int32_t max_bounces, double *__restrict__ adj_tab,
                                                       int32_t n_mat, double *__restrict__ grad_mat) {
    __shared__ double lds[kMaxAdjMat];
    for (int m = threadIdx.x; m < n_mat; m += kBlock) lds[m] = 0.0;
    __syncthreads();
    int64_t p = (int64_t)pmd::xcd_block(blockIdx.x, gridDim.x) * kBlock + threadIdx.x;
    float4 hn = p < P ? hp_nrm[p] : make_float4(0.0f, 0.0f, 0.0f, __int_as_float(-1));
    if (__float_as_int(hn.w) >= 0 && g[p] != 0.0f) {
        float4 hx = hp_pos[p];
        double r2 = R2k[p];
        double G = (double)g[p] / ((pmd::kPiD * r2) * K);
        Grid gr = make_grid(sc, r2max_bits, mask);
        int32_t bx = (int32_t)floorf((hx.x - gr.lo[0]) * gr.inv_h - 0.5f);
        int32_t by = (int32_t)floorf((hx.y - gr.lo[1]) * gr.inv_h - 0.5f);
        int32_t bz = (int32_t)floorf((hx.z - gr.lo[2]) * gr.inv_h - 0.5f);
        uint32_t seen[8];
        double wk = (double)hx.w, csum = 0.0;
        for (int c = 0; c < 8; ++c) {
            uint32_t hb = cell_hash(bx + (c & 1), by + ((c >> 1) & 1), bz + (c >> 2), mask);
            bool dup = false;
            for (int e = 0; e < c; ++e) dup |= (seen[e] == hb);
            seen[c] = hb;
            if (dup) continue;
            uint32_t q0 = start[hb], q1 = start[hb + 1];
            for (uint32_t q = q0; q < q1; ++q) {
                float4 a = sorted[2 * (size_t)q];
                float dx = a.x - hx.x, dy = a.y - hx.y, dz = a.z - hx.z;
                float d2 = (dx * dx + dy * dy) + dz * dz;
                if ((double)d2 < r2) {
                    float4 b = sorted[2 * (size_t)q + 1];
                    float c2 = (b.x * hn.x + b.y * hn.y) + b.z * hn.z;
                    if (c2 < 0.0f) {
                        double cc = wk * (double)a.w;
                        uint32_t meta = __float_as_uint(b.w);
                        unsafeAtomicAdd(&adj_tab[(size_t)(meta >> 5) * max_bounces + (meta & 31u)], G * cc);
                        csum += cc;
                    }
                }
            }
        }
        uint32_t m = __float_as_uint(hn.w);
        if (csum != 0.0) atomicAdd(&lds[m], G * csum / (double)sc.mat_rho[m]);
    }
    lds_flush(lds, n_mat, grad_mat);
}

__global__ __launch_bounds__(kBlock) void k_path_adj(const uint8_t *__restrict__ mat_tab,
                                                     const double *__restrict__ adj_tab, uint32_t n_paths,
                                                     int32_t max_bounces, const float *__restrict__ mat_rho,
                                                     int32_t n_mat, double *__restrict__ grad_mat) {
    __shared__ double lds[kMaxAdjMat];
    for (int m = threadIdx.x; m < n_mat; m += kBlock) lds[m] = 0.0;
    __syncthreads();
    uint32_t n = blockIdx.x * kBlock + threadIdx.x;
    if (n < n_paths) {
        const uint8_t *row = mat_tab + (size_t)n * max_bounces;
        const double *arow = adj_tab + (size_t)n * max_bounces;
        int end = 0;
        while (end < max_bounces && row[end] != 0xfeu) end++;
        double S = 0.0;  // sensitivity of the photons stored after bounce b
        for (int b = end - 1; b >= 0; --b) {
            uint32_t m = row[b];
            if (m == 0xffu) continue;
            if (S != 0.0) atomicAdd(&lds[m], S / (double)mat_rho[m]);
            S += arow[b];
        }
    }
    lds_flush(lds, n_mat, grad_mat);
}

// sum_p g_p L_p (every term of L_p is proportional to the emitted radiance)
__global__ __launch_bounds__(kBlock) void k_le_grad(const double *__restrict__ R2, const double *__restrict__ tau,
                                                    const double *__restrict__ D, int64_t P, double K,
                                                    const float *__restrict__ g, double *__restrict__ out) {
    __shared__ double lds[kBlock / 64];
    int64_t p = (int64_t)blockIdx.x * kBlock + threadIdx.x;
    double v = 0.0;
    if (p < P) v = (double)g[p] * (tau[p] / ((pmd::kPiD * R2[p]) * K) + D[p] / K);
    for (int off = 32; off > 0; off >>= 1) v += __shfl_xor(v, off);
    if ((threadIdx.x & 63) == 0) lds[threadIdx.x >> 6] = v;
    __syncthreads();
    if (threadIdx.x == 0) {
        double t = 0.0;
        for (int w = 0; w < kBlock / 64; ++w) t += lds[w];
        unsafeAtomicAdd(out, t);
    }
}

__global__ void k_fill_f64(double *p, int64_t n) {
    int64_t i = (int64_t)blockIdx.x * kBlock + threadIdx.x;
    if (i < n) p[i] = 0.0;
}

__global__ void k_collect_grad(const double *__restrict__ grad_mat, const int32_t *__restrict__ pmat, int32_t n_par,
                               const double *__restrict__ le_sum, double inv_Le, double *__restrict__ out) {
    int i = threadIdx.x;
    if (i < n_par) out[i] = grad_mat[pmat[i]];
    if (i == n_par) out[i] = *le_sum * inv_Le;
}

__global__ __launch_bounds__(kBlock) void k_resolve(const double *__restrict__ R2, const double *__restrict__ tau,
                                                    const double *__restrict__ D, int64_t P, int32_t K,
                                                    float *__restrict__ img) {
    int64_t p = (int64_t)blockIdx.x * kBlock + threadIdx.x;
    if (p >= P) return;
    double L = tau[p] / ((pmd::kPiD * R2[p]) * (double)K) + D[p] / (double)K;
    img[p] = (float)L;
}

__global__ __launch_bounds__(kBlock) void k_init_state(double *N, double *R2, double *tau, double *D, int64_t P,
                                                       double r0sq) {
    int64_t p = (int64_t)blockIdx.x * kBlock + threadIdx.x;
    if (p >= P) return;
    N[p] = 0.0;
    R2[p] = r0sq;
    tau[p] = 0.0;
    D[p] = 0.0;
}

inline uint32_t blocks_for(int64_t n) { return (uint32_t)((n + kBlock - 1) / kBlock); }

// host float3 helpers with the same evaluation order as the device
struct H3 {
    float x, y, z;
};
inline H3 hsub(H3 a, H3 b) { return {a.x - b.x, a.y - b.y, a.z - b.z}; }
inline float hdot(H3 a, H3 b) { return (a.x * b.x + a.y * b.y) + a.z * b.z; }
inline H3 hcross(H3 a, H3 b) { return {a.y * b.z - a.z * b.y, a.z * b.x - a.x * b.z, a.x * b.y - a.y * b.x}; }
inline H3 hnorm(H3 v) {
    float l = std::sqrt(hdot(v, v));
    return {v.x / l, v.y / l, v.z / l};
}

}  // namespace

struct pm_sppm {
    pm_sppm_params prm{};
    pm_bvh *bvh = nullptr;
    bool own_bvh = false;
    SceneDev sc{};
    int64_t P = 0;
    int32_t K = 0;
    uint32_t cap = 0;
    uint32_t table_bits = 0;
    float phi0 = 0.0f;
    // device buffers
    int32_t *mat_type = nullptr;
    float *mat_f = nullptr;  // rho | q | Le | ior, each n_mat
    uint32_t *emit_pos = nullptr;
    double *emit_cdf = nullptr;
    double *N = nullptr, *R2 = nullptr, *tau = nullptr, *D = nullptr;
    float4 *hp_pos = nullptr, *hp_nrm = nullptr;
    float4 *store = nullptr, *sorted = nullptr;
    uint32_t *counters = nullptr;  // [0] photons stored, [1] overflow flag
    unsigned long long *r2max = nullptr;
    uint32_t *cell_count = nullptr, *cell_start = nullptr, *cell_fill = nullptr, *bsum = nullptr;
    uint32_t *M = nullptr;
    unsigned long long *Phi = nullptr;
    // adjoint recording / replay buffers (record_iterations > 0)
    int32_t rec_iters = 0;
    int32_t n_mat = 0;
    double le_single = 0.0;  // Le of the single emitting material, 0 if not exactly one
    double *R2_hist = nullptr;    // [rec_iters][P] radius used in each iteration
    double *adj_tab = nullptr;    // [n_photons][max_bounces] photon sensitivities
    uint8_t *mat_tab = nullptr;   // [n_photons][max_bounces] stored-photon materials
    double *grad_mat = nullptr;   // [n_mat + 1]; last entry: sum g L
    int32_t *d_pmat = nullptr;    // [256] parameter materials
};

namespace pm {

static void sppm_free(pm_sppm *s) {
    // kernels of this handle may still be in flight on the caller's stream
    (void)hipDeviceSynchronize();
    void *bufs[] = {s->mat_type, s->mat_f, s->emit_pos, s->emit_cdf, s->N, s->R2, s->tau, s->D, s->hp_pos,
                    s->hp_nrm, s->store, s->sorted, s->counters, s->r2max, s->cell_count, s->cell_start,
                    s->cell_fill, s->bsum, s->M, s->Phi, s->R2_hist, s->adj_tab, s->mat_tab, s->grad_mat,
                    s->d_pmat};
    for (void *b : bufs)
        if (b) (void)hipFree(b);
    if (s->own_bvh && s->bvh) {
        free_bvh(s->bvh);
        delete s->bvh;
    }
    delete s;
}

int sppm_validate(const pm_scene_desc *d, const pm_sppm_params *p) {
    if (!d || !p) return set_error("scene and params must not be NULL"), PM_ERR_ARG;
    if (d->size < sizeof(pm_scene_desc) || p->size < sizeof(pm_sppm_params))
        return set_error("struct size field too small"), PM_ERR_ARG;
    if (!d->tri_verts || !d->tri_mat || d->n_tri < 1) return set_error("scene has no triangles"), PM_ERR_ARG;
    if (!d->mat_type || !d->mat_rho || !d->mat_q || !d->mat_Le || !d->mat_ior || d->n_mat < 1)
        return set_error("material arrays missing"), PM_ERR_ARG;
    for (int64_t i = 0; i < d->n_tri; ++i)
        if (d->tri_mat[i] >= (uint32_t)d->n_mat) return set_error("triangle material id out of range"), PM_ERR_ARG;
    for (int32_t m = 0; m < d->n_mat; ++m) {
        int t = d->mat_type[m];
        if (t < 0 || t > 2) return set_error("unknown material type"), PM_ERR_ARG;
        if (!(d->mat_rho[m] >= 0.0f && d->mat_rho[m] < 1.0f)) return set_error("albedo must be in [0,1)"), PM_ERR_ARG;
        if (!(d->mat_q[m] >= 0.0f && d->mat_q[m] <= 1.0f)) return set_error("RR probability must be in [0,1]"), PM_ERR_ARG;
        if (d->mat_rho[m] > 0.0f && !(d->mat_q[m] > 0.0f))
            return set_error("RR probability must be > 0 where albedo > 0"), PM_ERR_ARG;
        if (!(d->mat_Le[m] >= 0.0f) || !std::isfinite(d->mat_Le[m])) return set_error("Le must be finite and >= 0"), PM_ERR_ARG;
        if (t == PM_MAT_GLASS && !(d->mat_ior[m] > 0.0f)) return set_error("glass ior must be > 0"), PM_ERR_ARG;
    }
    if (d->width < 1 || d->height < 1 || (int64_t)d->width * d->height > (int64_t(1) << 28))
        return set_error("image size out of range"), PM_ERR_ARG;
    if (!(d->tan_half_fov > 0.0f) || !std::isfinite(d->tan_half_fov)) return set_error("tan_half_fov must be > 0"), PM_ERR_ARG;
    if (p->n_photons < 1 || p->n_photons > (int64_t(1) << 26)) return set_error("n_photons must be in [1, 2^26]"), PM_ERR_ARG;
    if (!(p->alpha > 0.0 && p->alpha <= 1.0)) return set_error("alpha must be in (0,1]"), PM_ERR_ARG;
    if (!(p->r0 > 0.0) || !std::isfinite(p->r0)) return set_error("r0 must be > 0"), PM_ERR_ARG;
    if (p->max_eye_depth < 1 || p->max_eye_depth > 64 || p->max_photon_bounces < 1 || p->max_photon_bounces > 32)
        return set_error("max_eye_depth must be in [1,64] and max_photon_bounces in [1,32]"), PM_ERR_ARG;
    if (p->fixed_shift < 0 || p->fixed_shift > 52) return set_error("fixed_shift must be in [0,52]"), PM_ERR_ARG;
    if (p->store_factor < 1 || p->n_photons * p->store_factor > (int64_t(1) << 30))
        return set_error("store_factor must be >= 1 and the store below 2^30 photons"), PM_ERR_ARG;
    if (d->bvh && d->bvh->n_tri != d->n_tri) return set_error("bvh was built over a different triangle count"), PM_ERR_ARG;
    if (p->record_iterations < 0 || p->record_iterations > 100000)
        return set_error("record_iterations must be in [0, 100000]"), PM_ERR_ARG;
    if (p->record_iterations > 0 && d->n_mat > kMaxAdjMat)
        return set_error("the adjoint supports at most 256 materials"), PM_ERR_ARG;
    return PM_OK;
}

int sppm_create(const pm_scene_desc *d, const pm_sppm_params *p, hipStream_t st, pm_sppm **out) {
    int rc = sppm_validate(d, p);
    if (rc) return rc;
    pm_sppm *s = new pm_sppm();
    s->prm = *p;
    auto fail = [&](int code) {
        sppm_free(s);
        return code;
    };
    if (d->bvh) {
        s->bvh = const_cast<pm_bvh *>(d->bvh);
    } else {
        HostBvh hb;
        std::string err;
        BuildOptions bo;
        if (!build_bvh_host(d->tri_verts, d->tri_mat, d->n_tri, bo, hb, err)) {
            set_error(err);
            return fail(PM_ERR_ARG);
        }
        s->bvh = new pm_bvh();
        s->own_bvh = true;
        if ((rc = upload_bvh(hb, st, s->bvh))) return fail(rc);
    }
    const pm_bvh *b = s->bvh;
    s->P = (int64_t)d->width * d->height;
    // emitters in original triangle order, by power = area * Le
    std::vector<uint32_t> epos;
    std::vector<double> ecdf;
    double acc = 0.0;
    for (int64_t i = 0; i < d->n_tri; ++i) {
        float Le = d->mat_Le[d->tri_mat[i]];
        if (!(Le > 0.0f)) continue;
        const float *v = d->tri_verts + 9 * i;
        H3 v0{v[0], v[1], v[2]}, v1{v[3], v[4], v[5]}, v2{v[6], v[7], v[8]};
        H3 c = hcross(hsub(v1, v0), hsub(v2, v0));
        float area = 0.5f * std::sqrt(hdot(c, c));
        acc += (double)area * (double)Le;
        epos.push_back((uint32_t)b->pos_of[i]);
        ecdf.push_back(acc);
    }
    // scene-size dependent constants
    H3 ext{b->hi[0] - b->lo[0], b->hi[1] - b->lo[1], b->hi[2] - b->lo[2]};
    float diag = std::sqrt(hdot(ext, ext));
    s->phi0 = (float)((pmd::kPiD * acc) / (double)p->n_photons);
    int64_t cap64 = p->n_photons * p->store_factor;
    s->cap = (uint32_t)cap64;
    uint32_t bits = 12;
    while (bits < 24 && (int64_t(1) << bits) < 4 * p->n_photons) bits++;
    s->table_bits = bits;
    const uint32_t T = 1u << bits;
    const uint32_t nb = T / kScanTile;
    const int32_t nm = d->n_mat;

    PM_HIP(hipMalloc(&s->mat_type, sizeof(int32_t) * nm));
    PM_HIP(hipMalloc(&s->mat_f, sizeof(float) * 4 * nm));
    PM_HIP(hipMalloc(&s->emit_pos, sizeof(uint32_t) * std::max<size_t>(1, epos.size())));
    PM_HIP(hipMalloc(&s->emit_cdf, sizeof(double) * std::max<size_t>(1, ecdf.size())));
    PM_HIP(hipMalloc(&s->N, sizeof(double) * s->P));
    PM_HIP(hipMalloc(&s->R2, sizeof(double) * s->P));
    PM_HIP(hipMalloc(&s->tau, sizeof(double) * s->P));
    PM_HIP(hipMalloc(&s->D, sizeof(double) * s->P));
    PM_HIP(hipMalloc(&s->hp_pos, sizeof(float4) * s->P));
    PM_HIP(hipMalloc(&s->hp_nrm, sizeof(float4) * s->P));
    PM_HIP(hipMalloc(&s->store, sizeof(float4) * 2 * (size_t)cap64));
    PM_HIP(hipMalloc(&s->sorted, sizeof(float4) * 2 * (size_t)cap64));
    PM_HIP(hipMalloc(&s->counters, sizeof(uint32_t) * 4));
    PM_HIP(hipMalloc(&s->r2max, sizeof(unsigned long long)));
    PM_HIP(hipMalloc(&s->cell_count, sizeof(uint32_t) * T));
    PM_HIP(hipMalloc(&s->cell_start, sizeof(uint32_t) * (T + 1)));
    PM_HIP(hipMalloc(&s->cell_fill, sizeof(uint32_t) * T));
    PM_HIP(hipMalloc(&s->bsum, sizeof(uint32_t) * (nb + 1)));
    PM_HIP(hipMalloc(&s->M, sizeof(uint32_t) * s->P));
    PM_HIP(hipMalloc(&s->Phi, sizeof(unsigned long long) * s->P));
    s->n_mat = nm;
    s->rec_iters = p->record_iterations;
    if (s->rec_iters > 0) {
        PM_HIP(hipMalloc(&s->R2_hist, sizeof(double) * (size_t)s->rec_iters * s->P));
        PM_HIP(hipMalloc(&s->adj_tab, sizeof(double) * (size_t)p->n_photons * p->max_photon_bounces));
        PM_HIP(hipMalloc(&s->mat_tab, (size_t)p->n_photons * p->max_photon_bounces));
        PM_HIP(hipMalloc(&s->grad_mat, sizeof(double) * (nm + 1)));
        PM_HIP(hipMalloc(&s->d_pmat, sizeof(int32_t) * kMaxAdjMat));
    }
    {
        int n_emit_mat = 0;
        double le = 0.0;
        for (int32_t m = 0; m < nm; ++m)
            if (d->mat_Le[m] > 0.0f) {
                n_emit_mat++;
                le = d->mat_Le[m];
            }
        s->le_single = n_emit_mat == 1 ? le : 0.0;
    }

    std::vector<float> mf(4 * (size_t)nm);
    for (int32_t m = 0; m < nm; ++m) {
        mf[m] = d->mat_rho[m];
        mf[nm + m] = d->mat_q[m];
        mf[2 * nm + m] = d->mat_Le[m];
        mf[3 * nm + m] = d->mat_ior[m];
    }
    PM_HIP(hipMemcpyAsync(s->mat_type, d->mat_type, sizeof(int32_t) * nm, hipMemcpyHostToDevice, st));
    PM_HIP(hipMemcpyAsync(s->mat_f, mf.data(), sizeof(float) * 4 * nm, hipMemcpyHostToDevice, st));
    if (!epos.empty()) {
        PM_HIP(hipMemcpyAsync(s->emit_pos, epos.data(), sizeof(uint32_t) * epos.size(), hipMemcpyHostToDevice, st));
        PM_HIP(hipMemcpyAsync(s->emit_cdf, ecdf.data(), sizeof(double) * ecdf.size(), hipMemcpyHostToDevice, st));
    }
    PM_HIP(hipMemsetAsync(s->counters, 0, sizeof(uint32_t) * 4, st));
    PM_HIP(hipMemsetAsync(s->hp_nrm, 0xff, sizeof(float4) * s->P, st));
    PM_HIP(hipMemsetAsync(s->M, 0, sizeof(uint32_t) * s->P, st));
    PM_HIP(hipMemsetAsync(s->Phi, 0, sizeof(unsigned long long) * s->P, st));
    PM_HIP(hipMemsetAsync(s->r2max, 0, sizeof(unsigned long long), st));
    hipLaunchKernelGGL(k_init_state, dim3(blocks_for(s->P)), dim3(kBlock), 0, st, s->N, s->R2, s->tau, s->D, s->P,
                       p->r0 * p->r0);
    PM_HIP(hipGetLastError());
    // host staging vectors go out of scope: finish the copies first
    PM_HIP(hipStreamSynchronize(st));

    SceneDev &sc = s->sc;
    sc.bvh = make_device_bvh(b);
    sc.mat_type = s->mat_type;
    sc.mat_rho = s->mat_f;
    sc.mat_q = s->mat_f + nm;
    sc.mat_Le = s->mat_f + 2 * nm;
    sc.mat_ior = s->mat_f + 3 * nm;
    sc.emit_pos = s->emit_pos;
    sc.emit_cdf = s->emit_cdf;
    sc.n_emit = (int32_t)epos.size();
    sc.power = acc;
    sc.eps = 1e-5f * diag;
    for (int a = 0; a < 3; ++a) sc.lo[a] = b->lo[a];
    H3 pos{d->cam_pos[0], d->cam_pos[1], d->cam_pos[2]};
    H3 look{d->cam_look[0], d->cam_look[1], d->cam_look[2]};
    H3 up{d->cam_up[0], d->cam_up[1], d->cam_up[2]};
    H3 f = hnorm(hsub(look, pos));
    H3 r = hnorm(hcross(f, up));
    H3 u = hcross(r, f);
    sc.cpos = pmd::V3{pos.x, pos.y, pos.z};
    sc.cf = pmd::V3{f.x, f.y, f.z};
    sc.cr = pmd::V3{r.x, r.y, r.z};
    sc.cu = pmd::V3{u.x, u.y, u.z};
    sc.tanh_fov = d->tan_half_fov;
    sc.aspect = (float)d->width / (float)d->height;
    sc.W = d->width;
    sc.H = d->height;
    *out = s;
    return PM_OK;
}

int sppm_destroy(pm_sppm *s) {
    if (!s) return set_error("NULL handle"), PM_ERR_ARG;
    sppm_free(s);
    return PM_OK;
}

int sppm_iterate(pm_sppm *s, int32_t n_iter, hipStream_t st) {
    if (!s || n_iter < 0) return set_error("invalid handle or iteration count"), PM_ERR_ARG;
    const uint32_t T = 1u << s->table_bits, mask = T - 1u, nb = T / kScanTile;
    const uint32_t np = (uint32_t)s->prm.n_photons;
    const double scale = std::ldexp(1.0, s->prm.fixed_shift), inv_scale = std::ldexp(1.0, -s->prm.fixed_shift);
    const uint32_t ph_blocks = std::min<uint32_t>(blocks_for(s->cap), 256u * 64u);
    for (int32_t it = 0; it < n_iter; ++it) {
        uint32_t k = (uint32_t)s->K;
        hipLaunchKernelGGL(k_eye, dim3(blocks_for(s->P)), dim3(kBlock), 0, st, s->sc, s->prm.seed, k,
                           s->prm.max_eye_depth, s->hp_pos, s->hp_nrm, s->D);
        hipLaunchKernelGGL(k_begin, dim3(1), dim3(64), 0, st, s->counters, s->r2max);
        hipLaunchKernelGGL(k_fill_u32, dim3(blocks_for(T)), dim3(kBlock), 0, st, s->cell_count, T, 0u);
        hipLaunchKernelGGL(k_photon<false>, dim3(blocks_for(np)), dim3(kBlock), 0, st, s->sc, s->prm.seed, k, np,
                           s->phi0, s->prm.max_photon_bounces, s->store, s->cap, s->counters, nullptr, nullptr);
        hipLaunchKernelGGL(k_rmax, dim3(blocks_for(s->P)), dim3(kBlock), 0, st, s->hp_nrm, s->R2, s->P, s->r2max);
        hipLaunchKernelGGL(k_count, dim3(ph_blocks), dim3(kBlock), 0, st, s->store, s->counters, s->cap, s->sc,
                           s->r2max, mask, s->cell_count);
        hipLaunchKernelGGL(k_scan_tiles, dim3(nb), dim3(kBlock), 0, st, s->cell_count, s->cell_start, s->bsum);
        hipLaunchKernelGGL(k_scan_sums, dim3(1), dim3(kBlock), 0, st, s->bsum, nb);
        hipLaunchKernelGGL(k_scan_add, dim3(nb), dim3(kBlock), 0, st, s->cell_start, s->cell_fill, s->bsum, nb);
        hipLaunchKernelGGL(k_scatter, dim3(ph_blocks), dim3(kBlock), 0, st, s->store, s->counters, s->cap, s->sc,
                           s->r2max, mask, s->cell_fill, s->sorted);
        hipLaunchKernelGGL(k_gather, dim3(blocks_for(s->P)), dim3(kBlock), 0, st, s->hp_pos, s->hp_nrm, s->R2, s->P,
                           s->sc, s->r2max, mask, s->cell_start, s->sorted, scale, s->M, s->Phi);
        double *hist = (int32_t)k < s->rec_iters ? s->R2_hist + (size_t)k * s->P : nullptr;
        hipLaunchKernelGGL(k_update, dim3(blocks_for(s->P)), dim3(kBlock), 0, st, s->hp_nrm, s->M, s->Phi, s->P,
                           s->prm.alpha, inv_scale, s->N, s->R2, s->tau, hist);
        PM_HIP(hipGetLastError());
        s->K++;
    }
    return PM_OK;
}

int sppm_resolve(pm_sppm *s, float *image, hipStream_t st) {
    if (!s || !image) return set_error("invalid handle or image pointer"), PM_ERR_ARG;
    if (s->K == 0) return set_error("no iteration has run"), PM_ERR_STATE;
    hipLaunchKernelGGL(k_resolve, dim3(blocks_for(s->P)), dim3(kBlock), 0, st, s->R2, s->tau, s->D, s->P, s->K, image);
    PM_HIP(hipGetLastError());
    return PM_OK;
}

int sppm_status(pm_sppm *s, hipStream_t st) {
    if (!s) return set_error("NULL handle"), PM_ERR_ARG;
    uint32_t c[4];
    PM_HIP(hipMemcpyAsync(c, s->counters, sizeof(c), hipMemcpyDeviceToHost, st));
    PM_HIP(hipStreamSynchronize(st));
    if (c[1]) return set_error("photon store overflow: raise store_factor"), PM_ERR_OVERFLOW;
    return PM_OK;
}

int sppm_adjoint(pm_sppm *s, const float *g, const int32_t *pmat, int32_t n_par, double *grad, hipStream_t st) {
    if (!s || !g || !grad || n_par < 0 || (n_par > 0 && !pmat))
        return set_error("invalid handle, gradient or parameter pointers"), PM_ERR_ARG;
    if (s->K < 1) return set_error("no iteration has run"), PM_ERR_STATE;
    if (s->K > s->rec_iters)
        return set_error("the forward iterations were not recorded: set record_iterations >= K"), PM_ERR_STATE;
    if (n_par >= kMaxAdjMat) return set_error("too many parameters"), PM_ERR_ARG;
    std::vector<float> rho(s->n_mat);
    PM_HIP(hipMemcpy(rho.data(), s->mat_f, sizeof(float) * s->n_mat, hipMemcpyDeviceToHost));
    for (int32_t i = 0; i < n_par; ++i) {
        if (pmat[i] < 0 || pmat[i] >= s->n_mat) return set_error("parameter material out of range"), PM_ERR_ARG;
        if (!(rho[pmat[i]] > 0.0f)) return set_error("albedo parameters must have rho > 0"), PM_ERR_ARG;
    }
    const uint32_t T = 1u << s->table_bits, mask = T - 1u, nb = T / kScanTile;
    const uint32_t np = (uint32_t)s->prm.n_photons;
    const int32_t mb = s->prm.max_photon_bounces;
    const uint32_t ph_blocks = std::min<uint32_t>(blocks_for(s->cap), 256u * 64u);
    const double K = (double)s->K;
    PM_HIP(hipMemcpyAsync(s->d_pmat, pmat, sizeof(int32_t) * std::max(1, n_par), hipMemcpyHostToDevice, st));
    hipLaunchKernelGGL(k_fill_f64, dim3(blocks_for(s->n_mat + 1)), dim3(kBlock), 0, st, s->grad_mat,
                       (int64_t)s->n_mat + 1);
    for (int32_t k = 0; k < s->K; ++k) {
        const double *R2k = s->R2_hist + (size_t)k * s->P;
        hipLaunchKernelGGL(k_eye, dim3(blocks_for(s->P)), dim3(kBlock), 0, st, s->sc, s->prm.seed, (uint32_t)k,
                           s->prm.max_eye_depth, s->hp_pos, s->hp_nrm, (double *)nullptr);
        hipLaunchKernelGGL(k_begin, dim3(1), dim3(64), 0, st, s->counters, s->r2max);
        hipLaunchKernelGGL(k_fill_u32, dim3(blocks_for(T)), dim3(kBlock), 0, st, s->cell_count, T, 0u);
        hipLaunchKernelGGL(k_photon<true>, dim3(blocks_for(np)), dim3(kBlock), 0, st, s->sc, s->prm.seed,
                           (uint32_t)k, np, s->phi0, mb, s->store, s->cap, s->counters, s->mat_tab, s->adj_tab);
        hipLaunchKernelGGL(k_rmax, dim3(blocks_for(s->P)), dim3(kBlock), 0, st, s->hp_nrm, R2k, s->P, s->r2max);
        hipLaunchKernelGGL(k_count, dim3(ph_blocks), dim3(kBlock), 0, st, s->store, s->counters, s->cap, s->sc,
                           s->r2max, mask, s->cell_count);
        hipLaunchKernelGGL(k_scan_tiles, dim3(nb), dim3(kBlock), 0, st, s->cell_count, s->cell_start, s->bsum);
        hipLaunchKernelGGL(k_scan_sums, dim3(1), dim3(kBlock), 0, st, s->bsum, nb);
        hipLaunchKernelGGL(k_scan_add, dim3(nb), dim3(kBlock), 0, st, s->cell_start, s->cell_fill, s->bsum, nb);
        hipLaunchKernelGGL(k_scatter, dim3(ph_blocks), dim3(kBlock), 0, st, s->store, s->counters, s->cap, s->sc,
                           s->r2max, mask, s->cell_fill, s->sorted);
        hipLaunchKernelGGL(k_gather_adj, dim3(blocks_for(s->P)), dim3(kBlock), 0, st, s->hp_pos, s->hp_nrm, R2k, s->P,
                           s->sc, s->r2max, mask, s->cell_start, s->sorted, g, K, mb, s->adj_tab, s->n_mat,
                           s->grad_mat);
        hipLaunchKernelGGL(k_path_adj, dim3(blocks_for(np)), dim3(kBlock), 0, st, s->mat_tab, s->adj_tab, np, mb,
                           s->sc.mat_rho, s->n_mat, s->grad_mat);
        PM_HIP(hipGetLastError());
    }
    hipLaunchKernelGGL(k_le_grad, dim3(blocks_for(s->P)), dim3(kBlock), 0, st, s->R2, s->tau, s->D, s->P, K, g,
                       s->grad_mat + s->n_mat);
    hipLaunchKernelGGL(k_collect_grad, dim3(1), dim3(kMaxAdjMat), 0, st, s->grad_mat, s->d_pmat, n_par,
                       s->grad_mat + s->n_mat, s->le_single > 0.0 ? 1.0 / s->le_single : 0.0, grad);
    PM_HIP(hipGetLastError());
    return PM_OK;
}

int sppm_views(pm_sppm *s, pm_sppm_views *v) {
    if (!s || !v || v->size < sizeof(pm_sppm_views)) return set_error("invalid handle or views struct"), PM_ERR_ARG;
    v->n_pixels = s->P;
    v->iterations = s->K;
    v->photon_capacity = s->cap;
    v->table_size = int64_t(1) << s->table_bits;
    v->N = s->N;
    v->R2 = s->R2;
    v->tau = s->tau;
    v->D = s->D;
    v->hp_pos = (float *)s->hp_pos;
    v->hp_nrm = (float *)s->hp_nrm;
    v->photons = (float *)s->store;
    v->photon_count = s->counters;
    v->gather_M = s->M;
    v->gather_Phi = (uint64_t *)s->Phi;
    return PM_OK;
}

}  // namespace pm
