// Stochastic progressive photon mapping on the device (Sec. 2): single-scene
// kernels (eye pass, photon pass, hashed-grid build, range query, progressive
// update, resolve, adjoint replay) and their host driver.
#include <algorithm>
#include <cmath>
#include <cstring>
#include <vector>

#include "runtime.h"
#include "sppm.h"
#include "sppm_dev.h"
#include "sppm_host.h"
#include "sppm_scan.h"

namespace {

using namespace pmd;

__global__ __launch_bounds__(kBlock) void k_eye(SppmDev d, uint32_t k, int32_t accumulate_D) {
    int64_t p = (int64_t)xcd_block(blockIdx.x, gridDim.x) * kBlock + threadIdx.x;
    if (p < d.P) eye_elem(d, k, p, accumulate_D != 0);
}

// The statistics variants (PM_PROFILE_COUNT): the same work, plus counts of
// paths, rays, box and triangle tests, and of the range query's buckets and
// photons, added to d.stats once per wavefront.
__global__ __launch_bounds__(kBlock) void k_eye_stats(SppmDev d, uint32_t k, int32_t accumulate_D) {
    int64_t p = (int64_t)xcd_block(blockIdx.x, gridDim.x) * kBlock + threadIdx.x;
    LaneStats ls;
    if (p < d.P) eye_elem<true>(d, k, p, accumulate_D != 0, &ls);
    wave_stats_flush(d.stats + kStatEyePaths, ls);
}

template <bool kRecord>
__global__ __launch_bounds__(kBlock) void k_photon(SppmDev d, uint32_t k, uint16_t *__restrict__ mat_tab,
                                                   long long *__restrict__ adj_tab) {
    uint32_t n = xcd_block(blockIdx.x, gridDim.x) * kBlock + threadIdx.x;
    if (n < d.n_paths) photon_elem<kRecord>(d, k, n, mat_tab, adj_tab);
}

// Persistent photon lanes with path regeneration.
__global__ __launch_bounds__(kBlock) void k_photon_regen(SppmDev d, uint32_t k) { photon_regen_loop(d, k, d.refill); }

__global__ __launch_bounds__(kBlock) void k_photon_regen_stats(SppmDev d, uint32_t k) {
    photon_regen_loop<false, true>(d, k, d.refill);
}

// Two-phase photon pass (PM_PHOTON_TWO_PHASE): regeneration that sets the
// last paths of each wavefront aside once the path counter has run out, then
// regeneration over the paths set aside.
template <bool kStats>
__global__ __launch_bounds__(kBlock) void k_photon_head(SppmDev d, uint32_t k, PathQueue q) {
    photon_regen_loop<false, kStats, true, false>(d, k, d.refill, nullptr, nullptr, q);
}

template <bool kStats>
__global__ __launch_bounds__(kBlock) void k_photon_tail(SppmDev d, uint32_t k, PathQueue q) {
    photon_regen_loop<false, kStats, false, true>(d, k, d.refill, nullptr, nullptr, q);
}

// The same two launches, recording each path's stored-photon materials for
// the adjoint (a queued path keeps its row of the tables).
__global__ __launch_bounds__(kBlock) void k_photon_head_rec(SppmDev d, uint32_t k, PathQueue q,
                                                            uint16_t *__restrict__ mat_tab,
                                                            long long *__restrict__ adj_tab) {
    photon_regen_loop<true, false, true, false>(d, k, d.refill, mat_tab, adj_tab, q);
}

__global__ __launch_bounds__(kBlock) void k_photon_tail_rec(SppmDev d, uint32_t k, PathQueue q,
                                                            uint16_t *__restrict__ mat_tab,
                                                            long long *__restrict__ adj_tab) {
    photon_regen_loop<true, false, false, true>(d, k, d.refill, mat_tab, adj_tab, q);
}

// Regeneration from a queue of started paths in LDS (PM_PHOTON_POOL): each
// wavefront owns kPoolWords x kPoolSlots words of the workgroup's LDS.
template <bool kStats>
__global__ __launch_bounds__(kBlock) __attribute__((amdgpu_waves_per_eu(5))) void k_photon_pool(SppmDev d, uint32_t k) {
    __shared__ uint32_t pool[kBlock / 64][kPoolWords * kPoolSlots];
    photon_pool_loop<kStats>(d, k, pool[threadIdx.x >> 6]);
}

// Regeneration at ray granularity (PM_PHOTON_RAY_REGEN).
__global__ __launch_bounds__(kBlock) void k_photon_stream(SppmDev d, uint32_t k) {
    photon_stream_loop(d, k, d.refill);
}

__global__ __launch_bounds__(kBlock) void k_photon_stream_stats(SppmDev d, uint32_t k) {
    photon_stream_loop<true>(d, k, d.refill);
}

// The same, recording each path's stored-photon materials for the adjoint.
__global__ __launch_bounds__(kBlock) void k_photon_regen_rec(SppmDev d, uint32_t k, uint16_t *__restrict__ mat_tab,
                                                             long long *__restrict__ adj_tab) {
    photon_regen_loop<true>(d, k, d.refill, mat_tab, adj_tab);
}

// One pass of the one-bounce-per-pass schedule; the grid covers the slots
// with the same workgroup-to-slot map in every pass.
__global__ __launch_bounds__(kBlock) void k_photon_pass(SppmDev d, uint32_t k, PassSlots ps) {
    photon_pass_elem(d, k, ps, xcd_block(blockIdx.x, gridDim.x) * kBlock + threadIdx.x);
}

// Paths no pass started, before the drain adds the paths still in flight.
__global__ void k_pass_tally(SppmDev d) {
    if (threadIdx.x == 0) d.counters[3] = d.n_paths - min(d.counters[2], d.n_paths);
}

__global__ __launch_bounds__(kBlock) void k_photon_drain(SppmDev d, uint32_t k, PassSlots ps) {
    photon_drain_elem(d, k, ps, xcd_block(blockIdx.x, gridDim.x) * kBlock + threadIdx.x);
}

// Start of a photon pass: clear its store's photon count and the path counter.
__global__ void k_photon_begin(SppmDev d) {
    if (threadIdx.x == 0) {
        d.counters[0] = 0u;
        d.counters[2] = 0u;
    }
}

// Start of an eye pass: clear the R_max accumulator.
__global__ void k_rmax_clear(SppmDev d) {
    if (threadIdx.x == 0) *d.r2max = 0ull;
}

// Frame setup: clear the photon and path counters and the R_max accumulator.
__global__ void k_begin(SppmDev d) {
    if (threadIdx.x == 0) {
        d.counters[0] = 0u;
        d.counters[2] = 0u;
        *d.r2max = 0ull;
    }
}

// Largest R^2 over valid hit points: a grid-stride maximum per lane, reduced
// across the workgroup, then one atomic per workgroup (positive doubles order
// like their bit patterns).  Launched with few workgroups so the atomics on
// the single result do not serialise.
constexpr uint32_t kRmaxBlocks = 512;

__global__ __launch_bounds__(kBlock) void k_rmax(SppmDev d, const double *__restrict__ R2src) {
    __shared__ unsigned long long part[kBlock / 64];
    unsigned long long v = 0ull;
    for (int64_t p = (int64_t)blockIdx.x * kBlock + threadIdx.x; p < d.P; p += (int64_t)gridDim.x * kBlock) {
        unsigned long long x = rmax_lane(d, R2src, p);
        v = x > v ? x : v;
    }
    for (int off = 32; off > 0; off >>= 1) {
        unsigned long long o = __shfl_xor(v, off);
        v = o > v ? o : v;
    }
    if ((threadIdx.x & 63) == 0) part[threadIdx.x >> 6] = v;
    __syncthreads();
    if (threadIdx.x == 0) {
        for (int w = 1; w < kBlock / 64; ++w) v = part[w] > v ? part[w] : v;
        if (v) atomicMax(d.r2max, v);
    }
}

__global__ __launch_bounds__(kBlock) void k_count(SppmDev d, uint32_t *__restrict__ cell_count) {
    uint32_t n_ph = stored_photons(d);
    Grid gr = make_grid(d);
    for (uint32_t j = blockIdx.x * kBlock + threadIdx.x; j < n_ph; j += gridDim.x * kBlock) count_elem(d, gr, j, cell_count);
}

__global__ __launch_bounds__(kBlock) void k_scatter(SppmDev d, const uint32_t *__restrict__ start,
                                                    float4 *__restrict__ sorted) {
    uint32_t n_ph = stored_photons(d);
    for (uint32_t j = blockIdx.x * kBlock + threadIdx.x; j < n_ph; j += gridDim.x * kBlock)
        scatter_elem(d, j, start, sorted);
}

__global__ __launch_bounds__(kBlock) void k_gather(SppmDev d, const uint32_t *__restrict__ start,
                                                   const float4 *__restrict__ sorted) {
    // every lane takes part (the wave may scan a dense hit point together)
    const int64_t p = (int64_t)xcd_block(blockIdx.x, gridDim.x) * kBlock + threadIdx.x;
    Grid gr = make_grid(d);
    gather_wave(d, gr, p, start, sorted);
}

__global__ __launch_bounds__(kBlock) void k_gather_stats(SppmDev d, const uint32_t *__restrict__ start,
                                                         const float4 *__restrict__ sorted) {
    const int64_t p = (int64_t)xcd_block(blockIdx.x, gridDim.x) * kBlock + threadIdx.x;
    Grid gr = make_grid(d);
    gather_wave<true>(d, gr, p, start, sorted);
}

// Stochastic spatial hashing: clear the keys, insert every stored photon
// (count and smallest key per entry), record each entry's survivor, gather.
__global__ __launch_bounds__(kBlock) void k_sh_clear(SppmDev d, uint32_t T) {
    for (uint32_t e = blockIdx.x * kBlock + threadIdx.x; e < T; e += gridDim.x * kBlock)
        d.sh_key[d.table_off + e] = ~0ull;
}

__global__ __launch_bounds__(kBlock) void k_sh_insert(SppmDev d, uint32_t k, uint32_t *__restrict__ count) {
    uint32_t n_ph = stored_photons(d);
    Grid gr = make_grid(d);
    for (uint32_t j = blockIdx.x * kBlock + threadIdx.x; j < n_ph; j += gridDim.x * kBlock)
        sh_insert_elem(d, gr, k, j, count);
}

__global__ __launch_bounds__(kBlock) void k_sh_pick(SppmDev d, uint32_t k) {
    uint32_t n_ph = stored_photons(d);
    Grid gr = make_grid(d);
    for (uint32_t j = blockIdx.x * kBlock + threadIdx.x; j < n_ph; j += gridDim.x * kBlock) sh_pick_elem(d, gr, k, j);
}

__global__ __launch_bounds__(kBlock) void k_sh_gather(SppmDev d, const uint32_t *__restrict__ count) {
    int64_t p = (int64_t)xcd_block(blockIdx.x, gridDim.x) * kBlock + threadIdx.x;
    if (p >= d.P) return;
    Grid gr = make_grid(d);
    sh_gather_elem(d, gr, p, count);
}

__global__ __launch_bounds__(kBlock) void k_update(SppmDev d, double *__restrict__ hist) {
    int64_t p = (int64_t)blockIdx.x * kBlock + threadIdx.x;
    if (p < d.P) update_elem(d, p, hist);
}

__global__ __launch_bounds__(kBlock) void k_resolve(SppmDev d, int32_t K, float *__restrict__ img) {
    int64_t p = (int64_t)blockIdx.x * kBlock + threadIdx.x;
    if (p < d.P) img[p] = resolve_elem(d, p, K);
}

__global__ __launch_bounds__(kBlock) void k_init_state(SppmDev d, double r0sq) {
    int64_t p = (int64_t)blockIdx.x * kBlock + threadIdx.x;
    if (p >= d.P) return;
    d.N[p] = 0.0;
    d.R2[p] = r0sq;
    d.tau[p] = 0.0;
    d.D[p] = 0.0;
}

// ---------------------------------------------------------------------------
// Adjoint (gradient of an image loss by replay).  With sampling held fixed the
// radiance of pixel p is sum_k sum_c c / (pi R2_{p,k} K) + D_p / K, each
// contribution c = W rho_h / pi * phi_j, where phi_j carries rho_m / q_m for
// every earlier diffuse bounce on m.  Per iteration the replayed gather adds
// G_h = g_h / (pi R2_{h,k} K) times c to the photon's (path, bounce) entry and
// to the hit point's own material; a per-path suffix sum then gives the
// earlier-bounce terms.  Dividing by rho_m is left to the end of the iteration.
//
// Every sum is an integer sum, so the gradient does not depend on the order of
// the atomics or of the photons in their buckets.  Each term G_h c is rounded
// on its own to a fixed point whose scale is a power of two chosen per
// iteration from two maxima (of |G_h| wk_h over hit points, of the flux over
// stored photons), so that no term exceeds 2^39 units.  A (path, bounce) entry
// is a signed 64-bit sum (fewer than 2^24 hit points reach one photon); the
// per-material sums are 96-bit (two 64-bit words: the low 32 bits of each
// addend, and the rest), and each iteration's are converted to double once
// and added to the gradient in iteration order.
// ---------------------------------------------------------------------------
constexpr int kAdjTermBits = 39;

using i128 = __int128;

__device__ __forceinline__ void wide_add(unsigned long long *lo, unsigned long long *hi, i128 v) {
    atomicAdd(lo, (unsigned long long)(uint32_t)(uint64_t)v);
    atomicAdd(hi, (unsigned long long)(long long)(v >> 32));
}

// Per-material 96-bit sums: accumulate in LDS, then add each workgroup's sums
// to the global pair with the carry of the low word moved into the high one.
struct WideLds {
    unsigned long long lo[kMaxAdjMat], hi[kMaxAdjMat];
};

__device__ __forceinline__ void wide_clear(WideLds &w, int n_mat) {
    for (int m = threadIdx.x; m < n_mat; m += kBlock) {
        w.lo[m] = 0ull;
        w.hi[m] = 0ull;
    }
    __syncthreads();
}

__device__ __forceinline__ void wide_flush(WideLds &w, int n_mat, unsigned long long *__restrict__ glob) {
    __syncthreads();
    for (int m = threadIdx.x; m < n_mat; m += kBlock) {
        const unsigned long long lo = w.lo[m], hi = w.hi[m];
        if (lo | hi) {
            atomicAdd(&glob[m], lo & 0xffffffffull);
            atomicAdd(&glob[n_mat + m], hi + (lo >> 32));
        }
    }
}

__device__ __forceinline__ double adj_G(const float *__restrict__ g, int64_t p, double r2, double K) {
    return (double)g[p] / ((kPiD * r2) * K);
}

// Clears the iteration's maxima and per-material sums.
__global__ void k_adj_begin(unsigned long long *__restrict__ adj_max, unsigned long long *__restrict__ wide,
                            int32_t n_mat) {
    for (int i = threadIdx.x; i < 2 * n_mat; i += blockDim.x) wide[i] = 0ull;
    if (threadIdx.x < 2) adj_max[threadIdx.x] = 0ull;
}

// Maximum of v over the workgroup (non-negative doubles compare as their bit
// patterns): one atomic per workgroup.
__device__ __forceinline__ void block_max_atomic(unsigned long long v, unsigned long long *__restrict__ out) {
    __shared__ unsigned long long wave_max[kBlock / 64];
    for (int off = 32; off > 0; off >>= 1) {
        unsigned long long o = __shfl_xor(v, off);
        v = o > v ? o : v;
    }
    if ((threadIdx.x & 63) == 0) wave_max[threadIdx.x >> 6] = v;
    __syncthreads();
    if (threadIdx.x == 0) {
        for (int w = 1; w < kBlock / 64; ++w) v = wave_max[w] > v ? wave_max[w] : v;
        if (v) atomicMax(out, v);
    }
}

// Workgroups of the two maxima below: a grid-stride loop each, so that at
// most this many same-address atomics are issued.
constexpr uint32_t kAdjMaxBlocks = 256;

// max over valid hit points of |G_h| wk_h (non-negative doubles order like
// their bit patterns, so the maximum is an integer maximum)
__global__ __launch_bounds__(kBlock) void k_adj_gmax(SppmDev d, const double *__restrict__ R2k,
                                                     const float *__restrict__ g, double K,
                                                     unsigned long long *__restrict__ adj_max) {
    unsigned long long v = 0ull;
    for (int64_t p = (int64_t)blockIdx.x * kBlock + threadIdx.x; p < d.P; p += (int64_t)gridDim.x * kBlock) {
        float4 hn = d.hp_nrm[p];
        if (__float_as_int(hn.w) >= 0) {
            double a = fabs(adj_G(g, p, R2k[p], K)) * (double)d.hp_pos[p].w;
            unsigned long long b = (unsigned long long)__double_as_longlong(a);
            v = b > v ? b : v;
        }
    }
    block_max_atomic(v, &adj_max[0]);
}

// max flux over the stored photons
__global__ __launch_bounds__(kBlock) void k_adj_phimax(SppmDev d, unsigned long long *__restrict__ adj_max) {
    const uint32_t n = min(d.counters[0], d.cap);
    unsigned long long v = 0ull;
    for (uint32_t i = blockIdx.x * kBlock + threadIdx.x; i < n; i += gridDim.x * kBlock) {
        unsigned long long b = (unsigned long long)__double_as_longlong((double)d.store[2 * (size_t)i].w);
        v = b > v ? b : v;
    }
    block_max_atomic(v, &adj_max[1]);
}

// Scale 2^(39 - e) with 2^e above the product of the two maxima, so
// |G_h wk_h phi_j| * scale < 2^39 for every pair (0: nothing to add).
__global__ void k_adj_scale(const unsigned long long *__restrict__ adj_max, double *__restrict__ scale) {
    if (threadIdx.x == 0) {
        const double bound = __longlong_as_double((long long)adj_max[0]) * __longlong_as_double((long long)adj_max[1]);
        double sc = 0.0;
        if (bound > 0.0 && bound < 1e300) {
            int e;
            (void)frexp(bound, &e);  // bound < 2^e
            sc = ldexp(1.0, kAdjTermBits - e);
        }
        *scale = sc;
    }
}

__global__ __launch_bounds__(kBlock) void k_gather_adj(SppmDev d, const double *__restrict__ R2k,
                                                       const uint32_t *__restrict__ start,
                                                       const float4 *__restrict__ sorted, const float *__restrict__ g,
                                                       double K, const double *__restrict__ scale_p,
                                                       long long *__restrict__ adj_tab, int32_t n_mat,
                                                       unsigned long long *__restrict__ wide) {
    __shared__ WideLds lds;
    wide_clear(lds, n_mat);
    const double scale = *scale_p;
    int64_t p = (int64_t)xcd_block(blockIdx.x, gridDim.x) * kBlock + threadIdx.x;
    float4 hn = p < d.P ? d.hp_nrm[p] : make_float4(0.0f, 0.0f, 0.0f, __int_as_float(-1));
    if (__float_as_int(hn.w) >= 0 && g[p] != 0.0f && scale > 0.0) {
        float4 hx = d.hp_pos[p];
        double r2 = R2k[p];
        double G = adj_G(g, p, r2, K);
        Grid gr = make_grid(d);
        double wk = (double)hx.w;
        i128 own = 0;
        const int32_t mb = d.max_bounces;
        for_each_photon_in_disc(d, gr, hx, hn, r2, start, sorted, [&](const float4 &a, const float4 &b) {
            double cc = wk * (double)a.w;
            long long q = __double2ll_rn((G * cc) * scale);
            uint32_t meta = __float_as_uint(b.w);
            if (q) atomicAdd((unsigned long long *)&adj_tab[(size_t)(meta >> 5) * mb + (meta & 31u)],
                             (unsigned long long)q);
            own += q;
        });
        if (own != 0) wide_add(&lds.lo[__float_as_uint(hn.w)], &lds.hi[__float_as_uint(hn.w)], own);
    }
    wide_flush(lds, n_mat, wide);
}

__global__ __launch_bounds__(kBlock) void k_path_adj(const uint16_t *__restrict__ mat_tab,
                                                     const long long *__restrict__ adj_tab, uint32_t n_paths,
                                                     int32_t max_bounces, int32_t n_mat,
                                                     unsigned long long *__restrict__ wide) {
    __shared__ WideLds lds;
    wide_clear(lds, n_mat);
    uint32_t n = blockIdx.x * kBlock + threadIdx.x;
    if (n < n_paths) {
        const uint16_t *row = mat_tab + (size_t)n * max_bounces;
        const long long *arow = adj_tab + (size_t)n * max_bounces;
        int end = 0;
        while (end < max_bounces && row[end] != kMatEnd) end++;
        i128 S = 0;  // sensitivity of the photons stored after bounce b
        for (int b = end - 1; b >= 0; --b) {
            uint32_t m = row[b];
            if (m == kMatNone) continue;
            if (S != 0) wide_add(&lds.lo[m], &lds.hi[m], S);
            S += arow[b];
        }
    }
    wide_flush(lds, n_mat, wide);
}

// grad_mat[m] += (iteration's integer sum for m) / scale / rho_m, one
// iteration after another (the order of these additions is fixed).
__global__ void k_adj_fold(const unsigned long long *__restrict__ wide, int32_t n_mat,
                           const double *__restrict__ scale_p, const float *__restrict__ mat_rho,
                           double *__restrict__ grad_mat) {
    const double scale = *scale_p;
    for (int m = threadIdx.x; m < n_mat; m += blockDim.x) {
        const unsigned long long lo = wide[m];
        const long long hi = (long long)(wide[n_mat + m] + (lo >> 32));
        if (scale > 0.0 && (hi != 0 || (lo & 0xffffffffull) != 0ull) && mat_rho[m] > 0.0f) {
            const double v = (double)hi * 4294967296.0 + (double)(lo & 0xffffffffull);
            grad_mat[m] += (v / scale) / (double)mat_rho[m];
        }
    }
}

// Per-workgroup partial sums of g_p L_p (every term of L_p is proportional to
// the emitted radiance); k_collect_grad adds them in a fixed order.
__global__ __launch_bounds__(kBlock) void k_le_grad(SppmDev d, double K, const float *__restrict__ g,
                                                    double *__restrict__ part) {
    __shared__ double lds[kBlock / 64];
    int64_t p = (int64_t)blockIdx.x * kBlock + threadIdx.x;
    double v = 0.0;
    if (p < d.P) v = (double)g[p] * (d.tau[p] / ((kPiD * d.R2[p]) * K) + d.D[p] / K);
    for (int off = 32; off > 0; off >>= 1) v += __shfl_xor(v, off);
    if ((threadIdx.x & 63) == 0) lds[threadIdx.x >> 6] = v;
    __syncthreads();
    if (threadIdx.x == 0) {
        double t = 0.0;
        for (int w = 0; w < kBlock / 64; ++w) t += lds[w];
        part[blockIdx.x] = t;
    }
}

__global__ void k_fill_f64(double *p, int64_t n) {
    int64_t i = (int64_t)blockIdx.x * kBlock + threadIdx.x;
    if (i < n) p[i] = 0.0;
}

struct ParamMats {
    uint8_t m[kMaxAdjMat];
};

// One workgroup of kMaxAdjMat threads: parameter gradients, and the emission
// gradient as a fixed-order sum of the partial sums of g L.
__global__ __launch_bounds__(kMaxAdjMat) void k_collect_grad(const double *__restrict__ grad_mat, ParamMats pm,
                                                             int32_t n_par, const double *__restrict__ le_part,
                                                             int32_t n_part, double inv_Le, double *__restrict__ out) {
    __shared__ double lds[kMaxAdjMat];
    const int i = threadIdx.x;
    double t = 0.0;
    for (int j = i; j < n_part; j += kMaxAdjMat) t += le_part[j];
    lds[i] = t;
    __syncthreads();
    for (int w = kMaxAdjMat / 2; w > 0; w >>= 1) {
        if (i < w) lds[i] += lds[i + w];
        __syncthreads();
    }
    if (i < n_par) out[i] = grad_mat[pm.m[i]];
    if (i == n_par) out[i] = lds[0] * inv_Le;
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

namespace pm {

void sppm_free(pm_sppm *s) {
    // kernels of this handle may still be in flight on the caller's stream
    (void)hipDeviceSynchronize();
    void *bufs[] = {s->mat_type, s->mat_f, s->emit_pos, s->emit_cdf, s->N, s->R2, s->tau, s->D, s->hp_pos,
                    s->hp_nrm, s->store, s->store2, s->sorted, s->counters, s->r2max, s->cell_count, s->cell_start,
                    s->cell_fill, s->bsum, s->M, s->Phi, s->R2_hist, s->adj_tab, s->mat_tab, s->adj_tab2,
                    s->mat_tab2, s->grad_mat,
                    s->adj_wide, s->adj_max, s->adj_scale, s->le_part, s->stats, s->sh_key, s->sh_surv, s->slot_mem, s->key_rank,
                    s->queue_mem, s->hp_pos2, s->hp_nrm2};
    for (void *b : bufs)
        if (b) (void)hipFree(b);
    for (hipEvent_t e : s->prof_ev)
        if (e) (void)hipEventDestroy(e);
    for (int i = 0; i < 2; ++i) {
        if (s->ev_ph[i]) (void)hipEventDestroy(s->ev_ph[i]);
        if (s->ev_scat[i]) (void)hipEventDestroy(s->ev_scat[i]);
    }
    if (s->phs) (void)hipStreamDestroy(s->phs);
    for (int i = 0; i < 2; ++i) {
        if (s->ev_head[i]) (void)hipEventDestroy(s->ev_head[i]);
        if (s->ev_eye[i]) (void)hipEventDestroy(s->ev_eye[i]);
        if (s->ev_upd[i]) (void)hipEventDestroy(s->ev_upd[i]);
    }
    if (s->tails) (void)hipStreamDestroy(s->tails);
    if (s->ev_fork) (void)hipEventDestroy(s->ev_fork);
    if (s->ev_join) (void)hipEventDestroy(s->ev_join);
    if (s->side) (void)hipStreamDestroy(s->side);
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
    if (p->photon_kernel < 0 || p->photon_kernel > PM_PHOTON_TWO_PHASE || p->refill < 0 || p->refill > 64)
        return set_error("photon_kernel must be 0..6 and refill 0..64"), PM_ERR_ARG;
    if (p->pass_threads < 0 || p->pass_threads > (1 << 26) || p->passes < 0 || p->passes > 1024)
        return set_error("pass_threads must be in [0, 2^26] and passes in [0, 1024]"), PM_ERR_ARG;
    if (p->photon_kernel != PM_PHOTON_PASSES && (p->pass_threads != 0 || p->passes != 0))
        return set_error("pass_threads and passes apply to photon_kernel PM_PHOTON_PASSES only"), PM_ERR_ARG;
    if (p->gather_mode != PM_GATHER_EXACT && p->gather_mode != PM_GATHER_STOCHASTIC)
        return set_error("gather_mode must be PM_GATHER_EXACT or PM_GATHER_STOCHASTIC"), PM_ERR_ARG;
    if (p->gather_mode == PM_GATHER_STOCHASTIC && p->record_iterations > 0)
        return set_error("the adjoint needs the exact gather (gather_mode 0)"), PM_ERR_ARG;
    if (p->profile < 0 || p->profile > (PM_PROFILE_COUNT | PM_PROFILE_TIME))
        return set_error("profile must be a combination of PM_PROFILE_COUNT and PM_PROFILE_TIME"), PM_ERR_ARG;
    if ((p->profile & PM_PROFILE_COUNT) &&
        (p->gather_mode != PM_GATHER_EXACT || p->photon_kernel == PM_PHOTON_PER_PATH || p->photon_kernel == PM_PHOTON_PASSES))
        return set_error("PM_PROFILE_COUNT counts the regenerating photon kernels and the exact gather"), PM_ERR_ARG;
    if (p->single_link_set < 0 || p->single_link_set > 6)
        return set_error("single_link_set must be 0 (by direction) or 1..6"), PM_ERR_ARG;
    if (p->record_iterations < 0 || p->record_iterations > 100000)
        return set_error("record_iterations must be in [0, 100000]"), PM_ERR_ARG;
    if (p->record_iterations > 0 && d->n_mat > kMaxAdjMat)
        return set_error("the adjoint supports at most 256 materials"), PM_ERR_ARG;
    // a photon's (path, bounce) entry sums at most one term of 2^39 units per pixel
    if (p->record_iterations > 0 && (int64_t)d->width * d->height >= (int64_t(1) << 24))
        return set_error("the adjoint supports images below 2^24 pixels"), PM_ERR_ARG;
    return PM_OK;
}

// The photon schedule a handle runs: the default is the two-phase pass on
// single-scene handles and regeneration for a batch member (whose photon
// stage the batch schedules).
static int32_t photon_kernel_of(const pm_sppm_params *p, bool own_grid) {
    if (p->photon_kernel != PM_PHOTON_AUTO) return p->photon_kernel;
    return own_grid ? PM_PHOTON_TWO_PHASE : PM_PHOTON_REGEN;
}

int sppm_create_ex(const pm_scene_desc *d, const pm_sppm_params *p, hipStream_t st, bool own_grid, pm_sppm **out) {
    int rc = sppm_validate(d, p);
    if (rc) return rc;
    pm_sppm *s = new pm_sppm();
    s->prm = *p;
    auto fail = [&](int code) {
        sppm_free(s);
        return code;
    };
#define PM_HIPF(call)                                            \
    do {                                                         \
        hipError_t e_ = (call);                                  \
        if (e_ != hipSuccess) return fail(hip_fail(e_, #call));  \
    } while (0)
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
    s->scene_hash = scene_fingerprint(d);
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
    H3 ext{b->hi[0] - b->lo[0], b->hi[1] - b->lo[1], b->hi[2] - b->lo[2]};
    float diag = std::sqrt(hdot(ext, ext));
    s->phi0 = (float)((kPiD * acc) / (double)p->n_photons);
    int64_t cap64 = p->n_photons * p->store_factor;
    s->cap = (uint32_t)cap64;
    uint32_t bits = 12;
    while (bits < 24 && (int64_t(1) << bits) < 4 * p->n_photons) bits++;
    s->table_bits = bits;
    const uint32_t T = 1u << bits;
    const uint32_t nb = T / kScanTile;
    const int32_t nm = d->n_mat;

    PM_HIPF(hipMalloc(&s->mat_type, sizeof(int32_t) * nm));
    PM_HIPF(hipMalloc(&s->mat_f, sizeof(float) * 4 * nm));
    PM_HIPF(hipMalloc(&s->emit_pos, sizeof(uint32_t) * std::max<size_t>(1, epos.size())));
    PM_HIPF(hipMalloc(&s->emit_cdf, sizeof(double) * std::max<size_t>(1, ecdf.size())));
    PM_HIPF(hipMalloc(&s->N, sizeof(double) * s->P));
    PM_HIPF(hipMalloc(&s->R2, sizeof(double) * s->P));
    PM_HIPF(hipMalloc(&s->tau, sizeof(double) * s->P));
    PM_HIPF(hipMalloc(&s->D, sizeof(double) * s->P));
    PM_HIPF(hipMalloc(&s->hp_pos, sizeof(float4) * s->P));
    PM_HIPF(hipMalloc(&s->hp_nrm, sizeof(float4) * s->P));
    PM_HIPF(hipMalloc(&s->store, sizeof(float4) * 2 * (size_t)cap64));
    PM_HIPF(hipMalloc(&s->counters, sizeof(uint32_t) * 8));
    PM_HIPF(hipMalloc(&s->r2max, sizeof(unsigned long long) * 2));  // one per iteration parity
    if (own_grid && !(p->profile & PM_PROFILE_TIME)) {
        // a second photon store and a photon stream: consecutive iterations overlap
        PM_HIPF(hipMalloc(&s->store2, sizeof(float4) * 2 * (size_t)cap64));
        PM_HIPF(hipStreamCreateWithFlags(&s->phs, hipStreamNonBlocking));
        for (int i = 0; i < 2; ++i) {
            PM_HIPF(hipEventCreateWithFlags(&s->ev_ph[i], hipEventDisableTiming));
            PM_HIPF(hipEventCreateWithFlags(&s->ev_scat[i], hipEventDisableTiming));
            PM_HIPF(hipEventCreateWithFlags(&s->ev_eye[i], hipEventDisableTiming));
            PM_HIPF(hipEventCreateWithFlags(&s->ev_upd[i], hipEventDisableTiming));
        }
        PM_HIPF(hipMalloc(&s->hp_pos2, sizeof(float4) * s->P));
        PM_HIPF(hipMalloc(&s->hp_nrm2, sizeof(float4) * s->P));
        if (photon_kernel_of(p, own_grid) == PM_PHOTON_TWO_PHASE) {
            PM_HIPF(hipStreamCreateWithFlags(&s->tails, hipStreamNonBlocking));
            for (int i = 0; i < 2; ++i) PM_HIPF(hipEventCreateWithFlags(&s->ev_head[i], hipEventDisableTiming));
        }
    }
    if (own_grid) {
        PM_HIPF(hipStreamCreateWithFlags(&s->side, hipStreamNonBlocking));
        PM_HIPF(hipEventCreateWithFlags(&s->ev_fork, hipEventDisableTiming));
        PM_HIPF(hipEventCreateWithFlags(&s->ev_join, hipEventDisableTiming));
        PM_HIPF(hipMalloc(&s->cell_count, sizeof(uint32_t) * T));
        if (p->gather_mode == PM_GATHER_STOCHASTIC) {
            PM_HIPF(hipMalloc(&s->sh_key, sizeof(unsigned long long) * T));
            PM_HIPF(hipMalloc(&s->sh_surv, sizeof(uint32_t) * T));
        } else {
            PM_HIPF(hipMalloc(&s->sorted, sizeof(float4) * 2 * (size_t)cap64));
            PM_HIPF(hipMalloc(&s->cell_start, sizeof(uint32_t) * (T + 1)));
            PM_HIPF(hipMalloc(&s->cell_fill, sizeof(uint32_t) * T));
            PM_HIPF(hipMalloc(&s->bsum, sizeof(uint32_t) * (nb + 1)));
        }
    }
    PM_HIPF(hipMalloc(&s->M, sizeof(uint32_t) * s->P));
    PM_HIPF(hipMalloc(&s->Phi, sizeof(unsigned long long) * s->P));
    if (p->gather_mode == PM_GATHER_EXACT) PM_HIPF(hipMalloc(&s->key_rank, sizeof(uint2) * (size_t)cap64));
    if (p->photon_kernel == PM_PHOTON_PASSES) {
        // one slot per thread of a pass; the paper runs one thread per pixel
        const uint32_t S = p->pass_threads > 0 ? (uint32_t)p->pass_threads
                                               : (uint32_t)std::min<int64_t>(s->P, int64_t(1) << 26);
        PM_HIPF(hipMalloc(&s->slot_mem, (size_t)56 * S));
        char *m = (char *)s->slot_mem;
        s->slots.g = (int4 *)m;
        s->slots.o = (float4 *)(m + (size_t)16 * S);
        s->slots.w = (float4 *)(m + (size_t)32 * S);
        s->slots.nb = (uint2 *)(m + (size_t)48 * S);
        s->slots.S = S;
        const int64_t auto_pass = (p->n_photons + S - 1) / S + 8;
        s->n_pass = p->passes > 0 ? p->passes : (int32_t)std::min<int64_t>(auto_pass, 1024);
    }
    if (p->profile & PM_PROFILE_COUNT) {
        PM_HIPF(hipMalloc(&s->stats, sizeof(unsigned long long) * kStatCount));
        PM_HIPF(hipMemsetAsync(s->stats, 0, sizeof(unsigned long long) * kStatCount, st));
    }
    if (p->profile & PM_PROFILE_TIME)
        for (hipEvent_t &e : s->prof_ev) PM_HIPF(hipEventCreate(&e));
    s->n_mat = nm;
    s->rho_host.assign(d->mat_rho, d->mat_rho + nm);
    s->rec_iters = p->record_iterations;
    if (s->rec_iters > 0) {
        PM_HIPF(hipMalloc(&s->R2_hist, sizeof(double) * (size_t)s->rec_iters * s->P));
        PM_HIPF(hipMalloc(&s->adj_tab, sizeof(long long) * (size_t)p->n_photons * p->max_photon_bounces));
        PM_HIPF(hipMalloc(&s->mat_tab, sizeof(uint16_t) * (size_t)p->n_photons * p->max_photon_bounces));
        PM_HIPF(hipMalloc(&s->grad_mat, sizeof(double) * (nm + 1)));
        PM_HIPF(hipMalloc(&s->adj_wide, sizeof(unsigned long long) * 2 * nm));
        PM_HIPF(hipMalloc(&s->adj_max, sizeof(unsigned long long) * 4));
        if (s->store2) {  // the adjoint overlaps consecutive iterations like the forward
            PM_HIPF(hipMalloc(&s->adj_tab2, sizeof(long long) * (size_t)p->n_photons * p->max_photon_bounces));
            PM_HIPF(hipMalloc(&s->mat_tab2, sizeof(uint16_t) * (size_t)p->n_photons * p->max_photon_bounces));
        }
        PM_HIPF(hipMalloc(&s->adj_scale, sizeof(double)));
        PM_HIPF(hipMalloc(&s->le_part, sizeof(double) * blocks_for(s->P)));
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
    PM_HIPF(hipMemcpyAsync(s->mat_type, d->mat_type, sizeof(int32_t) * nm, hipMemcpyHostToDevice, st));
    PM_HIPF(hipMemcpyAsync(s->mat_f, mf.data(), sizeof(float) * 4 * nm, hipMemcpyHostToDevice, st));
    if (!epos.empty()) {
        PM_HIPF(hipMemcpyAsync(s->emit_pos, epos.data(), sizeof(uint32_t) * epos.size(), hipMemcpyHostToDevice, st));
        PM_HIPF(hipMemcpyAsync(s->emit_cdf, ecdf.data(), sizeof(double) * ecdf.size(), hipMemcpyHostToDevice, st));
    }
    PM_HIPF(hipMemsetAsync(s->counters, 0, sizeof(uint32_t) * 8, st));
    PM_HIPF(hipMemsetAsync(s->hp_nrm, 0xff, sizeof(float4) * s->P, st));
    if (s->hp_nrm2) PM_HIPF(hipMemsetAsync(s->hp_nrm2, 0xff, sizeof(float4) * s->P, st));
    PM_HIPF(hipMemsetAsync(s->M, 0, sizeof(uint32_t) * s->P, st));
    PM_HIPF(hipMemsetAsync(s->Phi, 0, sizeof(unsigned long long) * s->P, st));
    PM_HIPF(hipMemsetAsync(s->r2max, 0, sizeof(unsigned long long) * 2, st));

    SceneDev &sc = s->dev.sc;
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
    sc.ext = std::max(b->hi[0] - b->lo[0], std::max(b->hi[1] - b->lo[1], b->hi[2] - b->lo[2]));
    H3 pos{d->cam_pos[0], d->cam_pos[1], d->cam_pos[2]};
    H3 look{d->cam_look[0], d->cam_look[1], d->cam_look[2]};
    H3 up{d->cam_up[0], d->cam_up[1], d->cam_up[2]};
    H3 f = hnorm(hsub(look, pos));
    H3 r = hnorm(hcross(f, up));
    H3 u = hcross(r, f);
    sc.cpos = V3{pos.x, pos.y, pos.z};
    sc.cf = V3{f.x, f.y, f.z};
    sc.cr = V3{r.x, r.y, r.z};
    sc.cu = V3{u.x, u.y, u.z};
    sc.tanh_fov = d->tan_half_fov;
    sc.aspect = (float)d->width / (float)d->height;
    sc.W = d->width;
    sc.H = d->height;
    SppmDev &dv = s->dev;
    dv.seed = p->seed;
    dv.max_depth = p->max_eye_depth;
    dv.max_bounces = p->max_photon_bounces;
    dv.n_paths = (uint32_t)p->n_photons;
    dv.cap = s->cap;
    dv.phi0 = s->phi0;
    dv.alpha = p->alpha;
    dv.scale = std::ldexp(1.0, p->fixed_shift);
    dv.inv_scale = std::ldexp(1.0, -p->fixed_shift);
    dv.P = s->P;
    dv.mask = T - 1u;
    dv.table_off = 0;
    dv.photon_kernel = photon_kernel_of(p, own_grid);
    dv.refill = p->refill > 0 ? (uint32_t)p->refill : 32u;
    dv.force_set = p->single_link_set - 1;
    // Paired node requests pay off on one large scene (2.65 -> 2.55 ms per
    // iteration of the 250k-triangle scene) but not on the many small scenes
    // of a batch, whose BVHs stay in cache (24.5 -> 25.3 ms).
    dv.paired_walk = own_grid ? 1 : 0;
    dv.gather_mode = p->gather_mode;
    dv.sh_key = s->sh_key;
    dv.sh_surv = s->sh_surv;
    {
        int dev = 0, cus = 0, per_cu = 0;
        PM_HIPF(hipGetDevice(&dev));
        PM_HIPF(hipDeviceGetAttribute(&cus, hipDeviceAttributeMultiprocessorCount, dev));
        PM_HIPF(hipOccupancyMaxActiveBlocksPerMultiprocessor(&per_cu, k_photon_regen, kBlock, 0));
        s->regen_grid = (uint32_t)std::max(1, cus * std::max(1, per_cu));
        PM_HIPF(hipOccupancyMaxActiveBlocksPerMultiprocessor(&per_cu, k_photon_regen_rec, kBlock, 0));
        s->regen_grid_rec = (uint32_t)std::max(1, cus * std::max(1, per_cu));
        PM_HIPF(hipOccupancyMaxActiveBlocksPerMultiprocessor(&per_cu, k_photon_stream, kBlock, 0));
        s->stream_grid = (uint32_t)std::max(1, cus * std::max(1, per_cu));
        PM_HIPF(hipOccupancyMaxActiveBlocksPerMultiprocessor(&per_cu, k_photon_pool<false>, kBlock, 0));
        s->pool_grid = (uint32_t)std::max(1, cus * std::max(1, per_cu));
        PM_HIPF(hipOccupancyMaxActiveBlocksPerMultiprocessor(&per_cu, k_photon_head<false>, kBlock, 0));
        s->head_grid = (uint32_t)std::max(1, cus * std::max(1, per_cu));
        PM_HIPF(hipOccupancyMaxActiveBlocksPerMultiprocessor(&per_cu, k_photon_tail<false>, kBlock, 0));
        s->tail_grid = (uint32_t)std::max(1, cus * std::max(1, per_cu));
        PM_HIPF(hipOccupancyMaxActiveBlocksPerMultiprocessor(&per_cu, k_photon_head_rec, kBlock, 0));
        s->head_grid_rec = (uint32_t)std::max(1, cus * std::max(1, per_cu));
        PM_HIPF(hipOccupancyMaxActiveBlocksPerMultiprocessor(&per_cu, k_photon_tail_rec, kBlock, 0));
        s->tail_grid_rec = (uint32_t)std::max(1, cus * std::max(1, per_cu));
    }
    if (dv.photon_kernel == PM_PHOTON_TWO_PHASE) {
        // per store parity: a queue slot for every lane of the first launch
        // (each parks at most one path), then the queue's two counters
        const uint32_t S = (uint32_t)std::min<int64_t>(
            p->n_photons, (int64_t)std::max(s->head_grid, s->head_grid_rec) * kBlock);
        const size_t per = (size_t)56 * S + 256;
        PM_HIPF(hipMalloc(&s->queue_mem, 2 * per));
        for (int i = 0; i < 2; ++i) {
            char *m = (char *)s->queue_mem + i * per;
            PathQueue &q = s->queue[i];
            q.s.g = (int4 *)m;
            q.s.o = (float4 *)(m + (size_t)16 * S);
            q.s.w = (float4 *)(m + (size_t)32 * S);
            q.s.nb = (uint2 *)(m + (size_t)48 * S);
            q.s.S = S;
            q.cnt = (uint32_t *)(m + (size_t)56 * S);
        }
    }
    dv.hp_pos = s->hp_pos;
    dv.hp_nrm = s->hp_nrm;
    dv.N = s->N;
    dv.R2 = s->R2;
    dv.tau = s->tau;
    dv.D = s->D;
    dv.store = s->store;
    dv.key_rank = s->key_rank;
    dv.counters = s->counters;
    dv.r2max = s->r2max;
    dv.M = s->M;
    dv.Phi = s->Phi;
    dv.stats = s->stats;
    hipLaunchKernelGGL(k_init_state, dim3(blocks_for(s->P)), dim3(kBlock), 0, st, dv, p->r0 * p->r0);
    PM_HIPF(hipGetLastError());
    // host staging vectors go out of scope: finish the copies first
    PM_HIPF(hipStreamSynchronize(st));
#undef PM_HIPF
    *out = s;
    return PM_OK;
}

int sppm_create(const pm_scene_desc *d, const pm_sppm_params *p, hipStream_t st, pm_sppm **out) {
    return sppm_create_ex(d, p, st, true, out);
}

int sppm_destroy(pm_sppm *s) {
    if (!s) return set_error("NULL handle"), PM_ERR_ARG;
    sppm_free(s);
    return PM_OK;
}

int sppm_reset(pm_sppm *s, hipStream_t st) {
    hipLaunchKernelGGL(k_init_state, dim3(blocks_for(s->P)), dim3(kBlock), 0, st, s->dev, s->prm.r0 * s->prm.r0);
    PM_HIP(hipGetLastError());
    s->K = 0;
    return PM_OK;
}

// Device view of iteration k: a pipelined handle alternates two photon stores
// (each with its block of four counters), two hit-point buffers and two R_max
// accumulators between consecutive iterations.
static SppmDev iteration_view(const pm_sppm *s, uint32_t k) {
    SppmDev dk = s->dev;
    const uint32_t par = s->store2 ? (k & 1u) : 0u;
    dk.store = par ? s->store2 : s->store;
    dk.counters = s->counters + 4 * par;
    dk.r2max = s->r2max + par;
    if (par && s->hp_pos2) {
        dk.hp_pos = s->hp_pos2;
        dk.hp_nrm = s->hp_nrm2;
    }
    return dk;
}

// The photon pass of iteration k (its counters cleared first) on stream q;
// the two-phase pass's second launch goes on stream tq (after the first).
// The pass has ended once tq's work enqueued so far is done.
static int enqueue_photon(pm_sppm *s, const SppmDev &dk, uint32_t k, bool count, hipStream_t q, hipStream_t tq) {
    const uint32_t np = (uint32_t)s->prm.n_photons;
    hipLaunchKernelGGL(k_photon_begin, dim3(1), dim3(64), 0, q, dk);
    if (dk.photon_kernel == PM_PHOTON_TWO_PHASE) {
        const PathQueue &pq = s->queue[s->store2 ? (k & 1u) : 0u];
        hipLaunchKernelGGL(k_fill_u32, dim3(1), dim3(64), 0, q, pq.cnt, 2u, 0u);
        if (count)
            hipLaunchKernelGGL(k_photon_head<true>, dim3(s->head_grid), dim3(kBlock), 0, q, dk, k, pq);
        else
            hipLaunchKernelGGL(k_photon_head<false>, dim3(s->head_grid), dim3(kBlock), 0, q, dk, k, pq);
        if (tq != q) {
            PM_HIP(hipEventRecord(s->ev_head[k & 1u], q));
            PM_HIP(hipStreamWaitEvent(tq, s->ev_head[k & 1u], 0));
        }
        if (count)
            hipLaunchKernelGGL(k_photon_tail<true>, dim3(s->tail_grid), dim3(kBlock), 0, tq, dk, k, pq);
        else
            hipLaunchKernelGGL(k_photon_tail<false>, dim3(s->tail_grid), dim3(kBlock), 0, tq, dk, k, pq);
    } else if (dk.photon_kernel == PM_PHOTON_RAY_REGEN) {
        if (count)
            hipLaunchKernelGGL(k_photon_stream_stats, dim3(s->stream_grid), dim3(kBlock), 0, q, dk, k);
        else
            hipLaunchKernelGGL(k_photon_stream, dim3(s->stream_grid), dim3(kBlock), 0, q, dk, k);
    } else if (dk.photon_kernel == PM_PHOTON_POOL) {
        if (count)
            hipLaunchKernelGGL(k_photon_pool<true>, dim3(s->pool_grid), dim3(kBlock), 0, q, dk, k);
        else
            hipLaunchKernelGGL(k_photon_pool<false>, dim3(s->pool_grid), dim3(kBlock), 0, q, dk, k);
    } else if (dk.photon_kernel == PM_PHOTON_REGEN) {
        if (count)
            hipLaunchKernelGGL(k_photon_regen_stats, dim3(s->regen_grid), dim3(kBlock), 0, q, dk, k);
        else
            hipLaunchKernelGGL(k_photon_regen, dim3(s->regen_grid), dim3(kBlock), 0, q, dk, k);
    } else if (dk.photon_kernel == PM_PHOTON_PASSES) {
        const PassSlots &ps = s->slots;
        hipLaunchKernelGGL(k_fill_u32, dim3(blocks_for(2 * (int64_t)ps.S)), dim3(kBlock), 0, q, (uint32_t *)ps.nb,
                           2u * ps.S, kSlotIdle);
        for (int32_t j = 0; j < s->n_pass; ++j)
            hipLaunchKernelGGL(k_photon_pass, dim3(blocks_for(ps.S)), dim3(kBlock), 0, q, dk, k, ps);
        hipLaunchKernelGGL(k_pass_tally, dim3(1), dim3(64), 0, q, dk);
        hipLaunchKernelGGL(k_photon_drain, dim3(blocks_for(ps.S)), dim3(kBlock), 0, q, dk, k, ps);
    } else {
        hipLaunchKernelGGL(k_photon<false>, dim3(blocks_for(np)), dim3(kBlock), 0, q, dk, k, (uint16_t *)nullptr,
                           (long long *)nullptr);
    }
    PM_HIP(hipGetLastError());
    return PM_OK;
}

// One call runs n_iter iterations.  Per iteration k: the eye pass and R_max
// on the side stream, the photon pass, then on the caller's stream the hashed
// grid, the range query and the update.  A pipelined handle (two photon
// stores) runs its photon passes on a third stream, one after another: the
// pass of iteration k + 1 needs nothing of iteration k except a free store,
// so it overlaps iteration k's grid, range query and update and keeps the
// device full while the photon pass drains.  Events order the rest: the
// photon pass of k + 1 waits for the scatter of k - 1 (the last reader of its
// store), the eye pass of k for the update of k - 1 (it overwrites the hit
// points and R_max that k - 1 read), and the grid of k for the eye pass and
// photon pass of k.  At the end of the call the caller's stream has waited
// for every stream.  Results are those of the serial order.
int sppm_iterate(pm_sppm *s, int32_t n_iter, hipStream_t st) {
    if (!s || n_iter < 0) return set_error("invalid handle or iteration count"), PM_ERR_ARG;
    if (!s->cell_count) return set_error("handle belongs to a batch: iterate the batch"), PM_ERR_STATE;
    if (n_iter == 0) return PM_OK;
    const uint32_t T = 1u << s->table_bits;
    const uint32_t ph_blocks = std::min<uint32_t>(blocks_for(s->cap), 256u * 64u);
    const bool count = (s->prm.profile & PM_PROFILE_COUNT) != 0, timed = (s->prm.profile & PM_PROFILE_TIME) != 0;
    const bool pipe = s->store2 != nullptr;
    hipEvent_t *ev = s->prof_ev;
    const uint32_t k0 = (uint32_t)s->K;
    int rc;
    // the two-phase pass's second launch runs on its own stream, so that the
    // next pass's first launch can start beside it
    hipStream_t tq = s->tails ? s->tails : s->phs;
    auto eye_pass = [&](const SppmDev &dv, uint32_t kk, hipStream_t q) {
        if (count)
            hipLaunchKernelGGL(k_eye_stats, dim3(blocks_for(s->P)), dim3(kBlock), 0, q, dv, kk, 1);
        else
            hipLaunchKernelGGL(k_eye, dim3(blocks_for(s->P)), dim3(kBlock), 0, q, dv, kk, 1);
    };
    if (pipe) {
        // photon pass and eye pass of the first iteration, each on its stream
        PM_HIP(hipEventRecord(s->ev_fork, st));
        PM_HIP(hipStreamWaitEvent(s->phs, s->ev_fork, 0));
        PM_HIP(hipStreamWaitEvent(s->side, s->ev_fork, 0));
        if ((rc = enqueue_photon(s, iteration_view(s, k0), k0, count, s->phs, tq))) return rc;
        PM_HIP(hipEventRecord(s->ev_ph[k0 & 1u], tq));
        eye_pass(iteration_view(s, k0), k0, s->side);
        PM_HIP(hipEventRecord(s->ev_eye[k0 & 1u], s->side));
    }
    for (int32_t it = 0; it < n_iter; ++it) {
        const uint32_t k = k0 + (uint32_t)it;
        const SppmDev dk = iteration_view(s, k);
        if (pipe && it + 1 < n_iter) {
            // the next photon pass refills the store (and queue) that the scatter of k - 1 read
            if (it >= 1) PM_HIP(hipStreamWaitEvent(s->phs, s->ev_scat[(k + 1u) & 1u], 0));
            if ((rc = enqueue_photon(s, iteration_view(s, k + 1u), k + 1u, count, s->phs, tq))) return rc;
            PM_HIP(hipEventRecord(s->ev_ph[(k + 1u) & 1u], tq));
            // the next eye pass refills the hit points that the update of k - 1 read
            if (it >= 1) PM_HIP(hipStreamWaitEvent(s->side, s->ev_upd[(k + 1u) & 1u], 0));
            eye_pass(iteration_view(s, k + 1u), k + 1u, s->side);
            PM_HIP(hipEventRecord(s->ev_eye[(k + 1u) & 1u], s->side));
        }
        if (timed) PM_HIP(hipEventRecord(ev[0], st));
        if (pipe) {
            // R_max over the radii after the update of k - 1 and the hit points of k
            PM_HIP(hipStreamWaitEvent(st, s->ev_eye[k & 1u], 0));
            hipLaunchKernelGGL(k_rmax_clear, dim3(1), dim3(64), 0, st, dk);
            hipLaunchKernelGGL(k_rmax, dim3(std::min(blocks_for(s->P), kRmaxBlocks)), dim3(kBlock), 0, st, dk,
                               (const double *)s->R2);
        } else {
            // eye pass and R_max on the side stream, beside the photon pass:
            // they share no data, and the eye pass's long specular paths would
            // otherwise leave the device idle at its end
            PM_HIP(hipEventRecord(s->ev_fork, st));
            PM_HIP(hipStreamWaitEvent(s->side, s->ev_fork, 0));
            if (timed) PM_HIP(hipEventRecord(ev[1], s->side));
            hipLaunchKernelGGL(k_rmax_clear, dim3(1), dim3(64), 0, s->side, dk);
            eye_pass(dk, k, s->side);
            hipLaunchKernelGGL(k_rmax, dim3(std::min(blocks_for(s->P), kRmaxBlocks)), dim3(kBlock), 0, s->side, dk,
                               (const double *)s->R2);
            if (timed) PM_HIP(hipEventRecord(ev[2], s->side));
            PM_HIP(hipEventRecord(s->ev_join, s->side));
            if (timed) PM_HIP(hipEventRecord(ev[3], st));
            if ((rc = enqueue_photon(s, dk, k, count, st, st))) return rc;
            if (timed) PM_HIP(hipEventRecord(ev[4], st));
        }
        hipLaunchKernelGGL(k_fill_u32, dim3(blocks_for(T)), dim3(kBlock), 0, st, s->cell_count, T, 0u);
        if (!pipe) PM_HIP(hipStreamWaitEvent(st, s->ev_join, 0));
        if (pipe) PM_HIP(hipStreamWaitEvent(st, s->ev_ph[k & 1u], 0));
        if (timed) PM_HIP(hipEventRecord(ev[5], st));
        if (dk.gather_mode == PM_GATHER_STOCHASTIC) {
            hipLaunchKernelGGL(k_sh_clear, dim3(std::min<uint32_t>(blocks_for(T), 4096u)), dim3(kBlock), 0, st, dk, T);
            hipLaunchKernelGGL(k_sh_insert, dim3(ph_blocks), dim3(kBlock), 0, st, dk, k, s->cell_count);
            hipLaunchKernelGGL(k_sh_pick, dim3(ph_blocks), dim3(kBlock), 0, st, dk, k);
            if (pipe) PM_HIP(hipEventRecord(s->ev_scat[k & 1u], st));
            if (timed) PM_HIP(hipEventRecord(ev[6], st));
            hipLaunchKernelGGL(k_sh_gather, dim3(blocks_for(s->P)), dim3(kBlock), 0, st, dk,
                               (const uint32_t *)s->cell_count);
        } else {
            hipLaunchKernelGGL(k_count, dim3(ph_blocks), dim3(kBlock), 0, st, dk, s->cell_count);
            launch_bucket_scan(s->cell_count, s->cell_start, s->cell_fill, s->bsum, T, st);
            hipLaunchKernelGGL(k_scatter, dim3(ph_blocks), dim3(kBlock), 0, st, dk, (const uint32_t *)s->cell_start,
                               s->sorted);
            if (pipe) PM_HIP(hipEventRecord(s->ev_scat[k & 1u], st));
            if (timed) PM_HIP(hipEventRecord(ev[6], st));
            if (count)
                hipLaunchKernelGGL(k_gather_stats, dim3(blocks_for(s->P)), dim3(kBlock), 0, st, dk,
                                   (const uint32_t *)s->cell_start, (const float4 *)s->sorted);
            else
                hipLaunchKernelGGL(k_gather, dim3(blocks_for(s->P)), dim3(kBlock), 0, st, dk,
                                   (const uint32_t *)s->cell_start, (const float4 *)s->sorted);
        }
        if (timed) PM_HIP(hipEventRecord(ev[7], st));
        double *hist = (int32_t)k < s->rec_iters ? s->R2_hist + (size_t)k * s->P : nullptr;
        hipLaunchKernelGGL(k_update, dim3(blocks_for(s->P)), dim3(kBlock), 0, st, dk, hist);
        if (pipe) PM_HIP(hipEventRecord(s->ev_upd[k & 1u], st));
        PM_HIP(hipGetLastError());
        if (timed) {  // wait for the iteration and add its stage times
            PM_HIP(hipEventRecord(ev[8], st));
            PM_HIP(hipEventSynchronize(ev[8]));
            float ms[kProfTimes];
            PM_HIP(hipEventElapsedTime(&ms[0], ev[1], ev[2]));  // eye pass + R_max (side stream)
            PM_HIP(hipEventElapsedTime(&ms[1], ev[3], ev[4]));  // photon pass
            PM_HIP(hipEventElapsedTime(&ms[2], ev[5], ev[6]));  // hashed grid
            PM_HIP(hipEventElapsedTime(&ms[3], ev[6], ev[7]));  // range query
            PM_HIP(hipEventElapsedTime(&ms[4], ev[7], ev[8]));  // update
            PM_HIP(hipEventElapsedTime(&ms[5], ev[0], ev[8]));  // whole iteration
            for (int i = 0; i < kProfTimes; ++i) s->prof_ms[i] += ms[i];
            s->prof_timed_iters++;
        }
        if (count) s->prof_counted_iters++;
        s->K++;
    }
    return PM_OK;
}

int sppm_get_stats(pm_sppm *s, pm_sppm_stats *out, int32_t reset, hipStream_t st) {
    if (!s || !out) return set_error("NULL handle or output"), PM_ERR_ARG;
    if (out->size < sizeof(pm_sppm_stats)) return set_error("pm_sppm_stats.size too small"), PM_ERR_ARG;
    unsigned long long c[kStatCount] = {};
    if (s->stats) {
        PM_HIP(hipMemcpyAsync(c, s->stats, sizeof(c), hipMemcpyDeviceToHost, st));
        PM_HIP(hipStreamSynchronize(st));
    }
    const uint32_t size = out->size;
    memset(out, 0, sizeof(pm_sppm_stats));
    out->size = size;
    out->counted_iterations = s->prof_counted_iters;
    out->eye_paths = c[kStatEyePaths];
    out->eye_rays = c[kStatEyeRays];
    out->eye_box_tests = c[kStatEyeBoxes];
    out->eye_tri_tests = c[kStatEyeTris];
    out->photon_paths = c[kStatPhotonPaths];
    out->photon_rays = c[kStatPhotonRays];
    out->photon_box_tests = c[kStatPhotonBoxes];
    out->photon_tri_tests = c[kStatPhotonTris];
    out->gather_hit_points = c[kStatGatherHits];
    out->gather_buckets = c[kStatGatherBuckets];
    out->gather_examined = c[kStatGatherExamined];
    out->gather_accepted = c[kStatGatherAccepted];
    out->photons_stored = c[kStatPhotonStored];
    out->timed_iterations = s->prof_timed_iters;
    out->ms_eye = s->prof_ms[0];
    out->ms_photon = s->prof_ms[1];
    out->ms_grid = s->prof_ms[2];
    out->ms_gather = s->prof_ms[3];
    out->ms_update = s->prof_ms[4];
    out->ms_iteration = s->prof_ms[5];
    if (reset) {
        if (s->stats) {
            hipLaunchKernelGGL(k_fill_u32, dim3(1), dim3(kBlock), 0, st, (uint32_t *)s->stats, 2u * kStatCount, 0u);
            PM_HIP(hipGetLastError());
        }
        s->prof_counted_iters = s->prof_timed_iters = 0;
        for (double &m : s->prof_ms) m = 0.0;
    }
    return PM_OK;
}

int sppm_resolve(pm_sppm *s, float *image, hipStream_t st) {
    if (!s || !image) return set_error("invalid handle or image pointer"), PM_ERR_ARG;
    if (s->K == 0) return set_error("no iteration has run"), PM_ERR_STATE;
    hipLaunchKernelGGL(k_resolve, dim3(blocks_for(s->P)), dim3(kBlock), 0, st, s->dev, s->K, image);
    PM_HIP(hipGetLastError());
    return PM_OK;
}

int sppm_status(pm_sppm *s, hipStream_t st) {
    if (!s) return set_error("NULL handle"), PM_ERR_ARG;
    uint32_t c[8];
    PM_HIP(hipMemcpyAsync(c, s->counters, sizeof(c), hipMemcpyDeviceToHost, st));
    PM_HIP(hipStreamSynchronize(st));
    const uint32_t flags = c[1] | c[5];  // the sticky flags of both photon stores' counter blocks
    if (flags & 1u) return set_error("photon store overflow: raise store_factor"), PM_ERR_OVERFLOW;
    if (flags & 2u)
        return set_error("flux fixed-point overflow (a term or a pixel's sum passed 2^64): lower fixed_shift"),
               PM_ERR_OVERFLOW;
    return PM_OK;
}

// The adjoint's replay with consecutive iterations overlapped, as in the
// forward iteration: the replayed photon pass of k + 1 (with its flux
// maximum) runs on the photon stream beside the grid, gather and path sums of
// k, into the other photon store, (path, bounce) tables and maxima; the
// replayed eye pass of k, R_max and the |G| wk maximum run on the side stream
// once iteration k - 1 is done with the hit points.  Every sum is an integer
// sum, so the gradient equals the serial schedule's bit for bit.
static int adjoint_overlapped(pm_sppm *s, const float *g, hipStream_t st) {
    const uint32_t T = 1u << s->table_bits;
    const uint32_t np = (uint32_t)s->prm.n_photons;
    const int32_t mb = s->prm.max_photon_bounces;
    const uint32_t ph_blocks = std::min<uint32_t>(blocks_for(s->cap), 256u * 64u);
    const uint32_t K = (uint32_t)s->K;
    const double Kd = (double)s->K;
    auto mat_of = [&](uint32_t k) { return (k & 1u) ? s->mat_tab2 : s->mat_tab; };
    auto tab_of = [&](uint32_t k) { return (k & 1u) ? s->adj_tab2 : s->adj_tab; };
    auto max_of = [&](uint32_t k) { return s->adj_max + 2 * (k & 1u); };
    // the replayed photon pass: on the photon stream, or (two-phase handles)
    // its first launch there and the second on the tail stream, beside the
    // first launch of the next replay; the flux maximum follows the pass
    const bool two = s->dev.photon_kernel == PM_PHOTON_TWO_PHASE && s->tails;
    hipStream_t tq = two ? s->tails : s->phs;
    auto replay = [&](uint32_t k) -> int {
        const SppmDev dk = iteration_view(s, k);
        hipLaunchKernelGGL(k_photon_begin, dim3(1), dim3(64), 0, s->phs, dk);
        hipLaunchKernelGGL(k_fill_u32, dim3(1), dim3(64), 0, s->phs, (uint32_t *)(max_of(k) + 1), 2u, 0u);
        if (two) {
            const PathQueue &pq = s->queue[k & 1u];
            hipLaunchKernelGGL(k_fill_u32, dim3(1), dim3(64), 0, s->phs, pq.cnt, 2u, 0u);
            hipLaunchKernelGGL(k_photon_head_rec, dim3(s->head_grid_rec), dim3(kBlock), 0, s->phs, dk, k, pq,
                               mat_of(k), tab_of(k));
            PM_HIP(hipEventRecord(s->ev_head[k & 1u], s->phs));
            PM_HIP(hipStreamWaitEvent(tq, s->ev_head[k & 1u], 0));
            hipLaunchKernelGGL(k_photon_tail_rec, dim3(s->tail_grid_rec), dim3(kBlock), 0, tq, dk, k, pq, mat_of(k),
                               tab_of(k));
        } else {
            hipLaunchKernelGGL(k_photon_regen_rec, dim3(s->regen_grid_rec), dim3(kBlock), 0, s->phs, dk, k,
                               mat_of(k), tab_of(k));
        }
        hipLaunchKernelGGL(k_adj_phimax, dim3(std::min<uint32_t>(ph_blocks, kAdjMaxBlocks)), dim3(kBlock), 0, tq, dk,
                           max_of(k));
        PM_HIP(hipGetLastError());
        PM_HIP(hipEventRecord(s->ev_ph[k & 1u], tq));
        return PM_OK;
    };
    // the replayed eye pass, R_max (over the recorded radii) and max |G| wk of
    // iteration k, on the side stream, into the hit-point buffer, R_max
    // accumulator and maxima of k's parity
    auto eye_chain = [&](uint32_t k) -> int {
        const SppmDev dk = iteration_view(s, k);
        const double *R2k = s->R2_hist + (size_t)k * s->P;
        hipLaunchKernelGGL(k_rmax_clear, dim3(1), dim3(64), 0, s->side, dk);
        hipLaunchKernelGGL(k_eye, dim3(blocks_for(s->P)), dim3(kBlock), 0, s->side, dk, k, 0);
        hipLaunchKernelGGL(k_rmax, dim3(std::min(blocks_for(s->P), kRmaxBlocks)), dim3(kBlock), 0, s->side, dk, R2k);
        hipLaunchKernelGGL(k_fill_u32, dim3(1), dim3(64), 0, s->side, (uint32_t *)max_of(k), 2u, 0u);
        hipLaunchKernelGGL(k_adj_gmax, dim3(std::min<uint32_t>(blocks_for(s->P), kAdjMaxBlocks)), dim3(kBlock), 0,
                           s->side, dk, R2k, g, Kd, max_of(k));
        PM_HIP(hipGetLastError());
        PM_HIP(hipEventRecord(s->ev_eye[k & 1u], s->side));
        return PM_OK;
    };
    PM_HIP(hipEventRecord(s->ev_fork, st));
    PM_HIP(hipStreamWaitEvent(s->phs, s->ev_fork, 0));
    PM_HIP(hipStreamWaitEvent(s->side, s->ev_fork, 0));
    int rc = replay(0);
    if (rc) return rc;
    if ((rc = eye_chain(0))) return rc;
    for (uint32_t k = 0; k < K; ++k) {
        const SppmDev dk = iteration_view(s, k);
        const double *R2k = s->R2_hist + (size_t)k * s->P;
        if (k + 1 < K) {
            // the replay of k + 1 reuses the store and tables that iteration k - 1 read
            if (k >= 1) PM_HIP(hipStreamWaitEvent(s->phs, s->ev_scat[(k + 1u) & 1u], 0));
            if ((rc = replay(k + 1))) return rc;
            // and its eye pass the hit points, R_max and maxima that the range query of k - 1 read
            if (k >= 1) PM_HIP(hipStreamWaitEvent(s->side, s->ev_upd[(k + 1u) & 1u], 0));
            if ((rc = eye_chain(k + 1))) return rc;
        }
        hipLaunchKernelGGL(k_fill_u32, dim3(blocks_for(T)), dim3(kBlock), 0, st, s->cell_count, T, 0u);
        hipLaunchKernelGGL(k_fill_u32, dim3(blocks_for(4 * s->n_mat)), dim3(kBlock), 0, st, (uint32_t *)s->adj_wide,
                           (uint32_t)(4 * s->n_mat), 0u);
        PM_HIP(hipStreamWaitEvent(st, s->ev_eye[k & 1u], 0));
        PM_HIP(hipStreamWaitEvent(st, s->ev_ph[k & 1u], 0));
        hipLaunchKernelGGL(k_adj_scale, dim3(1), dim3(64), 0, st, (const unsigned long long *)max_of(k), s->adj_scale);
        hipLaunchKernelGGL(k_count, dim3(ph_blocks), dim3(kBlock), 0, st, dk, s->cell_count);
        launch_bucket_scan(s->cell_count, s->cell_start, s->cell_fill, s->bsum, T, st);
        hipLaunchKernelGGL(k_scatter, dim3(ph_blocks), dim3(kBlock), 0, st, dk, (const uint32_t *)s->cell_start,
                           s->sorted);
        hipLaunchKernelGGL(k_gather_adj, dim3(blocks_for(s->P)), dim3(kBlock), 0, st, dk, R2k,
                           (const uint32_t *)s->cell_start, (const float4 *)s->sorted, g, Kd,
                           (const double *)s->adj_scale, tab_of(k), s->n_mat, s->adj_wide);
        PM_HIP(hipEventRecord(s->ev_upd[k & 1u], st));
        hipLaunchKernelGGL(k_path_adj, dim3(blocks_for(np)), dim3(kBlock), 0, st, (const uint16_t *)mat_of(k),
                           (const long long *)tab_of(k), np, mb, s->n_mat, s->adj_wide);
        PM_HIP(hipEventRecord(s->ev_scat[k & 1u], st));
        hipLaunchKernelGGL(k_adj_fold, dim3(1), dim3(kMaxAdjMat), 0, st, (const unsigned long long *)s->adj_wide,
                           s->n_mat, (const double *)s->adj_scale, dk.sc.mat_rho, s->grad_mat);
        PM_HIP(hipGetLastError());
    }
    return PM_OK;
}

int sppm_adjoint(pm_sppm *s, const float *g, const int32_t *pmat, int32_t n_par, double *grad, hipStream_t st) {
    if (!s || !g || !grad || n_par < 0 || (n_par > 0 && !pmat))
        return set_error("invalid handle, gradient or parameter pointers"), PM_ERR_ARG;
    if (!s->cell_count) return set_error("handle belongs to a batch"), PM_ERR_STATE;
    if (s->K < 1) return set_error("no iteration has run"), PM_ERR_STATE;
    if (s->K > s->rec_iters)
        return set_error("the forward iterations were not recorded: set record_iterations >= K"), PM_ERR_STATE;
    if (n_par >= kMaxAdjMat) return set_error("too many parameters"), PM_ERR_ARG;
    for (int32_t i = 0; i < n_par; ++i) {
        if (pmat[i] < 0 || pmat[i] >= s->n_mat) return set_error("parameter material out of range"), PM_ERR_ARG;
        if (!(s->rho_host[pmat[i]] > 0.0f)) return set_error("albedo parameters must have rho > 0"), PM_ERR_ARG;
    }
    const uint32_t T = 1u << s->table_bits;
    const uint32_t np = (uint32_t)s->prm.n_photons;
    const int32_t mb = s->prm.max_photon_bounces;
    const uint32_t ph_blocks = std::min<uint32_t>(blocks_for(s->cap), 256u * 64u);
    const double K = (double)s->K;
    const SppmDev &d = s->dev;
    ParamMats pms;
    for (int32_t i = 0; i < n_par; ++i) pms.m[i] = (uint8_t)pmat[i];
    hipLaunchKernelGGL(k_fill_f64, dim3(blocks_for(s->n_mat + 1)), dim3(kBlock), 0, st, s->grad_mat,
                       (int64_t)s->n_mat + 1);
    if (s->adj_tab2) {
        int rc = adjoint_overlapped(s, g, st);
        if (rc) return rc;
    }
    for (int32_t k = 0; k < (s->adj_tab2 ? 0 : s->K); ++k) {
        const double *R2k = s->R2_hist + (size_t)k * s->P;
        hipLaunchKernelGGL(k_begin, dim3(1), dim3(64), 0, st, d);
        hipLaunchKernelGGL(k_adj_begin, dim3(1), dim3(kBlock), 0, st, s->adj_max, s->adj_wide, s->n_mat);
        hipLaunchKernelGGL(k_fill_u32, dim3(blocks_for(T)), dim3(kBlock), 0, st, s->cell_count, T, 0u);
        // replayed eye pass, R_max and max |G| wk beside the replayed photon pass, as in the forward iteration
        PM_HIP(hipEventRecord(s->ev_fork, st));
        PM_HIP(hipStreamWaitEvent(s->side, s->ev_fork, 0));
        hipLaunchKernelGGL(k_eye, dim3(blocks_for(s->P)), dim3(kBlock), 0, s->side, d, (uint32_t)k, 0);
        hipLaunchKernelGGL(k_rmax, dim3(std::min(blocks_for(s->P), kRmaxBlocks)), dim3(kBlock), 0, s->side, d, R2k);
        hipLaunchKernelGGL(k_adj_gmax, dim3(std::min<uint32_t>(blocks_for(s->P), kAdjMaxBlocks)), dim3(kBlock), 0,
                           s->side, d, R2k, g, K, s->adj_max);
        PM_HIP(hipEventRecord(s->ev_join, s->side));
        hipLaunchKernelGGL(k_photon_regen_rec, dim3(s->regen_grid_rec), dim3(kBlock), 0, st, d, (uint32_t)k,
                           s->mat_tab, s->adj_tab);
        hipLaunchKernelGGL(k_adj_phimax, dim3(std::min<uint32_t>(ph_blocks, kAdjMaxBlocks)), dim3(kBlock), 0, st, d,
                           s->adj_max);
        PM_HIP(hipStreamWaitEvent(st, s->ev_join, 0));
        hipLaunchKernelGGL(k_adj_scale, dim3(1), dim3(64), 0, st, (const unsigned long long *)s->adj_max,
                           s->adj_scale);
        hipLaunchKernelGGL(k_count, dim3(ph_blocks), dim3(kBlock), 0, st, d, s->cell_count);
        launch_bucket_scan(s->cell_count, s->cell_start, s->cell_fill, s->bsum, T, st);
        hipLaunchKernelGGL(k_scatter, dim3(ph_blocks), dim3(kBlock), 0, st, d, (const uint32_t *)s->cell_start,
                           s->sorted);
        hipLaunchKernelGGL(k_gather_adj, dim3(blocks_for(s->P)), dim3(kBlock), 0, st, d, R2k,
                           (const uint32_t *)s->cell_start, (const float4 *)s->sorted, g, K,
                           (const double *)s->adj_scale, s->adj_tab, s->n_mat, s->adj_wide);
        hipLaunchKernelGGL(k_path_adj, dim3(blocks_for(np)), dim3(kBlock), 0, st, (const uint16_t *)s->mat_tab,
                           (const long long *)s->adj_tab, np, mb, s->n_mat, s->adj_wide);
        hipLaunchKernelGGL(k_adj_fold, dim3(1), dim3(kMaxAdjMat), 0, st, (const unsigned long long *)s->adj_wide,
                           s->n_mat, (const double *)s->adj_scale, d.sc.mat_rho, s->grad_mat);
        PM_HIP(hipGetLastError());
    }
    const uint32_t n_part = blocks_for(s->P);
    hipLaunchKernelGGL(k_le_grad, dim3(n_part), dim3(kBlock), 0, st, d, K, g, s->le_part);
    hipLaunchKernelGGL(k_collect_grad, dim3(1), dim3(kMaxAdjMat), 0, st, s->grad_mat, pms, n_par,
                       (const double *)s->le_part, (int32_t)n_part, s->le_single > 0.0 ? 1.0 / s->le_single : 0.0,
                       grad);
    PM_HIP(hipGetLastError());
    return PM_OK;
}

namespace {

struct HashWords {  // FNV-1a over 32-bit words
    uint64_t h = 0xcbf29ce484222325ull;
    void add(const void *p, size_t bytes) {
        const uint8_t *b = (const uint8_t *)p;
        for (size_t i = 0; i + 4 <= bytes; i += 4) {
            uint32_t w;
            memcpy(&w, b + i, 4);
            h = (h ^ w) * 0x100000001b3ull;
        }
        for (size_t i = bytes & ~(size_t)3; i < bytes; ++i) h = (h ^ b[i]) * 0x100000001b3ull;
    }
};

// Checkpoint layout: this header, then N, R2, tau, D (f64 [P] each), then
// n_hist recorded radii (f64 [n_hist][P]).
struct CheckpointHeader {
    char magic[8];  // "PMSPPMCK"
    uint32_t version, header_bytes;
    int64_t n_pixels, n_photons;
    uint64_t seed, scene_hash;
    double alpha, r0;
    int32_t fixed_shift, max_eye_depth, max_photon_bounces, record_iterations;
    int32_t iterations, n_hist;
    uint32_t overflow;
    int32_t gather_mode;
};
constexpr uint32_t kCheckpointVersion = 1;

uint64_t checkpoint_bytes(const pm_sppm *s, int32_t n_hist) {
    return sizeof(CheckpointHeader) + (uint64_t)(4 + n_hist) * (uint64_t)s->P * sizeof(double);
}

}  // namespace

uint64_t scene_fingerprint(const pm_scene_desc *d) {
    HashWords h;
    h.add(&d->n_tri, sizeof(d->n_tri));
    h.add(d->tri_verts, sizeof(float) * 9 * (size_t)d->n_tri);
    h.add(d->tri_mat, sizeof(uint32_t) * (size_t)d->n_tri);
    h.add(&d->n_mat, sizeof(d->n_mat));
    h.add(d->mat_type, sizeof(int32_t) * (size_t)d->n_mat);
    h.add(d->mat_rho, sizeof(float) * (size_t)d->n_mat);
    h.add(d->mat_q, sizeof(float) * (size_t)d->n_mat);
    h.add(d->mat_Le, sizeof(float) * (size_t)d->n_mat);
    h.add(d->mat_ior, sizeof(float) * (size_t)d->n_mat);
    h.add(d->cam_pos, sizeof(d->cam_pos));
    h.add(d->cam_look, sizeof(d->cam_look));
    h.add(d->cam_up, sizeof(d->cam_up));
    h.add(&d->tan_half_fov, sizeof(d->tan_half_fov));
    h.add(&d->width, sizeof(d->width));
    h.add(&d->height, sizeof(d->height));
    return h.h;
}

int sppm_save(pm_sppm *s, void *buf, uint64_t *size, hipStream_t st) {
    if (!s || !size) return set_error("NULL handle or size pointer"), PM_ERR_ARG;
    if (!s->cell_count) return set_error("handle belongs to a batch"), PM_ERR_STATE;
    const int32_t n_hist = std::min(s->K, s->rec_iters);
    const uint64_t need = checkpoint_bytes(s, n_hist);
    if (!buf) {
        *size = need;
        return PM_OK;
    }
    if (*size < need) {
        *size = need;
        return set_error("checkpoint buffer too small (the required size is returned in *size)"), PM_ERR_ARG;
    }
    uint32_t c[8];
    PM_HIP(hipMemcpyAsync(c, s->counters, sizeof(c), hipMemcpyDeviceToHost, st));
    c[1] |= c[5];
    CheckpointHeader h{};
    memcpy(h.magic, "PMSPPMCK", 8);
    h.version = kCheckpointVersion;
    h.header_bytes = sizeof(CheckpointHeader);
    h.n_pixels = s->P;
    h.n_photons = s->prm.n_photons;
    h.seed = s->prm.seed;
    h.scene_hash = s->scene_hash;
    h.alpha = s->prm.alpha;
    h.r0 = s->prm.r0;
    h.fixed_shift = s->prm.fixed_shift;
    h.max_eye_depth = s->prm.max_eye_depth;
    h.max_photon_bounces = s->prm.max_photon_bounces;
    h.record_iterations = s->rec_iters;
    h.iterations = s->K;
    h.n_hist = n_hist;
    h.gather_mode = s->prm.gather_mode;
    uint8_t *out = (uint8_t *)buf;
    const size_t pb = sizeof(double) * (size_t)s->P;
    const double *arrays[4] = {s->N, s->R2, s->tau, s->D};
    for (int a = 0; a < 4; ++a)
        PM_HIP(hipMemcpyAsync(out + sizeof(h) + a * pb, arrays[a], pb, hipMemcpyDeviceToHost, st));
    if (n_hist > 0)
        PM_HIP(hipMemcpyAsync(out + sizeof(h) + 4 * pb, s->R2_hist, pb * (size_t)n_hist, hipMemcpyDeviceToHost, st));
    PM_HIP(hipStreamSynchronize(st));
    h.overflow = c[1];
    memcpy(out, &h, sizeof(h));
    *size = need;
    return PM_OK;
}

int sppm_load(pm_sppm *s, const void *buf, uint64_t size, hipStream_t st) {
    if (!s || !buf) return set_error("NULL handle or buffer"), PM_ERR_ARG;
    if (!s->cell_count) return set_error("handle belongs to a batch"), PM_ERR_STATE;
    CheckpointHeader h;
    if (size < sizeof(h)) return set_error("checkpoint too short"), PM_ERR_ARG;
    memcpy(&h, buf, sizeof(h));
    if (memcmp(h.magic, "PMSPPMCK", 8) != 0 || h.version != kCheckpointVersion || h.header_bytes != sizeof(h))
        return set_error("not a checkpoint of this format version"), PM_ERR_ARG;
    if (h.n_pixels != s->P || h.n_photons != s->prm.n_photons || h.seed != s->prm.seed ||
        h.scene_hash != s->scene_hash || h.alpha != s->prm.alpha || h.r0 != s->prm.r0 ||
        h.fixed_shift != s->prm.fixed_shift || h.max_eye_depth != s->prm.max_eye_depth ||
        h.max_photon_bounces != s->prm.max_photon_bounces || h.record_iterations != s->rec_iters ||
        h.gather_mode != s->prm.gather_mode)
        return set_error("checkpoint was taken from a handle with another scene or parameters"), PM_ERR_ARG;
    if (h.iterations < 0 || h.n_hist != std::min(h.iterations, s->rec_iters) ||
        size < checkpoint_bytes(s, h.n_hist))
        return set_error("checkpoint is truncated or inconsistent"), PM_ERR_ARG;
    const uint8_t *in = (const uint8_t *)buf;
    const size_t pb = sizeof(double) * (size_t)s->P;
    double *arrays[4] = {s->N, s->R2, s->tau, s->D};
    for (int a = 0; a < 4; ++a)
        PM_HIP(hipMemcpyAsync(arrays[a], in + sizeof(h) + a * pb, pb, hipMemcpyHostToDevice, st));
    if (h.n_hist > 0)
        PM_HIP(hipMemcpyAsync(s->R2_hist, in + sizeof(h) + 4 * pb, pb * (size_t)h.n_hist, hipMemcpyHostToDevice, st));
    if (h.overflow) PM_HIP(hipMemcpyAsync(s->counters + 1, &h.overflow, sizeof(h.overflow), hipMemcpyHostToDevice, st));
    PM_HIP(hipStreamSynchronize(st));
    s->K = h.iterations;
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
    // the last iteration's hit points, photon store and counters (a pipelined handle alternates two of each)
    const uint32_t par = (s->store2 && s->K > 0) ? (uint32_t)((s->K - 1) & 1) : 0u;
    v->hp_pos = (float *)(par ? s->hp_pos2 : s->hp_pos);
    v->hp_nrm = (float *)(par ? s->hp_nrm2 : s->hp_nrm);
    v->photons = (float *)(par ? s->store2 : s->store);
    v->photon_count = s->counters + 4 * par;
    v->gather_M = s->M;
    v->gather_Phi = (uint64_t *)s->Phi;
    return PM_OK;
}

}  // namespace pm
