// Internal state of an SPPM handle (shared by the single-scene driver and the
// batched driver).
#pragma once
#include <hip/hip_runtime.h>

#include <vector>

#include "runtime.h"
#include "sppm_dev.h"

struct pm_sppm {
    pm_sppm_params prm{};
    pm_bvh *bvh = nullptr;
    bool own_bvh = false;
    pmd::SppmDev dev{};  // device view passed to the kernels
    int64_t P = 0;
    int32_t K = 0;
    uint32_t cap = 0;
    uint32_t table_bits = 0;
    uint32_t regen_grid = 1;      // workgroups of the regenerating photon kernel
    uint32_t regen_grid_rec = 1;  // and of its recording variant (adjoint replay)
    uint32_t stream_grid = 1;     // workgroups of the ray-granularity regenerating photon kernel
    uint32_t pool_grid = 1;       // workgroups of the LDS-queue photon kernel
    uint32_t head_grid = 1;       // workgroups of the two-phase pass's first launch
    uint32_t tail_grid = 1;       // and of its second
    uint32_t head_grid_rec = 1;   // the same two launches recording for the adjoint replay
    uint32_t tail_grid_rec = 1;
    float phi0 = 0.0f;
    // device buffers
    int32_t *mat_type = nullptr;
    float *mat_f = nullptr;  // rho | q | Le | ior, each n_mat
    uint32_t *emit_pos = nullptr;
    double *emit_cdf = nullptr;
    double *N = nullptr, *R2 = nullptr, *tau = nullptr, *D = nullptr;
    float4 *hp_pos = nullptr, *hp_nrm = nullptr;
    float4 *store = nullptr, *sorted = nullptr;
    // pipelined handles: a second photon store, the stream the photon passes
    // run on, and events per store (photon pass done, scatter done)
    float4 *store2 = nullptr;
    hipStream_t phs = nullptr;
    hipEvent_t ev_ph[2] = {}, ev_scat[2] = {};
    // two-phase photon pass (PM_PHOTON_TWO_PHASE): a queue per store parity
    // for the paths set aside by the first launch; on a pipelined handle the
    // second launch runs on its own stream after the first (event ev_head)
    void *queue_mem = nullptr;
    // a second hit-point buffer (pipelined handles): the eye pass of k + 1
    // writes it while the range query and update of k read the first; events
    // per buffer: eye pass done, update done
    float4 *hp_pos2 = nullptr, *hp_nrm2 = nullptr;
    hipEvent_t ev_eye[2] = {}, ev_upd[2] = {};
    pmd::PathQueue queue[2] = {};
    hipStream_t tails = nullptr;
    hipEvent_t ev_head[2] = {};
    uint2 *key_rank = nullptr;  // exact gather: [cap] bucket and rank of each stored photon
    uint32_t *counters = nullptr;  // [8]: per photon store [0] photons stored, [1] sticky flags, [2] next path, [3] pass leftovers
    unsigned long long *r2max = nullptr;
    // bucket arrays (absent for a batch member, which uses the batch's)
    uint32_t *cell_count = nullptr, *cell_start = nullptr, *cell_fill = nullptr, *bsum = nullptr;
    uint32_t *M = nullptr;
    unsigned long long *Phi = nullptr;
    // adjoint recording / replay buffers (record_iterations > 0)
    int32_t rec_iters = 0;
    int32_t n_mat = 0;
    std::vector<float> rho_host;  // albedos (validation of adjoint parameters)
    double le_single = 0.0;  // Le of the single emitting material, 0 if not exactly one
    double *R2_hist = nullptr;    // [rec_iters][P] radius used in each iteration
    long long *adj_tab = nullptr;  // [n_photons][max_bounces] photon sensitivities (fixed point, see adj_*)
    uint16_t *mat_tab = nullptr;   // [n_photons][max_bounces] stored-photon materials
    // second copies for odd iterations when the adjoint overlaps iterations (with store2)
    long long *adj_tab2 = nullptr;
    uint16_t *mat_tab2 = nullptr;
    double *grad_mat = nullptr;    // [n_mat + 1]; last entry: sum g L
    unsigned long long *adj_wide = nullptr;  // [2][n_mat] per-material integer sums of one iteration (lo | hi)
    unsigned long long *adj_max = nullptr;   // [2][2] per iteration parity: max |G| wk over hit points, max
                                             // flux over photons (double bits)
    double *adj_scale = nullptr;             // [1] fixed-point scale of the current iteration
    double *le_part = nullptr;               // [blocks over pixels] partial sums of g L
    uint64_t scene_hash = 0;      // fingerprint of the scene description (checkpoint matching)
    // the eye pass runs beside the photon pass on a second stream (default
    // priority), forked from and joined back to the caller's stream by events
    hipStream_t side = nullptr;
    hipEvent_t ev_fork = nullptr, ev_join = nullptr;
    unsigned long long *sh_key = nullptr;  // stochastic hashing (gather_mode 1): [T] keys
    uint32_t *sh_surv = nullptr;           // and [T] survivors
    // one-bounce-per-pass photon schedule (PM_PHOTON_PASSES): path slots and
    // the number of passes enqueued per iteration before the drain
    void *slot_mem = nullptr;
    pmd::PassSlots slots{};
    int32_t n_pass = 0;
    // profiling (params.profile): device counts, and stage times of each timed iteration
    unsigned long long *stats = nullptr;  // [pmd::kStatCount]
    hipEvent_t prof_ev[9] = {};
    double prof_ms[6] = {};
    int64_t prof_counted_iters = 0, prof_timed_iters = 0;
};

constexpr int kProfTimes = 6;

namespace pm {

// own_grid = false: no bucket arrays (a batch member uses the batch's arrays).
int sppm_create_ex(const pm_scene_desc *d, const pm_sppm_params *p, hipStream_t st, bool own_grid, pm_sppm **out);
void sppm_free(pm_sppm *s);
// Back to the initial state (N = 0, R^2 = r0^2, tau = 0, D = 0, K = 0).
int sppm_reset(pm_sppm *s, hipStream_t st);
// 64-bit fingerprint of everything in a scene description that the render reads.
uint64_t scene_fingerprint(const pm_scene_desc *d);

}  // namespace pm
