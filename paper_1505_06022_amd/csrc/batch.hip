// Batched SPPM: many scenes of uneven size advance together.  Each stage of an
// iteration is ONE persistent launch for all scenes: workgroups pull items
// (scene, chunk of elements) from a device work counter, so small and large
// scenes share the GPU without per-scene launches or tail effects.  An
// iteration (all stages, scan included) is captured once as a hipGraph and
// replayed; the iteration index lives in device memory.  The chunk size and
// the workgroup size come from a timed sweep (autotuner) whose result is
// cached on disk.
#include <algorithm>
#include <chrono>
#include <cstdio>
#include <cstdlib>
#include <cstring>
#include <fstream>
#include <sstream>
#include <string>
#include <vector>

#include "runtime.h"
#include "sppm.h"
#include "sppm_dev.h"
#include "sppm_host.h"
#include "sppm_scan.h"

namespace {

using namespace pmd;

enum Stage : int { kStEye = 0, kStPhoton, kStRmax, kStCount, kStScatter, kStGather, kStUpdate, kNumStages };

// A photon-stage item holds kPhotonItem chunks of paths, split between the
// workgroup's wavefronts, which regenerate paths within their share.
constexpr uint32_t kPhotonItem = 8;

struct BatchDev {
    const SppmDev *scenes;  // [S]
    int32_t S;
    uint32_t *queue;        // [kNumStages] work counters
    const uint32_t *item_off;  // [kNumStages][S + 1] first item of each scene
    uint32_t chunk;         // elements per item
    uint32_t *iter;         // iteration index k
    uint32_t *cell_count, *cell_start, *cell_fill;
    float4 *sorted;
};

__device__ __forceinline__ int find_scene(const uint32_t *off, int S, uint32_t it) {
    int lo = 0, hi = S - 1;  // largest s with off[s] <= it
    while (lo < hi) {
        int mid = (lo + hi + 1) >> 1;
        if (off[mid] <= it) lo = mid;
        else hi = mid - 1;
    }
    return lo;
}

template <int kStage>
__device__ __forceinline__ int64_t stage_elems(const SppmDev &d) {
    if (kStage == kStPhoton) return d.n_paths;
    if (kStage == kStCount || kStage == kStScatter) return stored_photons(d);
    return d.P;
}

// Persistent stage kernel: every workgroup loops taking items until the
// stage's item count is exhausted (each item is taken exactly once, so every
// workgroup reaches the exit).
template <int kStage, int kBs>
__global__ __launch_bounds__(kBs) void k_batch(BatchDev b) {
    __shared__ uint32_t s_item;
    const uint32_t *off = b.item_off + kStage * (b.S + 1);
    const uint32_t total = off[b.S];
    const uint32_t k = *b.iter;
    for (;;) {
        if (threadIdx.x == 0) s_item = atomicAdd(&b.queue[kStage], 1u);
        __syncthreads();
        const uint32_t it = s_item;
        __syncthreads();
        if (it >= total) break;
        const int s = __builtin_amdgcn_readfirstlane(find_scene(off, b.S, it));
        const SppmDev &d = b.scenes[s];
        const int64_t per = kStage == kStPhoton ? (int64_t)b.chunk * kPhotonItem : (int64_t)b.chunk;
        const int64_t e0 = (int64_t)(it - off[s]) * per;
        const int64_t end = min(e0 + per, stage_elems<kStage>(d));
        if (kStage == kStPhoton) {
            constexpr int kWaves = kBs / 64;
            const int64_t span = (end - e0 + kWaves - 1) / kWaves;
            const int64_t w0 = min(e0 + (int64_t)(threadIdx.x >> 6) * span, end), w1 = min(w0 + span, end);
            photon_regen_range(d, k, (uint32_t)w0, (uint32_t)w1, d.refill);
            continue;
        }
        if (kStage == kStRmax) {
            unsigned long long v = 0ull;
            for (int64_t e = e0 + threadIdx.x; e < end; e += kBs) {
                unsigned long long x = rmax_lane(d, d.R2, e);
                v = x > v ? x : v;
            }
            rmax_flush(d, v);
            continue;
        }
        if (kStage == kStGather) {
            // every lane of the workgroup takes part in each round (p = P: no pixel)
            Grid gr = make_grid(d);
            for (int64_t e = e0; e < end; e += kBs) {
                const int64_t p = e + threadIdx.x;
                gather_wave(d, gr, p < end ? p : d.P, b.cell_start, b.sorted);
            }
            continue;
        }
        if (kStage == kStCount || kStage == kStScatter) {
            Grid gr = make_grid(d);
            for (int64_t e = e0 + threadIdx.x; e < end; e += kBs) {
                if (kStage == kStCount) count_elem(d, gr, (uint32_t)e, b.cell_count);
                if (kStage == kStScatter) scatter_elem(d, (uint32_t)e, b.cell_start, b.sorted);
            }
            continue;
        }
        for (int64_t e = e0 + threadIdx.x; e < end; e += kBs) {
            if (kStage == kStEye) eye_elem(d, k, e, true);
            if (kStage == kStUpdate) update_elem(d, e, nullptr);
        }
    }
}

// Iteration setup: clear work counters, photon counters and R_max of all scenes.
__global__ void k_batch_begin(BatchDev b) {
    if (threadIdx.x < kNumStages) b.queue[threadIdx.x] = 0u;
    for (int s = threadIdx.x; s < b.S; s += blockDim.x) {
        b.scenes[s].counters[0] = 0u;
        b.scenes[s].counters[2] = 0u;
        *b.scenes[s].r2max = 0ull;
    }
}

// Items of the photon-indexed stages, from the device photon counts.
__global__ void k_batch_plan(BatchDev b, uint32_t *item_off) {
    if (threadIdx.x != 0) return;
    uint32_t acc = 0;
    uint32_t *oc = item_off + kStCount * (b.S + 1), *os = item_off + kStScatter * (b.S + 1);
    for (int s = 0; s < b.S; ++s) {
        oc[s] = acc;
        os[s] = acc;
        acc += (stored_photons(b.scenes[s]) + b.chunk - 1) / b.chunk;
    }
    oc[b.S] = acc;
    os[b.S] = acc;
}

__global__ void k_batch_end(BatchDev b) {
    if (threadIdx.x == 0) *b.iter += 1u;
}

__global__ void k_batch_set_iter(BatchDev b, uint32_t v) {
    if (threadIdx.x == 0) *b.iter = v;
}

__global__ __launch_bounds__(kBlock) void k_batch_resolve(SppmDev d, int32_t K, float *__restrict__ img) {
    int64_t p = (int64_t)blockIdx.x * kBlock + threadIdx.x;
    if (p < d.P) img[p] = resolve_elem(d, p, K);
}

inline uint32_t blocks_for(int64_t n) { return (uint32_t)((n + kBlock - 1) / kBlock); }

}  // namespace

struct pm_batch {
    std::vector<pm_sppm *> members;
    int32_t S = 0;
    int32_t K = 0;
    uint32_t chunk = 1024;
    int32_t block = 256;
    bool use_graph = true;
    // device
    SppmDev *d_scenes = nullptr;
    uint32_t *queue = nullptr, *item_off = nullptr, *iter = nullptr;
    uint32_t *cell_count = nullptr, *cell_start = nullptr, *cell_fill = nullptr, *bsum = nullptr;
    float4 *sorted = nullptr;
    uint32_t total_buckets = 0;
    uint32_t grid[kNumStages] = {};
    hipStream_t cap_stream = nullptr;
    hipStream_t side = nullptr;  // eye and r_max stages beside the photon stage (default priority)
    hipEvent_t ev_fork = nullptr, ev_join = nullptr;
    hipGraph_t graph = nullptr;
    hipGraphExec_t exec = nullptr;
    std::vector<double> tune_ms;  // per candidate
    std::vector<std::pair<uint32_t, int32_t>> tune_cfg;
    bool tuned_from_cache = false;
};

namespace pm {

namespace {

BatchDev batch_dev(const pm_batch *b) {
    BatchDev d;
    d.scenes = b->d_scenes;
    d.S = b->S;
    d.queue = b->queue;
    d.item_off = b->item_off;
    d.chunk = b->chunk;
    d.iter = b->iter;
    d.cell_count = b->cell_count;
    d.cell_start = b->cell_start;
    d.cell_fill = b->cell_fill;
    d.sorted = b->sorted;
    return d;
}

template <int kBs>
int occupancy_grids(pm_batch *b) {
    int dev = 0, cus = 0;
    PM_HIP(hipGetDevice(&dev));
    PM_HIP(hipDeviceGetAttribute(&cus, hipDeviceAttributeMultiprocessorCount, dev));
    const void *kern[kNumStages] = {(const void *)k_batch<kStEye, kBs>, (const void *)k_batch<kStPhoton, kBs>,
                                    (const void *)k_batch<kStRmax, kBs>, (const void *)k_batch<kStCount, kBs>,
                                    (const void *)k_batch<kStScatter, kBs>, (const void *)k_batch<kStGather, kBs>,
                                    (const void *)k_batch<kStUpdate, kBs>};
    for (int st = 0; st < kNumStages; ++st) {
        int per_cu = 0;
        PM_HIP(hipOccupancyMaxActiveBlocksPerMultiprocessor(&per_cu, kern[st], kBs, 0));
        b->grid[st] = (uint32_t)std::max(1, cus * std::max(1, per_cu));
    }
    return PM_OK;
}

template <int kBs>
void enqueue_stage(const pm_batch *b, int stage, const BatchDev &bd, hipStream_t st) {
    dim3 g(b->grid[stage]), blk(kBs);
    switch (stage) {
        case kStEye: hipLaunchKernelGGL((k_batch<kStEye, kBs>), g, blk, 0, st, bd); break;
        case kStPhoton: hipLaunchKernelGGL((k_batch<kStPhoton, kBs>), g, blk, 0, st, bd); break;
        case kStRmax: hipLaunchKernelGGL((k_batch<kStRmax, kBs>), g, blk, 0, st, bd); break;
        case kStCount: hipLaunchKernelGGL((k_batch<kStCount, kBs>), g, blk, 0, st, bd); break;
        case kStScatter: hipLaunchKernelGGL((k_batch<kStScatter, kBs>), g, blk, 0, st, bd); break;
        case kStGather: hipLaunchKernelGGL((k_batch<kStGather, kBs>), g, blk, 0, st, bd); break;
        default: hipLaunchKernelGGL((k_batch<kStUpdate, kBs>), g, blk, 0, st, bd); break;
    }
}

// One iteration of every scene (graph-capturable: kernels only).
int enqueue_iteration(const pm_batch *b, hipStream_t st) {
    BatchDev bd = batch_dev(b);
    auto stage = [&](int s) {
        if (b->block == 128) enqueue_stage<128>(b, s, bd, st);
        else enqueue_stage<256>(b, s, bd, st);
    };
    auto stage_on = [&](int s, hipStream_t q) {
        if (b->block == 128) enqueue_stage<128>(b, s, bd, q);
        else enqueue_stage<256>(b, s, bd, q);
    };
    hipLaunchKernelGGL(k_batch_begin, dim3(1), dim3(256), 0, st, bd);
    // eye and r_max stages on the side stream, photon stage on st: they share
    // no data, and the photon stage fills the device while eye paths finish
    PM_HIP(hipEventRecord(b->ev_fork, st));
    PM_HIP(hipStreamWaitEvent(b->side, b->ev_fork, 0));
    stage_on(kStEye, b->side);
    stage_on(kStRmax, b->side);
    PM_HIP(hipEventRecord(b->ev_join, b->side));
    hipLaunchKernelGGL(k_fill_u32, dim3(blocks_for(b->total_buckets)), dim3(kBlock), 0, st, b->cell_count,
                       b->total_buckets, 0u);
    stage(kStPhoton);
    PM_HIP(hipStreamWaitEvent(st, b->ev_join, 0));
    hipLaunchKernelGGL(k_batch_plan, dim3(1), dim3(64), 0, st, bd, b->item_off);
    stage(kStCount);
    launch_bucket_scan(b->cell_count, b->cell_start, b->cell_fill, b->bsum, b->total_buckets, st);
    stage(kStScatter);
    stage(kStGather);
    stage(kStUpdate);
    hipLaunchKernelGGL(k_batch_end, dim3(1), dim3(64), 0, st, bd);
    PM_HIP(hipGetLastError());
    return PM_OK;
}

// Static items per scene for the pixel- and path-indexed stages.
int upload_items(pm_batch *b, hipStream_t st) {
    const int S = b->S;
    std::vector<uint32_t> off((size_t)kNumStages * (S + 1), 0u);
    for (int stg = 0; stg < kNumStages; ++stg) {
        uint32_t acc = 0;
        for (int s = 0; s < S; ++s) {
            off[(size_t)stg * (S + 1) + s] = acc;
            const pm_sppm *m = b->members[s];
            int64_t n = stg == kStPhoton ? m->prm.n_photons : (stg == kStCount || stg == kStScatter ? 0 : m->P);
            const int64_t per = stg == kStPhoton ? (int64_t)b->chunk * kPhotonItem : (int64_t)b->chunk;
            acc += (uint32_t)((n + per - 1) / per);
        }
        off[(size_t)stg * (S + 1) + S] = acc;
    }
    PM_HIP(hipMemcpyAsync(b->item_off, off.data(), sizeof(uint32_t) * off.size(), hipMemcpyHostToDevice, st));
    PM_HIP(hipStreamSynchronize(st));
    return PM_OK;
}

void drop_graph(pm_batch *b) {
    if (b->exec) (void)hipGraphExecDestroy(b->exec);
    if (b->graph) (void)hipGraphDestroy(b->graph);
    b->exec = nullptr;
    b->graph = nullptr;
}

int configure(pm_batch *b, uint32_t chunk, int32_t block, hipStream_t st) {
    drop_graph(b);
    b->chunk = chunk;
    b->block = block;
    int rc = block == 128 ? occupancy_grids<128>(b) : occupancy_grids<256>(b);
    if (rc) return rc;
    if ((rc = upload_items(b, st))) return rc;
    if (b->use_graph) {
        PM_HIP(hipStreamBeginCapture(b->cap_stream, hipStreamCaptureModeThreadLocal));
        rc = enqueue_iteration(b, b->cap_stream);
        hipGraph_t g = nullptr;
        hipError_t e = hipStreamEndCapture(b->cap_stream, &g);
        if (rc) {
            if (g) (void)hipGraphDestroy(g);
            return rc;
        }
        if (e != hipSuccess) return hip_fail(e, "hipStreamEndCapture");
        b->graph = g;
        PM_HIP(hipGraphInstantiate(&b->exec, b->graph, nullptr, nullptr, 0));
    }
    return PM_OK;
}

int run_iterations(pm_batch *b, int32_t n, hipStream_t st) {
    for (int32_t i = 0; i < n; ++i) {
        if (b->exec) {
            PM_HIP(hipGraphLaunch(b->exec, st));
        } else {
            int rc = enqueue_iteration(b, st);
            if (rc) return rc;
        }
        b->K++;
    }
    return PM_OK;
}

int reset_all(pm_batch *b, hipStream_t st) {
    for (pm_sppm *m : b->members) {
        int rc = sppm_reset(m, st);
        if (rc) return rc;
    }
    BatchDev bd = batch_dev(b);
    hipLaunchKernelGGL(k_batch_set_iter, dim3(1), dim3(64), 0, st, bd, 0u);
    PM_HIP(hipGetLastError());
    b->K = 0;
    return PM_OK;
}

std::string signature(const pm_batch *b) {
    std::ostringstream os;
    int dev = 0;
    hipDeviceProp_t prop;
    if (hipGetDevice(&dev) == hipSuccess && hipGetDeviceProperties(&prop, dev) == hipSuccess) os << prop.gcnArchName;
    os << ":" << b->S;
    for (const pm_sppm *m : b->members)
        os << ":" << m->P << "," << m->prm.n_photons << "," << (m->bvh ? m->bvh->n_tri : 0);
    std::string s = os.str();
    // FNV-1a of the description
    uint64_t h = 1469598103934665603ull;
    for (char c : s) {
        h ^= (uint8_t)c;
        h *= 1099511628211ull;
    }
    char buf[32];
    std::snprintf(buf, sizeof(buf), "%016llx", (unsigned long long)h);
    return buf;
}

std::string cache_path() {
    const char *p = std::getenv("PM_AUTOTUNE_CACHE");
    if (p && *p) return p;
    const char *home = std::getenv("HOME");
    if (home && *home) return std::string(home) + "/.cache/pm_autotune.txt";
    return "";
}

bool cache_lookup(const std::string &sig, uint32_t &chunk, int32_t &block) {
    std::string path = cache_path();
    if (path.empty()) return false;
    std::ifstream f(path);
    std::string key;
    uint32_t c;
    int32_t bl;
    double ms;
    bool found = false;
    while (f >> key >> c >> bl >> ms)
        if (key == sig) {
            chunk = c;
            block = bl;
            found = true;
        }
    return found;
}

void cache_store(const std::string &sig, uint32_t chunk, int32_t block, double ms) {
    std::string path = cache_path();
    if (path.empty()) return;
    std::ofstream f(path, std::ios::app);
    if (f) f << sig << " " << chunk << " " << block << " " << ms << "\n";
}

// Timed sweep over (chunk, block); the state is reset afterwards.
int autotune(pm_batch *b, hipStream_t st) {
    const uint32_t chunks[] = {64, 128, 256, 1024};
    const int32_t blocks[] = {128, 256};
    hipEvent_t e0, e1;
    PM_HIP(hipEventCreate(&e0));
    PM_HIP(hipEventCreate(&e1));
    double best = 1e300;
    uint32_t bc = 1024;
    int32_t bb = 256;
    int rc = PM_OK;
    for (uint32_t c : chunks)
        for (int32_t bl : blocks) {
            if ((rc = configure(b, c, bl, st))) break;
            if ((rc = run_iterations(b, 1, st))) break;  // warm-up
            if (hipEventRecord(e0, st) != hipSuccess) break;
            if ((rc = run_iterations(b, 2, st))) break;
            if (hipEventRecord(e1, st) != hipSuccess || hipEventSynchronize(e1) != hipSuccess) break;
            float ms = 0.0f;
            (void)hipEventElapsedTime(&ms, e0, e1);
            b->tune_cfg.push_back({c, bl});
            b->tune_ms.push_back(ms / 2.0);
            if (ms / 2.0 < best) {
                best = ms / 2.0;
                bc = c;
                bb = bl;
            }
        }
    (void)hipEventDestroy(e0);
    (void)hipEventDestroy(e1);
    if (rc) return rc;
    if ((rc = reset_all(b, st))) return rc;
    if ((rc = configure(b, bc, bb, st))) return rc;
    cache_store(signature(b), bc, bb, best);
    return PM_OK;
}

void batch_free(pm_batch *b) {
    (void)hipDeviceSynchronize();
    drop_graph(b);
    void *bufs[] = {b->d_scenes, b->queue, b->item_off, b->iter, b->cell_count, b->cell_start, b->cell_fill,
                    b->bsum, b->sorted};
    for (void *p : bufs)
        if (p) (void)hipFree(p);
    for (pm_sppm *m : b->members) sppm_free(m);
    if (b->cap_stream) (void)hipStreamDestroy(b->cap_stream);
    if (b->ev_fork) (void)hipEventDestroy(b->ev_fork);
    if (b->ev_join) (void)hipEventDestroy(b->ev_join);
    if (b->side) (void)hipStreamDestroy(b->side);
    delete b;
}

}  // namespace

int batch_create(const pm_scene_desc *const *descs, const pm_sppm_params *const *params, int32_t n,
                 const pm_batch_opts *opts, hipStream_t st, pm_batch **out) {
    if (!descs || !params || !out || n < 1 || n > 4096) return set_error("need 1..4096 scenes"), PM_ERR_ARG;
    if (opts && opts->size < sizeof(pm_batch_opts)) return set_error("pm_batch_opts.size too small"), PM_ERR_ARG;
    int32_t want_chunk = opts ? opts->chunk : 0, want_block = opts ? opts->block : 0;
    if (want_chunk < 0 || want_chunk > (1 << 20) || (want_block != 0 && want_block != 128 && want_block != 256))
        return set_error("chunk must be in [0, 2^20] and block 0, 128 or 256"), PM_ERR_ARG;
    for (int32_t i = 0; i < n; ++i) {
        int rc = sppm_validate(descs[i], params[i]);
        if (rc) return set_error("scene " + std::to_string(i) + ": " + last_error()), rc;
        if (params[i]->gather_mode != PM_GATHER_EXACT)
            return set_error("scene " + std::to_string(i) + ": a batch uses the exact gather"), PM_ERR_ARG;
        if (params[i]->photon_kernel == PM_PHOTON_PASSES || params[i]->photon_kernel == PM_PHOTON_TWO_PHASE)
            return set_error("scene " + std::to_string(i) + ": a batch schedules its own photon stage"), PM_ERR_ARG;
        if (params[i]->profile != 0)
            return set_error("scene " + std::to_string(i) + ": profiling applies to single-scene handles"), PM_ERR_ARG;
    }
    pm_batch *b = new pm_batch();
    auto fail = [&](int code) {
        batch_free(b);
        return code;
    };
    b->S = n;
    b->use_graph = opts ? opts->use_graph != 0 : true;
    int rc;
    for (int32_t i = 0; i < n; ++i) {
        pm_sppm *m = nullptr;
        if ((rc = sppm_create_ex(descs[i], params[i], st, false, &m))) return fail(rc);
        b->members.push_back(m);
    }
    // shared bucket arrays: scene s owns [table_off_s, table_off_s + T_s)
    uint64_t tot = 0, cap = 0;
    std::vector<SppmDev> devs(n);
    for (int32_t i = 0; i < n; ++i) {
        pm_sppm *m = b->members[i];
        m->dev.table_off = (uint32_t)tot;
        tot += uint64_t(1) << m->table_bits;
        cap += m->cap;
        devs[i] = m->dev;
    }
    if (tot >= (uint64_t(1) << 31) || cap >= (uint64_t(1) << 31))
        return set_error("batch too large for 32-bit bucket offsets"), fail(PM_ERR_ARG);
    b->total_buckets = (uint32_t)tot;
    const uint32_t nbt = b->total_buckets / kScanTile;
    hipError_t e;
#define PM_HIPB(call)                                           \
    do {                                                        \
        e = (call);                                             \
        if (e != hipSuccess) return fail(hip_fail(e, #call));   \
    } while (0)
    PM_HIPB(hipMalloc(&b->d_scenes, sizeof(SppmDev) * n));
    PM_HIPB(hipMalloc(&b->queue, sizeof(uint32_t) * kNumStages));
    PM_HIPB(hipMalloc(&b->item_off, sizeof(uint32_t) * kNumStages * (n + 1)));
    PM_HIPB(hipMalloc(&b->iter, sizeof(uint32_t)));
    PM_HIPB(hipMalloc(&b->cell_count, sizeof(uint32_t) * b->total_buckets));
    PM_HIPB(hipMalloc(&b->cell_start, sizeof(uint32_t) * (b->total_buckets + 1)));
    PM_HIPB(hipMalloc(&b->cell_fill, sizeof(uint32_t) * b->total_buckets));
    PM_HIPB(hipMalloc(&b->bsum, sizeof(uint32_t) * (nbt + 1)));
    PM_HIPB(hipMalloc(&b->sorted, sizeof(float4) * 2 * cap));
    PM_HIPB(hipMemcpyAsync(b->d_scenes, devs.data(), sizeof(SppmDev) * n, hipMemcpyHostToDevice, st));
    PM_HIPB(hipMemsetAsync(b->iter, 0, sizeof(uint32_t), st));
    PM_HIPB(hipStreamSynchronize(st));
    PM_HIPB(hipStreamCreateWithFlags(&b->cap_stream, hipStreamNonBlocking));
    PM_HIPB(hipStreamCreateWithFlags(&b->side, hipStreamNonBlocking));
    PM_HIPB(hipEventCreateWithFlags(&b->ev_fork, hipEventDisableTiming));
    PM_HIPB(hipEventCreateWithFlags(&b->ev_join, hipEventDisableTiming));
#undef PM_HIPB
    uint32_t chunk = 1024;
    int32_t block = 256;
    bool tune = opts && opts->autotune;
    if (want_chunk > 0) chunk = (uint32_t)want_chunk;
    if (want_block > 0) block = want_block;
    if (tune && cache_lookup(signature(b), chunk, block)) {
        tune = false;
        b->tuned_from_cache = true;
    }
    if (tune) rc = autotune(b, st);
    else rc = configure(b, chunk, block, st);
    if (rc) return fail(rc);
    *out = b;
    return PM_OK;
}

int batch_destroy(pm_batch *b) {
    if (!b) return set_error("NULL batch"), PM_ERR_ARG;
    batch_free(b);
    return PM_OK;
}

int batch_iterate(pm_batch *b, int32_t n, hipStream_t st) {
    if (!b || n < 0) return set_error("invalid batch or iteration count"), PM_ERR_ARG;
    return run_iterations(b, n, st);
}

int batch_resolve(pm_batch *b, float *const *images, hipStream_t st) {
    if (!b || !images) return set_error("invalid batch or images"), PM_ERR_ARG;
    if (b->K == 0) return set_error("no iteration has run"), PM_ERR_STATE;
    for (int32_t s = 0; s < b->S; ++s) {
        if (!images[s]) return set_error("NULL image pointer"), PM_ERR_ARG;
        const pm_sppm *m = b->members[s];
        hipLaunchKernelGGL(k_batch_resolve, dim3(blocks_for(m->P)), dim3(kBlock), 0, st, m->dev, b->K, images[s]);
    }
    PM_HIP(hipGetLastError());
    return PM_OK;
}

int batch_status(pm_batch *b, hipStream_t st) {
    if (!b) return set_error("NULL batch"), PM_ERR_ARG;
    for (int32_t s = 0; s < b->S; ++s) {
        int rc = sppm_status(b->members[s], st);
        if (rc) return set_error("scene " + std::to_string(s) + ": " + last_error()), rc;
    }
    return PM_OK;
}

int batch_info(const pm_batch *b, pm_batch_info *info) {
    if (!b || !info || info->size < sizeof(pm_batch_info)) return set_error("invalid batch or info"), PM_ERR_ARG;
    info->n_scenes = b->S;
    info->iterations = b->K;
    info->chunk = (int32_t)b->chunk;
    info->block = b->block;
    info->uses_graph = b->exec != nullptr;
    info->tuned_from_cache = b->tuned_from_cache;
    info->n_candidates = (int32_t)std::min<size_t>(b->tune_ms.size(), 8);
    for (int i = 0; i < info->n_candidates; ++i) {
        info->cand_chunk[i] = (int32_t)b->tune_cfg[i].first;
        info->cand_block[i] = b->tune_cfg[i].second;
        info->cand_ms[i] = b->tune_ms[i];
    }
    return PM_OK;
}

int batch_views(pm_batch *b, int32_t scene, pm_sppm_views *v) {
    if (!b || scene < 0 || scene >= b->S) return set_error("invalid batch or scene index"), PM_ERR_ARG;
    pm_sppm *m = b->members[scene];
    int rc = sppm_views(m, v);
    if (rc) return rc;
    v->iterations = b->K;
    return PM_OK;
}

}  // namespace pm
