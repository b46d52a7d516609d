// extern "C" boundary of libpm.so: argument validation, error reporting and
// dispatch to the host runtime.  No C++ exception escapes these functions.
#include <cmath>
#include <cstring>
#include <new>
#include <string>

#include <rocprofiler-sdk-roctx/roctx.h>

#include "bvh_build.h"
#include "pm.h"
#include "runtime.h"
#include "sppm.h"

namespace pm {

// A roctx range around each entry point that enqueues device work (host
// time of the call; visible with rocprofv3 --marker-trace).
struct TraceRange {
    explicit TraceRange(const char *name) { roctxRangePushA(name); }
    ~TraceRange() { roctxRangePop(); }
    TraceRange(const TraceRange &) = delete;
    TraceRange &operator=(const TraceRange &) = delete;
};

static thread_local std::string g_err;

void set_error(const std::string &msg) { g_err = msg; }
void clear_error() { g_err.clear(); }
const char *last_error() { return g_err.c_str(); }

int hip_fail(hipError_t e, const char *what) {
    g_err = std::string(what) + ": " + hipGetErrorString(e);
    return e == hipErrorOutOfMemory ? PM_ERR_NOMEM : PM_ERR_HIP;
}

static bool read_opts(const pm_bvh_opts *o, BuildOptions &bo) {
    if (!o) return true;
    if (o->size < sizeof(pm_bvh_opts)) {
        set_error("pm_bvh_opts.size too small");
        return false;
    }
    bo.bins = o->bins;
    bo.max_leaf = o->max_leaf;
    bo.n_threads = o->n_threads;
    bo.trav_cost = o->trav_cost == 0.0f ? 1.0 : (double)o->trav_cost;
    bo.builder = o->builder;
    bo.split_alpha = (double)o->split_alpha;
    if (bo.builder != PM_BUILD_HOST_SAH && bo.builder != PM_BUILD_GPU_LBVH) {
        set_error("builder must be PM_BUILD_HOST_SAH or PM_BUILD_GPU_LBVH");
        return false;
    }
    if (bo.builder == PM_BUILD_GPU_LBVH && bo.split_alpha != 0.0) {
        set_error("spatial splits (split_alpha) are an option of the host SAH build");
        return false;
    }
    return true;
}

}  // namespace pm

#define PM_GUARD(...)                                    \
    try {                                                \
        pm::clear_error();                               \
        __VA_ARGS__                                      \
    } catch (const std::bad_alloc &) {                   \
        pm::set_error("host allocation failed");         \
        return PM_ERR_NOMEM;                             \
    } catch (const std::exception &e) {                  \
        pm::set_error(e.what());                         \
        return PM_ERR_STATE;                             \
    } catch (...) {                                      \
        pm::set_error("unknown C++ exception");          \
        return PM_ERR_STATE;                             \
    }

extern "C" {

int pm_abi_version(void) { return PM_ABI_VERSION; }

const char *pm_last_error(void) { return pm::last_error(); }

int pm_build_bvh_host(const float *tri_verts, const uint32_t *tri_mat, int64_t n_tri, const pm_bvh_opts *opts,
                      int64_t *n_nodes, uint32_t *nodes, uint32_t *tris, pm_bvh_info *info) {
    PM_GUARD({
        if (!tri_verts || !n_nodes) return pm::set_error("tri_verts and n_nodes must not be NULL"), PM_ERR_ARG;
        if (info && info->size < sizeof(pm_bvh_info)) return pm::set_error("pm_bvh_info.size too small"), PM_ERR_ARG;
        pm::BuildOptions bo;
        if (!pm::read_opts(opts, bo)) return PM_ERR_ARG;
        if (bo.builder != PM_BUILD_HOST_SAH) return pm::set_error("the host build is the SAH builder"), PM_ERR_ARG;
        pm::HostBvh hb;
        std::string err;
        if (!pm::build_bvh_host(tri_verts, tri_mat, n_tri, bo, hb, err)) return pm::set_error(err), PM_ERR_ARG;
        *n_nodes = hb.n_nodes;
        if (nodes) std::memcpy(nodes, hb.nodes.data(), hb.nodes.size() * sizeof(uint32_t));
        if (tris) std::memcpy(tris, hb.tris.data(), hb.tris.size() * sizeof(uint32_t));
        if (info) {
            info->n_tri = hb.n_tri;
            info->n_refs = hb.n_refs;
            info->n_nodes = hb.n_nodes;
            info->n_leaves = hb.n_leaves;
            info->depth = hb.depth;
            info->max_leaf = hb.max_leaf;
            info->sah_cost = hb.sah_cost;
            info->device_bytes = (int64_t)(hb.nodes.size() + hb.tris.size()) * 4;
            info->build_ms = hb.build_ms;
            for (int a = 0; a < 3; ++a) {
                info->grid_lo[a] = hb.qlo[a];
                info->grid_step[a] = hb.qstep[a];
            }
        }
        return PM_OK;
    })
}

int pm_build_bvh(const float *tri_verts, const uint32_t *tri_mat, int64_t n_tri, const pm_bvh_opts *opts,
                 void *stream, pm_bvh **out) {
    pm::TraceRange range_("pm_build_bvh");
    PM_GUARD({
        if (!tri_verts || !out) return pm::set_error("tri_verts and out must not be NULL"), PM_ERR_ARG;
        *out = nullptr;
        pm::BuildOptions bo;
        if (!pm::read_opts(opts, bo)) return PM_ERR_ARG;
        pm_bvh *b = nullptr;
        int rc;
        if (bo.builder == PM_BUILD_GPU_LBVH) {
            if (n_tri < 1 || n_tri >= (int64_t(1) << 28)) return pm::set_error("n_tri must be in [1, 2^28)"), PM_ERR_ARG;
            if (bo.max_leaf < 1 || bo.max_leaf > 7 || !(bo.trav_cost > 0.0) || bo.trav_cost > 64.0)
                return pm::set_error("max_leaf must be in [1,7] and trav_cost in (0,64]"), PM_ERR_ARG;
            for (int64_t i = 0; i < 9 * n_tri; ++i)
                if (!std::isfinite(tri_verts[i]))
                    return pm::set_error("non-finite vertex coordinate at triangle " + std::to_string(i / 9)),
                           PM_ERR_ARG;
            b = new pm_bvh();
            rc = pm::build_bvh_gpu(tri_verts, tri_mat, n_tri, bo.max_leaf, bo.trav_cost, (hipStream_t)stream, b);
        } else {
            pm::HostBvh hb;
            std::string err;
            if (!pm::build_bvh_host(tri_verts, tri_mat, n_tri, bo, hb, err)) return pm::set_error(err), PM_ERR_ARG;
            b = new pm_bvh();
            rc = pm::upload_bvh(hb, (hipStream_t)stream, b);
        }
        if (rc) {
            pm::free_bvh(b);
            delete b;
            return rc;
        }
        *out = b;
        return PM_OK;
    })
}

int pm_bvh_destroy(pm_bvh *bvh) {
    PM_GUARD({
        if (!bvh) return pm::set_error("NULL bvh"), PM_ERR_ARG;
        pm::free_bvh(bvh);
        delete bvh;
        return PM_OK;
    })
}

int pm_bvh_download(const pm_bvh *b, uint32_t *nodes, uint32_t *tris, void *stream) {
    PM_GUARD({
        if (!b) return pm::set_error("NULL bvh"), PM_ERR_ARG;
        hipStream_t s = (hipStream_t)stream;
        if (nodes)
            PM_HIP(hipMemcpyAsync(nodes, b->d_nodes, sizeof(uint32_t) * 4 * 6 * (size_t)b->n_nodes,
                                  hipMemcpyDeviceToHost, s));
        if (tris)
            PM_HIP(hipMemcpyAsync(tris, b->d_tris, sizeof(uint32_t) * 12 * (size_t)b->n_refs, hipMemcpyDeviceToHost, s));
        PM_HIP(hipStreamSynchronize(s));
        return PM_OK;
    })
}

int pm_bvh_get_info(const pm_bvh *b, pm_bvh_info *info) {
    PM_GUARD({
        if (!b || !info || info->size < sizeof(pm_bvh_info)) return pm::set_error("invalid bvh or info"), PM_ERR_ARG;
        info->n_tri = b->n_tri;
        info->n_refs = b->n_refs;
        info->n_nodes = b->n_nodes;
        info->n_leaves = b->n_leaves;
        info->depth = b->depth;
        info->max_leaf = b->max_leaf;
        info->sah_cost = b->sah_cost;
        info->device_bytes = b->n_nodes * 6 * 16 + b->n_refs * 48;
        info->build_ms = b->build_ms;
        for (int a = 0; a < 3; ++a) {
            info->grid_lo[a] = b->qlo[a];
            info->grid_step[a] = b->qstep[a];
        }
        return PM_OK;
    })
}

// Host validation of one batch (pm_trace_rays_ex's rules); fills a.
static int parse_trace(const float *rays, int64_t n, int32_t *hit, float *t, const pm_trace_opts *opts,
                       pm::TraceArgs &a) {
    if (n < 0) return pm::set_error("n must be >= 0"), PM_ERR_ARG;
    if (n > 0 && (!rays || !hit || !t)) return pm::set_error("NULL ray or output pointer"), PM_ERR_ARG;
    a = pm::TraceArgs{};
    a.rays = rays;
    a.n = n;
    a.hit = hit;
    a.t = t;
    if (opts) {
        if (opts->size < sizeof(pm_trace_opts)) return pm::set_error("pm_trace_opts.size too small"), PM_ERR_ARG;
        if (opts->link_set < -1 || opts->link_set > 5) return pm::set_error("link_set must be in [-1,5]"), PM_ERR_ARG;
        if (opts->kernel < 0 || opts->kernel > PM_TRACE_SLICES)
            return pm::set_error("unknown traversal kernel"), PM_ERR_ARG;
        if (opts->refill < 0 || opts->refill > 64) return pm::set_error("refill must be in [0,64]"), PM_ERR_ARG;
        if ((opts->kernel == PM_TRACE_POSTPONED || opts->kernel == PM_TRACE_SLICES) && opts->refill > 63)
            return pm::set_error("postponed and slice kernels: refill (lanes still searching) must be in [0,63]"),
                   PM_ERR_ARG;
        if (opts->slice < 0 || opts->slice > (1 << 24))
            return pm::set_error("slice must be in [0, 2^24]"), PM_ERR_ARG;
        if (opts->reorder < 0 || opts->reorder > 2) return pm::set_error("reorder must be 0, 1 or 2"), PM_ERR_ARG;
        if (opts->block != 0 && opts->block != 64 && opts->block != 128 && opts->block != 256)
            return pm::set_error("block must be 0, 64, 128 or 256"), PM_ERR_ARG;
        if (opts->tile_width < 0) return pm::set_error("tile_width must be >= 0"), PM_ERR_ARG;
        if (opts->tile_width > 0) {
            if (n % opts->tile_width != 0)
                return pm::set_error("tile_width must divide the number of rays"), PM_ERR_ARG;
            if (opts->reorder != 0 || opts->kernel == PM_TRACE_PERSISTENT || opts->kernel == PM_TRACE_TWO_RAYS ||
                opts->kernel == PM_TRACE_SLICES)
                return pm::set_error("tile_width takes the rays in image order: no reorder, persistent, "
                                     "two-ray or slice kernel"),
                       PM_ERR_ARG;
        }
        a.link_set = opts->link_set;
        a.counters = opts->counters;
        a.tile_w = opts->tile_width;
        a.kernel = opts->kernel;
        a.refill = opts->refill;
        a.reorder = opts->reorder;
        a.block = opts->block;
        a.slice = opts->slice;
    }
    if (n >= (int64_t(1) << 31)) return pm::set_error("n must be below 2^31"), PM_ERR_ARG;
    return PM_OK;
}

int pm_trace_rays_ex(const pm_bvh *bvh, const float *rays, int64_t n, int32_t *hit, float *t,
                     const pm_trace_opts *opts, void *stream) {
    pm::TraceRange range_("pm_trace_rays_ex");
    PM_GUARD({
        if (!bvh) return pm::set_error("NULL bvh"), PM_ERR_ARG;
        pm::TraceArgs a;
        int rc = parse_trace(rays, n, hit, t, opts, a);
        if (rc) return rc;
        return pm::launch_trace(bvh, a, (hipStream_t)stream);
    })
}

int pm_trace_rays_noalloc(const pm_bvh *bvh, const float *rays, int64_t n, int32_t *hit, float *t,
                          const pm_trace_opts *opts, void *stream) {
    pm::TraceRange range_("pm_trace_rays_noalloc");
    PM_GUARD({
        if (n > (int64_t)PM_NOALLOC_MAX_RAYS)
            return pm::set_error("n = " + std::to_string(n) + " exceeds PM_NOALLOC_MAX_RAYS = " +
                                 std::to_string((int64_t)PM_NOALLOC_MAX_RAYS)),
                   PM_ERR_ARG;
        if (!bvh) return pm::set_error("NULL bvh"), PM_ERR_ARG;
        pm::TraceArgs a;
        int rc = parse_trace(rays, n, hit, t, opts, a);
        if (rc) return rc;
        if (a.reorder == 0) a.reorder = 1;
        if (a.tile_w != 0) return pm::set_error("tile_width does not apply to the bucketed trace"), PM_ERR_ARG;
        return pm::launch_trace_noalloc(bvh, a, (hipStream_t)stream);
    })
}

int pm_trace_rays_multi(const pm_bvh *bvh, int32_t n_batches, const pm_trace_batch *batches, void *stream) {
    pm::TraceRange range_("pm_trace_rays_multi");
    PM_GUARD({
        if (!bvh) return pm::set_error("NULL bvh"), PM_ERR_ARG;
        if (!batches) return pm::set_error("NULL batches"), PM_ERR_ARG;
        if (n_batches < 1 || n_batches > PM_MAX_TRACE_BATCHES)
            return pm::set_error("n_batches must be in [1, PM_MAX_TRACE_BATCHES]"), PM_ERR_ARG;
        pm::TraceArgs args[PM_MAX_TRACE_BATCHES];
        int scratch_users = 0;
        for (int32_t k = 0; k < n_batches; ++k) {
            const pm_trace_batch &bt = batches[k];
            if (bt.size < sizeof(pm_trace_batch)) return pm::set_error("pm_trace_batch.size too small"), PM_ERR_ARG;
            int rc = parse_trace(bt.rays, bt.n, bt.hit, bt.t, bt.opts, args[k]);
            if (rc) return pm::set_error("batch " + std::to_string(k) + ": " + pm::last_error()), rc;
            if (args[k].reorder != 0 || args[k].kernel == PM_TRACE_PERSISTENT) ++scratch_users;
        }
        if (scratch_users > 1)
            return pm::set_error("at most one batch may reorder or use the persistent kernel"), PM_ERR_ARG;
        return pm::launch_trace_multi(const_cast<pm_bvh *>(bvh), args, n_batches, (hipStream_t)stream);
    })
}

int pm_trace_rays(const pm_bvh *bvh, const float *rays, int64_t n, int32_t *hit, float *t, void *stream) {
    return pm_trace_rays_ex(bvh, rays, n, hit, t, nullptr, stream);
}

int pm_sppm_create(const pm_scene_desc *desc, const pm_sppm_params *params, void *stream, pm_sppm **out) {
    pm::TraceRange range_("pm_sppm_create");
    PM_GUARD({
        if (!out) return pm::set_error("out must not be NULL"), PM_ERR_ARG;
        *out = nullptr;
        return pm::sppm_create(desc, params, (hipStream_t)stream, out);
    })
}

int pm_sppm_destroy(pm_sppm *s) { PM_GUARD({ return pm::sppm_destroy(s); }) }

int pm_sppm_iterate(pm_sppm *s, int32_t n_iter, void *stream) {
    pm::TraceRange range_("pm_sppm_iterate");
    PM_GUARD({ return pm::sppm_iterate(s, n_iter, (hipStream_t)stream); })
}

int pm_sppm_resolve(pm_sppm *s, float *image, void *stream) {
    pm::TraceRange range_("pm_sppm_resolve");
    PM_GUARD({ return pm::sppm_resolve(s, image, (hipStream_t)stream); })
}

int pm_sppm_status(pm_sppm *s, void *stream) { PM_GUARD({ return pm::sppm_status(s, (hipStream_t)stream); }) }

int pm_sppm_get_views(pm_sppm *s, pm_sppm_views *v) { PM_GUARD({ return pm::sppm_views(s, v); }) }

int pm_sppm_get_stats(pm_sppm *s, pm_sppm_stats *out, int32_t reset, void *stream) {
    PM_GUARD({ return pm::sppm_get_stats(s, out, reset, (hipStream_t)stream); })
}

int pm_sppm_adjoint(pm_sppm *s, const float *dloss_dimage, const int32_t *param_mats, int32_t n_par, double *grad,
                    void *stream) {
    pm::TraceRange range_("pm_sppm_adjoint");
    PM_GUARD({ return pm::sppm_adjoint(s, dloss_dimage, param_mats, n_par, grad, (hipStream_t)stream); })
}

int pm_sppm_save(pm_sppm *s, void *buf, uint64_t *size, void *stream) {
    PM_GUARD({ return pm::sppm_save(s, buf, size, (hipStream_t)stream); })
}

int pm_sppm_load(pm_sppm *s, const void *buf, uint64_t size, void *stream) {
    PM_GUARD({ return pm::sppm_load(s, buf, size, (hipStream_t)stream); })
}

int pm_render(const pm_scene_desc *desc, const pm_sppm_params *params, int32_t K, float *image, void *stream) {
    pm::TraceRange range_("pm_render");
    PM_GUARD({
        if (K < 1 || !image) return pm::set_error("K must be >= 1 and image non-NULL"), PM_ERR_ARG;
        int rc = pm::sppm_validate(desc, params);
        if (rc) return rc;
        pm_sppm *s = nullptr;
        hipStream_t st = (hipStream_t)stream;
        if ((rc = pm::sppm_create(desc, params, st, &s))) return rc;
        if (!(rc = pm::sppm_iterate(s, K, st)))
            if (!(rc = pm::sppm_resolve(s, image, st))) rc = pm::sppm_status(s, st);
        (void)hipStreamSynchronize(st);
        pm::sppm_destroy(s);
        return rc;
    })
}

int pm_batch_create(const pm_scene_desc *const *descs, const pm_sppm_params *const *params, int32_t n_scenes,
                    const pm_batch_opts *opts, void *stream, pm_batch **out) {
    pm::TraceRange range_("pm_batch_create");
    PM_GUARD({
        if (!out) return pm::set_error("out must not be NULL"), PM_ERR_ARG;
        *out = nullptr;
        return pm::batch_create(descs, params, n_scenes, opts, (hipStream_t)stream, out);
    })
}

int pm_batch_destroy(pm_batch *b) { PM_GUARD({ return pm::batch_destroy(b); }) }

int pm_batch_iterate(pm_batch *b, int32_t n_iter, void *stream) {
    pm::TraceRange range_("pm_batch_iterate");
    PM_GUARD({ return pm::batch_iterate(b, n_iter, (hipStream_t)stream); })
}

int pm_batch_resolve(pm_batch *b, float *const *images, void *stream) {
    pm::TraceRange range_("pm_batch_resolve");
    PM_GUARD({ return pm::batch_resolve(b, images, (hipStream_t)stream); })
}

int pm_batch_status(pm_batch *b, void *stream) { PM_GUARD({ return pm::batch_status(b, (hipStream_t)stream); }) }

int pm_batch_get_info(const pm_batch *b, pm_batch_info *info) { PM_GUARD({ return pm::batch_info(b, info); }) }

int pm_batch_get_views(pm_batch *b, int32_t scene, pm_sppm_views *v) {
    PM_GUARD({ return pm::batch_views(b, scene, v); })
}

int pm_render_batch(const pm_scene_desc *const *descs, const pm_sppm_params *const *params, int32_t n_scenes,
                    int32_t K, float *const *images, const pm_batch_opts *opts, void *stream) {
    pm::TraceRange range_("pm_render_batch");
    PM_GUARD({
        if (K < 1 || !images) return pm::set_error("K must be >= 1 and images non-NULL"), PM_ERR_ARG;
        pm_batch *b = nullptr;
        hipStream_t st = (hipStream_t)stream;
        int rc = pm::batch_create(descs, params, n_scenes, opts, st, &b);
        if (rc) return rc;
        if (!(rc = pm::batch_iterate(b, K, st)))
            if (!(rc = pm::batch_resolve(b, images, st))) rc = pm::batch_status(b, st);
        (void)hipStreamSynchronize(st);
        pm::batch_destroy(b);
        return rc;
    })
}

}  // extern "C"

int pm_probe_chase(const uint32_t *rows, int32_t log2_rows, int64_t n_lanes, int32_t steps, uint32_t *out,
                   void *stream) {
    PM_GUARD({
        if (!rows || !out) return pm::set_error("rows and out must not be NULL"), PM_ERR_ARG;
        if (log2_rows < 1 || log2_rows > 28) return pm::set_error("log2_rows must be in [1, 28]"), PM_ERR_ARG;
        if (n_lanes < 1 || n_lanes >= (int64_t(1) << 31))
            return pm::set_error("n_lanes must be in [1, 2^31)"), PM_ERR_ARG;
        if (steps < 1) return pm::set_error("steps must be at least 1"), PM_ERR_ARG;
        return pm::launch_chase(rows, log2_rows, (uint32_t)n_lanes, (uint32_t)steps, out, (hipStream_t)stream);
    })
}

int pm_probe_stream(const void *src, void *dst, uint64_t n_bytes, int32_t mode, uint32_t *out, void *stream) {
    PM_GUARD({
        if (mode != 0 && mode != 1) return pm::set_error("mode must be 0 (copy) or 1 (read)"), PM_ERR_ARG;
        if (!src || (mode == 0 && !dst) || (mode == 1 && !out))
            return pm::set_error("src, and dst (copy) or out (read), must not be NULL"), PM_ERR_ARG;
        if (n_bytes == 0 || n_bytes % 64 != 0) return pm::set_error("n_bytes must be a positive multiple of 64"), PM_ERR_ARG;
        if (((uintptr_t)src | (uintptr_t)dst) % 16 != 0) return pm::set_error("src and dst must be 16-byte aligned"), PM_ERR_ARG;
        return pm::launch_stream(src, dst, n_bytes, mode, out, (hipStream_t)stream);
    })
}
