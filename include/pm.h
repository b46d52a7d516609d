/*
 * pm.h -- C ABI of the MI355X photon-mapping library (libpm.so).
 *
 * The library implements the data-parallel hot path of a stochastic
 * progressive photon mapping renderer (Hachisuka, "Implementing a
 * Photorealistic Rendering System using GLSL", EGSR 2015): a multiple-threaded
 * BVH (Sec. 3.1) traversed stacklessly with closest-hit ray/triangle tests,
 * the float-only combined-MLCG random number generator (Sec. 3.2), photon
 * tracing with Russian roulette and path regeneration (Sec. 2, Sec. 3.3),
 * and the range query plus progressive radius/flux update of each iteration
 * (Sec. 2).
 *
 * Conventions
 *   - Every call returns PM_OK (0) or a negative pm_status.  On error
 *     pm_last_error() returns a thread-local message; nothing was enqueued
 *     if the error is PM_ERR_ARG (arguments are validated on the host first).
 *   - "host" pointers are ordinary CPU memory read during the call; "device"
 *     pointers are HIP device allocations (e.g. PyTorch tensors) owned by the
 *     caller unless stated otherwise.
 *   - `stream` is a hipStream_t passed as void* (NULL = the null stream).
 *     Device work is enqueued asynchronously on it; the caller synchronises.
 *   - Option/parameter structs start with `uint32_t size` = sizeof(struct),
 *     so later versions can extend them.
 *   - Handles are not thread-safe; use one handle per stream.
 *   - No C++ exception crosses this boundary.
 */
#ifndef PM_H
#define PM_H

#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

#define PM_ABI_VERSION 2

#if defined(__GNUC__)
#define PM_API __attribute__((visibility("default")))
#else
#define PM_API
#endif

typedef enum {
    PM_OK = 0,
    PM_ERR_ARG = -1,      /* invalid argument (nothing enqueued) */
    PM_ERR_HIP = -2,      /* HIP runtime error */
    PM_ERR_OVERFLOW = -3, /* a fixed-capacity device buffer overflowed, or a
                             fixed-point flux sum left the range of u64 */
    PM_ERR_STATE = -4,    /* call not valid in the handle's current state */
    PM_ERR_NOMEM = -5     /* host or device allocation failed */
} pm_status;

/* Material kinds (diffuse is two-sided Lambertian; emission is one-sided,
 * along the geometric normal n = normalize((v1-v0) x (v2-v0))). */
enum { PM_MAT_DIFFUSE = 0, PM_MAT_MIRROR = 1, PM_MAT_GLASS = 2 };

typedef struct pm_bvh pm_bvh;
typedef struct pm_sppm pm_sppm;

/* ABI version of the loaded library (PM_ABI_VERSION at build time). */
PM_API int pm_abi_version(void);

/* Thread-local description of the last error on this thread ("" if none). */
PM_API const char *pm_last_error(void);

/* ------------------------------------------------------------------ */
/* Multiple-threaded BVH (Sec. 3.1)                                    */
/* ------------------------------------------------------------------ */
typedef struct {
    uint32_t size;     /* sizeof(pm_bvh_opts) */
    int32_t bins;      /* SAH bins per axis, 2..256 (default 32) */
    int32_t max_leaf;  /* triangles per leaf, 1..7 (default 4) */
    int32_t n_threads; /* host build threads, 0 = all */
    float trav_cost;   /* SAH cost of a node visit relative to a triangle
                          test (0 = default 1; range (0, 64]) */
    int32_t builder;   /* PM_BUILD_*: pm_build_bvh only */
    float split_alpha; /* host SAH build only: spatial splits (Stich et al.
                          2009) are tried at a node when its best object
                          split leaves children whose boxes overlap by more
                          than split_alpha x the scene box's surface area;
                          a triangle may then be referenced by several
                          leaves (n_refs > n_tri; spatial splits stop
                          adding references at 8 x n_tri, each subtree
                          holding its share of that allowance, so the
                          build stays deterministic).  0 = none
                          (default); range [0, 1] */
} pm_bvh_opts;

/* BVH builders.  HOST_SAH: binned SAH on the host threads, then threading and
 * upload (Sec. 3.1).  GPU_LBVH: on the device from sorted 30-bit Morton codes
 * of the triangle centres (a linear BVH, the GPU build named as future work
 * in Sec. 4.1), subtrees of at most max_leaf triangles collapsed into leaves,
 * threaded into the same six link sets; much faster to build, usually slower
 * to traverse.  Both give identical traversal results. */
enum { PM_BUILD_HOST_SAH = 0, PM_BUILD_GPU_LBVH = 1 };

typedef struct {
    uint32_t size;        /* sizeof(pm_bvh_info) */
    int64_t n_tri;
    int64_t n_refs;       /* triangle records in leaf order (n_tri without
                             spatial splits; each triangle at least once) */
    int64_t n_nodes;      /* nodes of the binary tree (each stored once per link set) */
    int64_t n_leaves;
    int32_t depth;
    int32_t max_leaf;
    double sah_cost;      /* C_trav = C_isect = 1, normalised by the root area */
    int64_t device_bytes; /* nodes (6 link sets x 16 B) + triangle records (48 B) */
    double build_ms;      /* host build + threading time */
    float grid_lo[3];     /* node boxes: coordinate = grid_lo + q * grid_step */
    float grid_step[3];
} pm_bvh_info;

/* Build the BVH on the host (top-down binned SAH; Sec. 3.1 builds top-down
 * with the SAH on the CPU), thread it six times with children pre-sorted
 * along +x,-x,+y,-y,+z,-z (the multiple-threaded BVH), and copy it to the
 * device on `stream`.
 *   tri_verts  host, float32 [n_tri][3][3] vertex positions (finite)
 *   tri_mat    host, uint32 [n_tri] material ids (may be NULL: all 0)
 *   opts       may be NULL (defaults above)
 *   out        receives a library-owned handle; free with pm_bvh_destroy.
 * Errors: PM_ERR_ARG for n_tri < 1, n_tri >= 2^28, non-finite vertices, bad
 * options, or spatial splits that make 2^28 or more triangle records;
 * PM_ERR_HIP / PM_ERR_NOMEM for device failures. */
PM_API int pm_build_bvh(const float *tri_verts, const uint32_t *tri_mat, int64_t n_tri, const pm_bvh_opts *opts,
                 void *stream, pm_bvh **out);

/* Host-only build (no device needed), for inspection and tests.  Two-phase:
 * call with nodes == tris == NULL to learn *n_nodes (and, with info,
 * info->n_refs); then call again with
 *   nodes  host, [6][n_nodes][4] 32-bit words per link set s (0:+x 1:-x 2:+y
 *          3:-y 4:+z 5:-z), node i in that set's preorder: its padded box
 *          rounded outward to 16-bit grid coordinates, one word per axis
 *          (lo.x | hi.x << 16, lo.y | hi.y << 16, lo.z | hi.z << 16; see
 *          info->grid_*), then the
 *          link word: an inner node stores its skip link (preorder index after
 *          its subtree, n_nodes at the end; its hit link is i + 1); a leaf has
 *          bit 31 set and first_tri << 3 | count (both of its links are i + 1)
 *   tris   host, [n_refs][12] 32-bit words in leaf order: v0.xyz, v1.xyz,
 *          v2.xyz (float bits, the vertices as given), original index,
 *          material, 0.  n_refs = n_tri unless opts->split_alpha > 0.
 * The build is deterministic: both calls give the same BVH. */
PM_API int pm_build_bvh_host(const float *tri_verts, const uint32_t *tri_mat, int64_t n_tri, const pm_bvh_opts *opts,
                      int64_t *n_nodes, uint32_t *nodes, uint32_t *tris, pm_bvh_info *info);

PM_API int pm_bvh_destroy(pm_bvh *bvh);
PM_API int pm_bvh_get_info(const pm_bvh *bvh, pm_bvh_info *info);

/* Copy a device BVH to host memory, in the layout of pm_build_bvh_host
 * (nodes [6][n_nodes][4] words, tris [n_refs][12] words; either may be NULL).
 * Synchronises `stream`.  Errors: PM_ERR_ARG for a NULL bvh. */
PM_API int pm_bvh_download(const pm_bvh *bvh, uint32_t *nodes, uint32_t *tris, void *stream);

/* Closest hit of every ray (the traversal loop of Sec. 3.1, Fig. "mtbvh").
 *   rays  device, float32 [n][8] = o.xyz, tmin, d.xyz, tmax
 *   hit   device, int32 [n]: ORIGINAL index of the closest triangle with
 *         tmin < t < tmax (ties in t go to the lower index), or -1
 *   t     device, float32 [n]: its distance along d, +inf on a miss
 * The result is independent of which link set is traversed.
 * Concurrent calls on one BVH must be on the same stream (a per-BVH work
 * counter is reset by each call).
 * Errors: PM_ERR_ARG for n < 0, n >= 2^31 or NULL pointers with n > 0. */
PM_API int pm_trace_rays(const pm_bvh *bvh, const float *rays, int64_t n, int32_t *hit, float *t, void *stream);

/* Traversal kernels: one ray per lane for the whole walk; persistent
 * wavefronts whose finished lanes take new rays from a work counter; one
 * ray per lane testing nodes i and i+1 from one memory round trip; one ray
 * per lane with leaf tests postponed until the wavefront's lanes hold leaf
 * hits together (box visits and triangle tests then run in separate phases
 * instead of sharing each iteration); two consecutive rays per lane walked
 * in lockstep (two node loads in flight per lane); or a wavefront's rays as
 * one packet (the wavefront follows one node index, taking the hit link when
 * any lane's box test passes; used when all its rays share a link set, else
 * the per-ray walk); or the postponed walk over a slice of consecutive rays
 * per wavefront (the order of reorder, else the input order), a lane taking
 * the slice's next ray when its own has ended.  All return the same
 * result. */
enum {
    PM_TRACE_AUTO = 0,
    PM_TRACE_PER_RAY = 1,
    PM_TRACE_PERSISTENT = 2,
    PM_TRACE_PAIRED = 3,
    PM_TRACE_POSTPONED = 4,
    PM_TRACE_TWO_RAYS = 5,
    PM_TRACE_PACKET = 6,
    PM_TRACE_SLICES = 7
};

typedef struct {
    uint32_t size;      /* sizeof(pm_trace_opts) */
    int32_t link_set;   /* -1: pick by ray direction (MTBVH); 0..5: force one
                           link set for every ray (single threaded BVH) */
    uint32_t *counters; /* optional device [n][2]: AABB tests, triangle tests */
    int32_t kernel;     /* PM_TRACE_* */
    int32_t refill;     /* persistent kernel: idle lanes that trigger a refill
                           (1..64; 0 = default 16).  Postponed kernel: lanes
                           of a wavefront still searching for a leaf hit at
                           which the held leaves are tested (0..63; 0 = only
                           once no lane is searching); the same for the slice
                           kernel, whose idle lanes also take new rays then */
    int32_t reorder;    /* 1: first bucket the rays by (origin cell of a 16^3
                           grid over the scene in Morton order, then link set)
                           and trace them in that order; 2: the same with a
                           32^3 grid and the signs of the two minor direction
                           components (for incoherent batches; results are
                           unchanged and written to each ray's own slot).
                           Uses a library-owned scratch of 12 B per ray, kept
                           with the BVH for later calls (grown when a call has
                           more rays; the growth waits for the call's stream).
                           Reordered calls on one BVH share that scratch, so
                           they must not overlap on different streams. */
    int32_t block;      /* threads per workgroup of every kernel but the
                           persistent one: 64, 128 or 256 (0 = default) */
    int32_t tile_width; /* > 0: the rays are the pixels of an image this
                           wide in row-major order (n a multiple of it); each
                           wavefront takes an 8x8 pixel tile.  Not with
                           reorder, the persistent, the two-ray or the slice
                           kernel. */
    int32_t slice;      /* slice kernel: rays per wavefront (0 = enough
                           wavefronts for two per wavefront slot of the
                           device, at least 64 rays each) */
} pm_trace_opts;

/* pm_trace_rays with options (ablation of the link-set choice; per-ray
 * traversal statistics for the algorithmic-bytes roofline). */
PM_API int pm_trace_rays_ex(const pm_bvh *bvh, const float *rays, int64_t n, int32_t *hit, float *t,
                     const pm_trace_opts *opts, void *stream);

/* For callers that cannot allocate device memory (code under HIP graph
 * capture, tight serving loops, harnesses that forbid hipMalloc): the
 * bucketed trace of pm_trace_rays_ex (reorder 1 or 2; 0 or NULL opts mean 1)
 * with its scratch in a static per-device array of the library instead of
 * the BVH handle's growable buffer.  The call allocates and frees nothing.
 *   rays, hit, t  device buffers as for pm_trace_rays (caller-owned)
 *   n             0 .. PM_NOALLOC_MAX_RAYS
 * The array (12 B per ray of PM_NOALLOC_MAX_RAYS plus 9.4 MB of bucket
 * arrays, about 60 MB) is set aside on every device the library's code is
 * loaded on and held until the process ends; its address is looked up on the
 * first call on each device.  Every call on one device shares it and it keeps
 * the last call's contents (the bucket counts are rewritten by kernels at
 * the start of each call): calls that overlap on one device, on different
 * streams or host threads, race and give wrong results.  Results equal those
 * of pm_trace_rays_ex with the same options.  The BVH must live on the current
 * device.  Asynchronous on `stream`.
 * Errors: PM_ERR_ARG for n above PM_NOALLOC_MAX_RAYS, reorder other than
 * 0..2, tile_width, another device or the rules of pm_trace_rays_ex. */
#define PM_NOALLOC_MAX_RAYS (1 << 22)
PM_API int pm_trace_rays_noalloc(const pm_bvh *bvh, const float *rays, int64_t n, int32_t *hit, float *t,
                                 const pm_trace_opts *opts, void *stream);

/* One batch of rays for pm_trace_rays_multi: arguments as for
 * pm_trace_rays_ex (opts may be NULL). */
typedef struct {
    uint32_t size;             /* sizeof(pm_trace_batch) */
    const float *rays;         /* device, float32 [n][8] */
    int64_t n;
    int32_t *hit;              /* device, int32 [n] */
    float *t;                  /* device, float32 [n] */
    const pm_trace_opts *opts; /* may be NULL */
} pm_trace_batch;

#define PM_MAX_TRACE_BATCHES 8

/* Several ray batches on one BVH (each as pm_trace_rays_ex would trace it),
 * run concurrently: batch 0 on `stream`, batch k > 0 on a stream the BVH
 * handle owns, which first waits for the work already enqueued on `stream`;
 * `stream` then waits for every batch, so work enqueued on it after the call
 * sees all results.  Kernels of different batches share the device (one
 * batch's last wavefronts leave room for another's), so the call takes less
 * time than the batches one after another; results are the same.  Two
 * batches of which one is bucketed (reorder) with the postponed kernel and
 * the other is traced as packets over image tiles, with equal workgroup
 * sizes and both with or without counters, go out on `stream` alone: the
 * bucketing, then one launch whose first workgroups walk the bucketed batch
 * and whose last ones take the tiles (dispatched as the walk's last
 * wavefronts drain).  The
 * batches' output arrays must not overlap.  At most one batch may use the
 * handle's scratch (reorder != 0 or the persistent kernel).  Calls on one
 * handle must be on the same stream or not overlap (the handle's streams are
 * shared).  Errors: PM_ERR_ARG for n_batches outside [1, PM_MAX_TRACE_BATCHES],
 * NULL bvh or batches, a batch that pm_trace_rays_ex would reject, or two
 * batches using the scratch; all checked before anything is enqueued. */
PM_API int pm_trace_rays_multi(const pm_bvh *bvh, int32_t n_batches, const pm_trace_batch *batches, void *stream);

/* ------------------------------------------------------------------ */
/* Stochastic progressive photon mapping (Sec. 2)                      */
/* ------------------------------------------------------------------ */
typedef struct {
    uint32_t size;            /* sizeof(pm_scene_desc) */
    const float *tri_verts;   /* host [n_tri][3][3] */
    const uint32_t *tri_mat;  /* host [n_tri] */
    int64_t n_tri;
    const int32_t *mat_type;  /* host [n_mat] PM_MAT_* */
    const float *mat_rho;     /* host [n_mat] diffuse albedo in [0,1) */
    const float *mat_q;       /* host [n_mat] Russian-roulette survival
                                 probability in [0,1] (nominal albedo, held
                                 fixed); 0 stores a photon and ends the path */
    const float *mat_Le;      /* host [n_mat] emitted radiance, >= 0 */
    const float *mat_ior;     /* host [n_mat] index of refraction (glass) */
    int32_t n_mat;
    float cam_pos[3], cam_look[3], cam_up[3];
    float tan_half_fov;       /* tan(vertical field of view / 2) */
    int32_t width, height;
    const pm_bvh *bvh;        /* optional BVH already built over tri_verts */
} pm_scene_desc;

typedef struct {
    uint32_t size;            /* sizeof(pm_sppm_params) */
    int64_t n_photons;        /* photon paths per iteration, 1..2^26 */
    double alpha;             /* radius reduction, (0,1] */
    double r0;                /* initial radius, > 0 */
    uint64_t seed;
    int32_t max_eye_depth;    /* specular eye-path length cap (16) */
    int32_t max_photon_bounces; /* photon path length cap (32) */
    int32_t fixed_shift;      /* flux fixed point: value * 2^shift (40); a term
                                 or a pixel's sum of 2^64 or more sets the
                                 flux-overflow flag */
    int32_t store_factor;     /* photon store capacity = n_photons * factor (8) */
    int32_t record_iterations; /* > 0: record what pm_sppm_adjoint needs for
                                  up to this many iterations (8 B per pixel
                                  per iteration, plus 10 B x n_photons x
                                  max_photon_bounces of replay scratch);
                                  needs gather_mode 0, at most 256 materials
                                  and fewer than 2^24 pixels */
    int32_t photon_kernel;    /* PM_PHOTON_*: 0 = default (two-phase
                                 regeneration; a batch member: regeneration) */
    int32_t refill;           /* regeneration: idle lanes of a wave that
                                 trigger taking new paths (1..64; 0 = 32) */
    int32_t single_link_set;  /* 0: each ray walks the link set of its
                                 direction (MTBVH, Sec. 3.1); s + 1 (1..6):
                                 every ray walks link set s, i.e. a single
                                 threaded BVH (the paper's TBVH comparison).
                                 Results are identical; only speed differs. */
    int32_t gather_mode;      /* PM_GATHER_*: the range query's estimator */
    int32_t pass_threads;     /* PM_PHOTON_PASSES: threads (path slots) per
                                 pass, 1..2^26; 0 = one per pixel, capped at
                                 2^26 (the paper's setting).  Must be 0 for
                                 the other photon kernels. */
    int32_t passes;           /* PM_PHOTON_PASSES: one-bounce passes per
                                 iteration, 1..1024; 0 = ceil(n_photons /
                                 threads) + 8.  Must be 0 for the other
                                 photon kernels. */
    int32_t profile;          /* PM_PROFILE_* flags (single-scene handles;
                                 0 for a batch member); see pm_sppm_get_stats */
} pm_sppm_params;

/* Profiling of the iterations (pm_sppm_params.profile), read with
 * pm_sppm_get_stats.  Results are unchanged by either flag.
 * COUNT: the eye pass, the regenerating photon pass and the exact range query
 *   run instrumented variants that count their work (slower; needs the
 *   default photon kernel and gather_mode EXACT).
 * TIME: HIP events around each stage; every iteration then waits for its end
 *   on the host, so iterations no longer queue behind each other. */
enum { PM_PROFILE_COUNT = 1, PM_PROFILE_TIME = 2 };

/* Range query.  EXACT: every photon inside a hit point's disc, found through
 * a hashed grid with cell edge R_max (1 + 2^-5) (2 R_max (1 + 2^-10) when the
 * scene would span more than 4096 such cells) and 2^bits entries,
 * bits = clamp(ceil(log2(4 n_photons)), 12, 24).  STOCHASTIC: the paper's
 * stochastic spatial hashing (Sec. 3.4) on a grid of cell edge
 * 2 R_max (1 + 2^-10) and the same table: each
 * entry keeps one photon, the one of smallest (random depth, path * 32 +
 * bounce), with the depth drawn for each photon from its own counter-keyed
 * stream, and a hit point counts that photon, when inside its disc, once per
 * photon the entry received.  The estimate is unbiased for the exact query
 * and independent of thread order; it needs no sort.  Not supported with
 * record_iterations > 0 (the adjoint) or in a batch. */
enum { PM_GATHER_EXACT = 0, PM_GATHER_STOCHASTIC = 1 };

/* Photon pass scheduling (results are identical): one lane traces one whole
 * path (PER_PATH); persistent lanes trace one bounce per step and switch to a
 * new path as soon as theirs ends (REGEN, the paper's photon path
 * regeneration of Sec. 3.3 inside one launch); or the paper's schedule as
 * written (PASSES): each launch is one pass in which every thread moves its
 * path by one bounce, so it stores at most one photon, and a thread whose
 * path was killed or left the scene starts the next path in the following
 * pass.  Path state stays in device memory between passes (56 B per thread).
 * The passes are enqueued without any host synchronisation, so their number
 * is fixed in advance (`passes`); one last launch finishes whatever paths the
 * passes left (views: photon_count[3] counts them).  RAY_REGEN: regeneration
 * at ray granularity: persistent lanes each walk their own ray, and once
 * `refill` lanes of a wavefront wait, those lanes shade their hits and start
 * the next ray of their path (or a new path) while the others keep walking,
 * so a wavefront does not wait for its longest walk at every bounce.
 * POOL: regeneration from a queue in LDS: each wavefront keeps up to 128
 * started paths in its own slice of LDS; when lanes are idle and the queue
 * is short, the whole wavefront starts 64 new paths at once and appends
 * them, compacted by ballot rank, and every idle lane then takes a queued
 * path, so the lanes of a bounce step stay full.
 * TWO_PHASE (the default of single-scene handles): regeneration in two
 * launches.  The first stops once the path counter has run out and at most
 * 32 lanes of a wavefront still hold a path; those paths wait in a queue in
 * device memory (56 B per path, at most one per lane of the launch) and the
 * second launch continues them.  A path that reflects inside a glass object
 * can run to max_photon_bounces, so the last paths of a pass leave the device
 * almost idle: on a pipelined handle the second launch runs on a stream of
 * its own, beside the next iteration's first launch. */
enum {
    PM_PHOTON_AUTO = 0,
    PM_PHOTON_PER_PATH = 1,
    PM_PHOTON_REGEN = 2,
    PM_PHOTON_PASSES = 3,
    PM_PHOTON_RAY_REGEN = 4,
    PM_PHOTON_POOL = 5,
    PM_PHOTON_TWO_PHASE = 6
};

/* Create a renderer: uploads the scene (building a BVH if desc->bvh is NULL)
 * and allocates the per-pixel state (N = 0, R^2 = r0^2, tau = 0, D = 0).
 * The handle owns all device buffers it allocates. */
PM_API int pm_sppm_create(const pm_scene_desc *desc, const pm_sppm_params *params, void *stream, pm_sppm **out);
PM_API int pm_sppm_destroy(pm_sppm *s);

/* Enqueue n_iter iterations (eye pass, photon pass, hashed-grid build,
 * range query, progressive update).  Counts stay on the device; a photon
 * store overflow sets a sticky device flag reported by pm_sppm_status.
 * Within an iteration the eye pass runs on a stream the handle owns, forked
 * from `stream` and joined back to it by events before the range query, so
 * everything enqueued later on `stream` sees the finished iteration. */
PM_API int pm_sppm_iterate(pm_sppm *s, int32_t n_iter, void *stream);

/* Radiance estimate of the iterations so far into `image` (device, float32
 * [height][width]): tau / (pi R^2 K) + D / K.  PM_ERR_STATE if K == 0. */
PM_API int pm_sppm_resolve(pm_sppm *s, float *image, void *stream);

/* Synchronise `stream` and report sticky device errors: PM_ERR_OVERFLOW for a
 * photon store overflow (raise store_factor) or a flux fixed-point overflow
 * (lower fixed_shift); pm_last_error() says which. */
PM_API int pm_sppm_status(pm_sppm *s, void *stream);

/* Checkpoint of an SPPM handle: the per-pixel state (N, R^2, tau, D as
 * float64), the iteration count K, the sticky overflow flag and, for a
 * handle that records iterations for the adjoint, the radii of the recorded
 * iterations.  Every random stream is keyed by (seed, kind, iteration,
 * index) (Sec. 3.2 with counter-keyed seeding), so a handle loaded from a
 * checkpoint taken after K iterations continues exactly as the saved run
 * would have: further iterations, images and gradients are bit-identical.
 *   buf   host memory owned by the caller; NULL queries the size
 *   size  in: capacity of buf in bytes; out: bytes written (or required)
 * Synchronises `stream`.  Errors: PM_ERR_ARG (NULL handle or size pointer;
 * buf smaller than required, with the required size in *size),
 * PM_ERR_STATE (a member of a batch). */
PM_API int pm_sppm_save(pm_sppm *s, void *buf, uint64_t *size, void *stream);

/* Restore a checkpoint into a handle created with the same scene and
 * parameters (checked through a fingerprint of the scene description and the
 * pixel count, photon count, seed, alpha, r0, fixed-point shift, path-length
 * caps, recorded-iteration count and gather mode).  On any mismatch, or a truncated or
 * foreign buffer, returns PM_ERR_ARG and leaves the handle unchanged.  The
 * photon store and hashed grid are rebuilt by the next iteration.
 * Synchronises `stream`. */
PM_API int pm_sppm_load(pm_sppm *s, const void *buf, uint64_t size, void *stream);

/* create -> K x iterate -> resolve -> status -> destroy. */
PM_API int pm_render(const pm_scene_desc *desc, const pm_sppm_params *params, int32_t K, float *image, void *stream);

/* Work counts and stage times of the profiled iterations (sums since the
 * handle was created or last reset), the per-unit counts of the stages'
 * algorithmic-bytes rooflines. */
typedef struct {
    uint32_t size;                 /* sizeof(pm_sppm_stats) */
    int64_t counted_iterations;    /* iterations run with PM_PROFILE_COUNT */
    uint64_t eye_paths, eye_rays, eye_box_tests, eye_tri_tests;
    uint64_t photon_paths, photon_rays, photon_box_tests, photon_tri_tests, photons_stored;
    uint64_t gather_hit_points;    /* valid hit points queried */
    uint64_t gather_buckets;       /* distinct buckets visited */
    uint64_t gather_examined;      /* photons in those buckets */
    uint64_t gather_accepted;      /* photons inside a disc from the eye's side (sum of M) */
    int64_t timed_iterations;      /* iterations run with PM_PROFILE_TIME */
    double ms_eye;                 /* eye pass + R_max (on the side stream, beside the photon pass) */
    double ms_photon;              /* photon pass */
    double ms_grid;                /* hashed grid: count, scan, scatter (after the eye pass joins) */
    double ms_gather;              /* range query */
    double ms_update;              /* progressive update */
    double ms_iteration;           /* whole iteration */
} pm_sppm_stats;

/* Copies the counts and times into *out (synchronises `stream`); reset != 0
 * then clears them.  PM_ERR_ARG: NULL pointers, out->size too small. */
PM_API int pm_sppm_get_stats(pm_sppm *s, pm_sppm_stats *out, int32_t reset, void *stream);

/* Gradient of a scalar image loss by replay (the adjoint of the K iterations
 * run so far; requires params.record_iterations >= K).
 *   dloss_dimage  device float32 [height][width]: dLoss/dL_p
 *   param_mats    host int32 [n_par]: materials whose diffuse albedo is a
 *                 parameter (each with rho > 0; n_par < 256)
 *   grad          device float64 [n_par + 1]: dLoss/drho for each listed
 *                 material, then dLoss/dLe of the single emitting material (0
 *                 when the scene has no or several emitting materials)
 * Sampling is held fixed (Russian roulette uses the nominal q), so every path,
 * hit point and radius is replayed from its counter-keyed random stream and
 * only the flux terms are differentiated.  Every sum is an integer sum of
 * terms rounded one by one (a per-iteration power-of-two scale keeps each
 * term below 2^39 units), so the gradient is bit-reproducible: it does not
 * depend on the order of atomics or of photons in their buckets.
 * Asynchronous on `stream`.
 * Errors: PM_ERR_STATE if nothing was recorded; PM_ERR_ARG for bad ids. */
PM_API int pm_sppm_adjoint(pm_sppm *s, const float *dloss_dimage, const int32_t *param_mats, int32_t n_par,
                           double *grad, void *stream);

/* Device buffers of a handle, for inspection (owned by the handle, valid
 * until it is destroyed). */
typedef struct {
    uint32_t size;            /* sizeof(pm_sppm_views) */
    int64_t n_pixels;
    int32_t iterations;       /* K so far */
    int64_t photon_capacity;
    int64_t table_size;       /* hashed-grid buckets */
    double *N, *R2, *tau, *D; /* [n_pixels] */
    float *hp_pos;            /* [n_pixels][4]: x, y, z, W*rho/pi */
    float *hp_nrm;            /* [n_pixels][4]: n (toward the eye), int bits: material or -1 */
    float *photons;           /* [capacity][8]: x, y, z, phi, w.xyz, bits: path << 5 | bounce */
    uint32_t *photon_count;   /* [4]: photons stored in the last iteration,
                                 overflow flag (sticky), paths handed out,
                                 and (PM_PHOTON_PASSES) paths the passes left
                                 unfinished or unstarted */
    uint32_t *gather_M;       /* [n_pixels] photons found in the last iteration */
    uint64_t *gather_Phi;     /* [n_pixels] their fixed-point flux */
} pm_sppm_views;

PM_API int pm_sppm_get_views(pm_sppm *s, pm_sppm_views *v);

/* ------------------------------------------------------------------ */
/* Batched rendering: many scenes of uneven size in one launch per stage */
/* ------------------------------------------------------------------ */
typedef struct pm_batch pm_batch;

typedef struct {
    uint32_t size;     /* sizeof(pm_batch_opts) */
    int32_t chunk;     /* elements (pixels, paths, photons) per work item; 0 = 1024 */
    int32_t block;     /* workgroup size: 0 (= 256), 128 or 256 */
    int32_t autotune;  /* 1: time every (chunk, block) candidate and keep the fastest
                          (result cached on disk: $PM_AUTOTUNE_CACHE, default
                          ~/.cache/pm_autotune.txt); overrides chunk/block */
    int32_t use_graph; /* 1: capture one iteration as a hipGraph and replay it */
} pm_batch_opts;

typedef struct {
    uint32_t size;     /* sizeof(pm_batch_info) */
    int32_t n_scenes, iterations, chunk, block, uses_graph, tuned_from_cache;
    int32_t n_candidates;          /* autotuner candidates timed (<= 8) */
    int32_t cand_chunk[8], cand_block[8];
    double cand_ms[8];             /* ms per iteration of each candidate */
} pm_batch_info;

/* Create a batch of SPPM renderers (one per scene; descs[i]/params[i] as for
 * pm_sppm_create, record_iterations ignored).  Every stage of an iteration is
 * one persistent launch for all scenes: workgroups take (scene, chunk) items
 * from a device work counter.  The library owns all device buffers.  Every
 * scene must use the exact gather and photon_kernel 0, 1 or 2 (the batch
 * schedules its own photon stage). */
PM_API int pm_batch_create(const pm_scene_desc *const *descs, const pm_sppm_params *const *params, int32_t n_scenes,
                           const pm_batch_opts *opts, void *stream, pm_batch **out);
PM_API int pm_batch_destroy(pm_batch *b);
/* Enqueue n_iter iterations of every scene (graph replays when use_graph). */
PM_API int pm_batch_iterate(pm_batch *b, int32_t n_iter, void *stream);
/* images: host array of n_scenes device pointers, each float32 [height][width]. */
PM_API int pm_batch_resolve(pm_batch *b, float *const *images, void *stream);
/* Synchronise and report sticky device errors of every scene. */
PM_API int pm_batch_status(pm_batch *b, void *stream);
PM_API int pm_batch_get_info(const pm_batch *b, pm_batch_info *info);
/* Device buffers of scene i (bucket fields refer to the batch's shared arrays). */
PM_API int pm_batch_get_views(pm_batch *b, int32_t scene, pm_sppm_views *v);
/* create -> K iterations -> resolve -> status -> destroy. */
PM_API int pm_render_batch(const pm_scene_desc *const *descs, const pm_sppm_params *const *params, int32_t n_scenes,
                           int32_t K, float *const *images, const pm_batch_opts *opts, void *stream);

/* ------------------------------------------------------------------------ */
/* Diagnostics                                                              */
/* ------------------------------------------------------------------------ */

/* Memory microbenchmark for the traversal's roofline: dependent random reads,
 * the access pattern of an incoherent stackless walk (Sec. 3.1: each node
 * visited decides the next) without its arithmetic.  rows: device buffer of
 * 2^log2_rows rows of four uint32 (16 bytes, the size of a node record), any
 * contents; random contents give random chains.  Lane l (0 <= l < n_lanes)
 * starts at row (l * 0x9E3779B1) & mask, mask = 2^log2_rows - 1, and reads
 * `steps` rows: after row (x, y, z, w) it moves to row (x ^ salt) & mask with
 * salt = l * 0x85EBCA77 (uint32 arithmetic).  out (device, n_lanes uint32,
 * caller-owned) gets, per lane, the XOR of every word it read.  One wavefront
 * per workgroup.  Asynchronous on stream; nothing is allocated.
 * PM_ERR_ARG: NULL rows or out, log2_rows outside [1, 28], n_lanes outside
 * [1, 2^31), steps < 1. */
PM_API int pm_probe_chase(const uint32_t *rows, int32_t log2_rows, int64_t n_lanes, int32_t steps, uint32_t *out,
                          void *stream);

/* Memory microbenchmark for the achievable HBM bandwidth of the streaming
 * stages (the measured ceiling beside the datasheet's 8 TB/s): n_bytes
 * (a positive multiple of 64) read from src with 16-byte vector loads,
 * contiguous per wavefront, four loads in flight per thread.  mode 0 copies
 * them to dst (n_bytes written); mode 1 only reads them and XORs every
 * 32-bit word into *out (device uint32, caller-owned; the caller clears it).
 * src and dst are caller-owned device buffers, 16-byte aligned.
 * Asynchronous on stream; nothing is allocated.
 * PM_ERR_ARG: bad mode, NULL or misaligned pointers, bad n_bytes. */
PM_API int pm_probe_stream(const void *src, void *dst, uint64_t n_bytes, int32_t mode, uint32_t *out, void *stream);

#ifdef __cplusplus
}
#endif

#endif /* PM_H */
