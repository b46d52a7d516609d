/*
 * pm_oracle.c -- plain, slow CPU oracle for the photon-mapping hot path.
 *
 * TEST INFRASTRUCTURE ONLY.  Only the test suite, the smoke check and the
 * benchmark's CPU-baseline leg load this library.  The product path (the HIP
 * library) never links, calls or includes anything from here, and this file
 * includes nothing from the product path.
 *
 * What it computes, each function citing the passage it follows:
 *   - the paper's float-only random number generator (Sec. 3.2, Fig. "rand"),
 *     evaluated as the integer Lehmer step it is equivalent to, with
 *     counter-keyed stream seeding through xorshift (Sec. 3.2, last sentence);
 *   - closest ray-triangle hits by brute force over every triangle (the plain
 *     definition of what the threaded-BVH traversal of Sec. 3.1 computes), and
 *     an independent median-split stack BVH used only where brute force is
 *     infeasible, itself checked against brute force by the tests;
 *   - one stochastic progressive photon mapping iteration (Sec. 2): eye pass
 *     to the first non-specular hit, photon tracing with Russian roulette,
 *     exact range query (brute force or a plain uniform grid), progressive
 *     radius / flux update, and the final radiance estimate;
 *   - the stochastic spatial hashing estimate of the range query (Sec. 3.4):
 *     one surviving photon per hash entry by a z-buffer test on independent
 *     random depths, counted as many times as the entry received photons;
 *   - forward-mode derivatives of the rendered image with respect to the
 *     diffuse albedos and the emitted radiance.
 *
 * Floating point: float32 geometry with a fixed evaluation order (no
 * contraction: build with -ffp-contract=off), correctly rounded + - * / sqrt,
 * no transcendental calls on the sampling path; per-pixel state in double;
 * flux terms rounded one by one to unsigned 64-bit fixed point so sums do not
 * depend on their order.
 */
#include <math.h>
#include <pthread.h>
#include <stdint.h>
#include <stdlib.h>
#include <string.h>

#define ORC_EXPORT __attribute__((visibility("default")))

/* ------------------------------------------------------------------------ */
/* Thread pool: dynamic chunks over an index range.                          */
/* ------------------------------------------------------------------------ */
typedef void (*orc_range_fn)(void *ctx, int64_t i0, int64_t i1, int tid);

typedef struct {
    orc_range_fn fn;
    void *ctx;
    int64_t n, chunk;
    int64_t next; /* atomic */
    int tid;
} par_job;

typedef struct {
    par_job *job;
    int tid;
} par_arg;

static void *par_worker(void *p) {
    par_arg *a = (par_arg *)p;
    par_job *j = a->job;
    for (;;) {
        int64_t i0 = __atomic_fetch_add(&j->next, j->chunk, __ATOMIC_RELAXED);
        if (i0 >= j->n) break;
        int64_t i1 = i0 + j->chunk < j->n ? i0 + j->chunk : j->n;
        j->fn(j->ctx, i0, i1, a->tid);
    }
    return NULL;
}

static void par_for(int64_t n, int nthreads, int64_t chunk, orc_range_fn fn, void *ctx) {
    if (n <= 0) return;
    if (nthreads < 1) nthreads = 1;
    if (nthreads > 256) nthreads = 256;
    if (chunk < 1) chunk = 1;
    par_job job = {fn, ctx, n, chunk, 0, 0};
    if (nthreads == 1) {
        par_arg a = {&job, 0};
        par_worker(&a);
        return;
    }
    pthread_t th[256];
    par_arg args[256];
    for (int t = 0; t < nthreads; ++t) {
        args[t].job = &job;
        args[t].tid = t;
        pthread_create(&th[t], NULL, par_worker, &args[t]);
    }
    for (int t = 0; t < nthreads; ++t) pthread_join(th[t], NULL);
}

/* ------------------------------------------------------------------------ */
/* Random numbers (Sec. 3.2, Fig. "rand").                                   */
/*                                                                            */
/* Four multiplicative linear congruential generators s <- a*s mod m (the     */
/* generator of L'Ecuyer 1988 the paper builds on).  The paper evaluates each  */
/* step with Schrage's decomposition in float arithmetic; every intermediate  */
/* there is an exact integer below 2^24, so the step equals the integer       */
/* product reduced mod m, which is what is written here.  The returned value  */
/* is the fractional part of the weighted sum of s_j/m_j with weights          */
/* (+1, -1, +1, -1); the state is advanced before the output is formed.       */
/* ------------------------------------------------------------------------ */
static const uint32_t RNG_A[4] = {3423u, 2646u, 1707u, 1999u};
static const uint32_t RNG_M[4] = {4194287u, 4194277u, 4194191u, 4194167u};

enum { KIND_EYE = 1, KIND_PHOTON = 2, KIND_DEPTH = 3 };

static inline void rng_step(uint32_t s[4]) {
    for (int j = 0; j < 4; ++j) s[j] = (uint32_t)(((uint64_t)RNG_A[j] * s[j]) % RNG_M[j]);
}

static inline float rng_next(uint32_t s[4]) {
    rng_step(s);
    float f0 = (float)s[0] / (float)RNG_M[0];
    float f1 = (float)s[1] / (float)RNG_M[1];
    float f2 = (float)s[2] / (float)RNG_M[2];
    float f3 = (float)s[3] / (float)RNG_M[3];
    float x = ((f0 - f1) + f2) - f3;
    float u = x - floorf(x);
    if (u >= 1.0f) u = 0x1.fffffep-1f;
    return u;
}

/* splitmix64 (Steele, Lea, Flood 2014): one output per call. */
static inline uint64_t splitmix64(uint64_t *st) {
    uint64_t z = (*st += 0x9E3779B97F4A7C15ull);
    z = (z ^ (z >> 30)) * 0xBF58476D1CE4E5B9ull;
    z = (z ^ (z >> 27)) * 0x94D049BB133111EBull;
    return z ^ (z >> 31);
}

/* Marsaglia's xorshift generator "xor128" (Marsaglia 2003, J. Stat. Softw.
 * 8(14)): four 32-bit words, one output (the new last word) per call. */
static inline uint32_t xor128_next(uint32_t st[4]) {
    uint32_t t = st[0] ^ (st[0] << 11);
    st[0] = st[1];
    st[1] = st[2];
    st[2] = st[3];
    st[3] = (st[3] ^ (st[3] >> 19)) ^ (t ^ (t >> 8));
    return st[3];
}

/* Stream seeding.  The paper seeds each thread's four-word state on the CPU
 * with Marsaglia's xorshift (Sec. 3.2).  Here the xorshift seed itself is
 * derived from a counter key (seed, kind, iteration, index) through
 * splitmix64, so any stream can be regenerated on its own:
 *   h1 = splitmix64 output of state seed,
 *   h2 = splitmix64 output of state h1 ^ (kind << 32 | k),
 *   w01, w23 = the next two splitmix64 outputs from state h2 ^ index,
 *   xor128 seeded with (lo w01, hi w01, lo w23, hi w23) (all-zero -> x = 1),
 *   s_j = 1 + (output 9 + j of xor128) mod (m_j - 1), j = 0..3. */
static void rng_seed(uint64_t seed, uint32_t kind, uint32_t k, uint64_t index, uint32_t s[4]) {
    uint64_t st = seed;
    uint64_t h = splitmix64(&st);
    st = h ^ (((uint64_t)kind << 32) | (uint64_t)k);
    h = splitmix64(&st);
    st = h ^ index;
    uint64_t w01 = splitmix64(&st);
    uint64_t w23 = splitmix64(&st);
    uint32_t x[4] = {(uint32_t)w01, (uint32_t)(w01 >> 32), (uint32_t)w23, (uint32_t)(w23 >> 32)};
    if ((x[0] | x[1] | x[2] | x[3]) == 0u) x[0] = 1u;
    for (int i = 0; i < 8; ++i) (void)xor128_next(x); /* outputs 1..8 are discarded */
    for (int j = 0; j < 4; ++j) s[j] = 1u + xor128_next(x) % (RNG_M[j] - 1u);
}

/* n successive splitmix64 outputs from the given state (known-answer hook). */
ORC_EXPORT void orc_splitmix64(uint64_t state, int64_t n, uint64_t *out) {
    for (int64_t i = 0; i < n; ++i) out[i] = splitmix64(&state);
}

/* n successive xor128 outputs from the four seed words (known-answer hook). */
ORC_EXPORT void orc_xor128(const uint32_t *seed, int64_t n, uint32_t *out) {
    uint32_t st[4] = {seed[0], seed[1], seed[2], seed[3]};
    for (int64_t i = 0; i < n; ++i) out[i] = xor128_next(st);
}

ORC_EXPORT void orc_rng_seed(uint64_t seed, uint32_t kind, uint32_t k, uint64_t index, uint32_t *s) {
    rng_seed(seed, kind, k, index, s);
}

/* Advance component j of n states by one step (for exhaustive checks). */
ORC_EXPORT void orc_rng_step_component(int j, const uint32_t *in, uint32_t *out, int64_t n) {
    for (int64_t i = 0; i < n; ++i) out[i] = (uint32_t)(((uint64_t)RNG_A[j] * in[i]) % RNG_M[j]);
}

/* Draw n numbers from one stream, starting at state s (updated in place). */
ORC_EXPORT void orc_rng_draw(uint32_t *s, float *out, int64_t n) {
    for (int64_t i = 0; i < n; ++i) out[i] = rng_next(s);
}

/* Draw n numbers from each of n_streams counter-keyed streams (row-major). */
ORC_EXPORT void orc_rng_streams(uint64_t seed, uint32_t kind, uint32_t k, uint64_t index0,
                                int64_t n_streams, int64_t n_draws, float *out) {
    for (int64_t i = 0; i < n_streams; ++i) {
        uint32_t s[4];
        rng_seed(seed, kind, k, index0 + (uint64_t)i, s);
        for (int64_t d = 0; d < n_draws; ++d) out[i * n_draws + d] = rng_next(s);
    }
}

/* ------------------------------------------------------------------------ */
/* float32 vector arithmetic, fixed evaluation order.                         */
/* ------------------------------------------------------------------------ */
typedef struct { float x, y, z; } v3;

static inline v3 mk(float x, float y, float z) { v3 r = {x, y, z}; return r; }
static inline v3 sub(v3 a, v3 b) { return mk(a.x - b.x, a.y - b.y, a.z - b.z); }
static inline float dot(v3 a, v3 b) { return (a.x * b.x + a.y * b.y) + a.z * b.z; }
static inline v3 cross(v3 a, v3 b) {
    return mk(a.y * b.z - a.z * b.y, a.z * b.x - a.x * b.z, a.x * b.y - a.y * b.x);
}
static inline v3 normalize(v3 v) {
    float l = sqrtf(dot(v, v));
    return mk(v.x / l, v.y / l, v.z / l);
}
static inline v3 neg(v3 a) { return mk(-a.x, -a.y, -a.z); }
/* o + t*d, component-wise */
static inline v3 along(v3 o, float t, v3 d) { return mk(o.x + t * d.x, o.y + t * d.y, o.z + t * d.z); }

/* ------------------------------------------------------------------------ */
/* Triangles and the closest-hit definition.                                  */
/* ------------------------------------------------------------------------ */
typedef struct { v3 v0, v1, v2, e1, e2; } tri_t;   /* e1 = v1 - v0, e2 = v2 - v0 */

/* The ray/triangle test (the paper leaves it open; Sec. 3.1): the watertight
 * test of Woop, Benthin and Wald (JCGT 2013), two-sided.  Seen along the ray,
 * after a shear that maps d onto its major axis kz, the ray is the point
 * (0, 0) of the plane; it hits the triangle when that point lies inside the
 * sheared triangle, i.e. the three edge functions (doubled signed areas of
 * the point with each edge) do not differ in sign.  The hit's t is the
 * depth of the point with those edge functions as barycentric weights.  The
 * edge functions use Kahan's 2x2 determinant so that their signs are exact
 * for the rounded, sheared vertices; all steps are float32 in a fixed order. */
typedef struct { int kx, ky, kz; float sx, sy, sz; } shear_t;

static shear_t ray_shear(v3 d) {
    float ad[3] = {fabsf(d.x), fabsf(d.y), fabsf(d.z)}, dv[3] = {d.x, d.y, d.z};
    shear_t h;
    h.kz = (ad[0] >= ad[1] && ad[0] >= ad[2]) ? 0 : (ad[1] >= ad[2] ? 1 : 2);
    h.kx = (h.kz + 1) % 3;
    h.ky = (h.kz + 2) % 3;
    h.sx = dv[h.kx] / dv[h.kz];
    h.sy = dv[h.ky] / dv[h.kz];
    h.sz = 1.0f / dv[h.kz];
    return h;
}

/* a b - c d, Kahan: c d rounded, its rounding error recovered exactly by a
 * fused multiply-add; relative error at most 2^-23. */
static inline float kahan_det(float a, float b, float c, float d) {
    float w = c * d;
    float e = fmaf(-c, d, w);
    float f = fmaf(a, b, -w);
    return f + e;
}

static inline int wt_hit(v3 o, const shear_t *h, const tri_t *tr, float *t_out) {
    const v3 *vs[3] = {&tr->v0, &tr->v1, &tr->v2};
    float x[3], y[3], z[3];
    for (int i = 0; i < 3; ++i) {
        v3 a = sub(*vs[i], o);
        float c[3] = {a.x, a.y, a.z};
        x[i] = fmaf(-h->sx, c[h->kz], c[h->kx]);
        y[i] = fmaf(-h->sy, c[h->kz], c[h->ky]);
        z[i] = c[h->kz];
    }
    float U = kahan_det(x[2], y[1], y[2], x[1]);   /* edge v1 v2 */
    float V = kahan_det(x[0], y[2], y[0], x[2]);   /* edge v2 v0 */
    float W = kahan_det(x[1], y[0], y[1], x[0]);   /* edge v0 v1 */
    if ((U < 0.0f || V < 0.0f || W < 0.0f) && (U > 0.0f || V > 0.0f || W > 0.0f)) return 0;
    float det = (U + V) + W;
    if (det == 0.0f) return 0;
    float T = fmaf(W, h->sz * z[2], fmaf(V, h->sz * z[1], U * (h->sz * z[0])));
    *t_out = T / det;
    return 1;
}

/* Acceptance rule of the closest hit: strictly inside (tmin, t_best), or a
 * tie in t broken toward the lower triangle index. */
static inline int better(float t, int32_t idx, float tmin, float tbest, int32_t best) {
    if (!(t > tmin)) return 0;
    if (t < tbest) return 1;
    return (t == tbest && best >= 0 && idx < best);
}

static tri_t *make_tris(const float *verts, int64_t n) {
    tri_t *T = (tri_t *)malloc(sizeof(tri_t) * (size_t)(n > 0 ? n : 1));
    for (int64_t i = 0; i < n; ++i) {
        const float *v = verts + 9 * i;
        v3 a = mk(v[0], v[1], v[2]), b = mk(v[3], v[4], v[5]), c = mk(v[6], v[7], v[8]);
        T[i].v0 = a;
        T[i].v1 = b;
        T[i].v2 = c;
        T[i].e1 = sub(b, a);
        T[i].e2 = sub(c, a);
    }
    return T;
}

/* ---------------- independent BVH (median/midpoint split, stack) -------- */
typedef struct {
    double lo[3], hi[3];
    int32_t left, right; /* children, or -1 for a leaf */
    int32_t start, count;
} obvh_node;

typedef struct {
    obvh_node *nodes;
    int32_t n_nodes, cap;
    int32_t *idx;
    double pad;
} obvh;

typedef struct {
    const float *verts;
    double *cen; /* [n][3] */
    int32_t *idx;
} obuild_ctx;

static int32_t obvh_new(obvh *b) {
    if (b->n_nodes == b->cap) {
        b->cap = b->cap ? 2 * b->cap : 1024;
        b->nodes = (obvh_node *)realloc(b->nodes, sizeof(obvh_node) * (size_t)b->cap);
    }
    return b->n_nodes++;
}

static int cmp_axis;
static const double *cmp_cen;
static int cmp_idx(const void *a, const void *b) {
    double x = cmp_cen[3 * *(const int32_t *)a + cmp_axis];
    double y = cmp_cen[3 * *(const int32_t *)b + cmp_axis];
    if (x < y) return -1;
    if (x > y) return 1;
    return (*(const int32_t *)a) - (*(const int32_t *)b);
}

static int32_t obvh_build_rec(obvh *b, obuild_ctx *c, int32_t start, int32_t count) {
    int32_t ni = obvh_new(b);
    double lo[3] = {INFINITY, INFINITY, INFINITY}, hi[3] = {-INFINITY, -INFINITY, -INFINITY};
    double clo[3] = {INFINITY, INFINITY, INFINITY}, chi[3] = {-INFINITY, -INFINITY, -INFINITY};
    for (int32_t i = start; i < start + count; ++i) {
        const float *v = c->verts + 9 * (int64_t)c->idx[i];
        for (int k = 0; k < 3; ++k)
            for (int a = 0; a < 3; ++a) {
                double x = v[3 * k + a];
                if (x < lo[a]) lo[a] = x;
                if (x > hi[a]) hi[a] = x;
            }
        for (int a = 0; a < 3; ++a) {
            double x = c->cen[3 * (int64_t)c->idx[i] + a];
            if (x < clo[a]) clo[a] = x;
            if (x > chi[a]) chi[a] = x;
        }
    }
    obvh_node *nd = &b->nodes[ni];
    for (int a = 0; a < 3; ++a) {
        nd->lo[a] = lo[a] - b->pad;
        nd->hi[a] = hi[a] + b->pad;
    }
    if (count <= 4) {
        nd->left = nd->right = -1;
        nd->start = start;
        nd->count = count;
        return ni;
    }
    int axis = 0;
    for (int a = 1; a < 3; ++a)
        if (chi[a] - clo[a] > chi[axis] - clo[axis]) axis = a;
    /* midpoint split of the centroid bounds, falling back to the median */
    double mid = 0.5 * (clo[axis] + chi[axis]);
    int32_t i = start, j = start + count - 1;
    while (i <= j) {
        if (c->cen[3 * (int64_t)c->idx[i] + axis] < mid) {
            ++i;
        } else {
            int32_t t = c->idx[i];
            c->idx[i] = c->idx[j];
            c->idx[j] = t;
            --j;
        }
    }
    int32_t nl = i - start;
    if (nl == 0 || nl == count) {
        cmp_axis = axis;
        cmp_cen = c->cen;
        qsort(c->idx + start, (size_t)count, sizeof(int32_t), cmp_idx);
        nl = count / 2;
    }
    int32_t l = obvh_build_rec(b, c, start, nl);
    int32_t r = obvh_build_rec(b, c, start + nl, count - nl);
    nd = &b->nodes[ni];
    nd->left = l;
    nd->right = r;
    nd->start = nd->count = 0;
    return ni;
}

static obvh *obvh_build(const float *verts, int64_t n, double diag) {
    obvh *b = (obvh *)calloc(1, sizeof(obvh));
    b->pad = 1e-4 * diag + 1e-30;
    obuild_ctx c;
    c.verts = verts;
    c.cen = (double *)malloc(sizeof(double) * 3 * (size_t)n);
    c.idx = (int32_t *)malloc(sizeof(int32_t) * (size_t)n);
    for (int64_t i = 0; i < n; ++i) {
        c.idx[i] = (int32_t)i;
        for (int a = 0; a < 3; ++a)
            c.cen[3 * i + a] = ((double)verts[9 * i + a] + verts[9 * i + 3 + a] + verts[9 * i + 6 + a]) / 3.0;
    }
    obvh_build_rec(b, &c, 0, (int32_t)n);
    free(c.cen);
    b->idx = c.idx;
    return b;
}

static void obvh_free(obvh *b) {
    if (!b) return;
    free(b->nodes);
    free(b->idx);
    free(b);
}

/* Slab test in double against the padded box, inclusive at both ends, with
 * the far end widened by 2^-16 of itself: an accepted triangle hit's point
 * o + t d may lie outside the triangle's box by a few 2^-24 of t |d_a| per
 * axis (its rounding), and the padding covers only absolute amounts. */
static inline int obox_hit(const obvh_node *nd, const double o[3], const double d[3], double tmin, double tmax) {
    double t0 = tmin, t1 = tmax;
    for (int a = 0; a < 3; ++a) {
        if (d[a] == 0.0) {
            if (o[a] < nd->lo[a] || o[a] > nd->hi[a]) return 0;
            continue;
        }
        double ta = (nd->lo[a] - o[a]) / d[a];
        double tb = (nd->hi[a] - o[a]) / d[a];
        if (ta > tb) { double t = ta; ta = tb; tb = t; }
        if (ta > t0) t0 = ta;
        if (tb < t1) t1 = tb;
    }
    return t0 <= t1 + fabs(t1) * 0x1p-16;
}

/* Closest hit in (tmin, tmax), ties to the lower index; excluded index skipped. */
static int32_t closest_bf(const tri_t *T, int64_t n, v3 o, v3 d, float tmin, float tmax, int32_t exclude, float *t_out) {
    int32_t best = -1;
    float tb = tmax;
    const shear_t h = ray_shear(d);
    for (int64_t i = 0; i < n; ++i) {
        if ((int32_t)i == exclude) continue;
        float t;
        if (wt_hit(o, &h, &T[i], &t) && better(t, (int32_t)i, tmin, tb, best)) {
            tb = t;
            best = (int32_t)i;
        }
    }
    *t_out = best >= 0 ? tb : INFINITY;
    return best;
}

static int32_t closest_bvh(const obvh *b, const tri_t *T, v3 o, v3 d, float tmin, float tmax, int32_t exclude, float *t_out) {
    int32_t best = -1;
    float tb = tmax;
    const shear_t h = ray_shear(d);
    double od[3] = {o.x, o.y, o.z}, dd[3] = {d.x, d.y, d.z};
    int32_t stack[256];
    int sp = 0;
    stack[sp++] = 0;
    while (sp) {
        const obvh_node *nd = &b->nodes[stack[--sp]];
        if (!obox_hit(nd, od, dd, (double)tmin, (double)tb)) continue;
        if (nd->left < 0) {
            for (int32_t k = nd->start; k < nd->start + nd->count; ++k) {
                int32_t i = b->idx[k];
                if (i == exclude) continue;
                float t;
                if (wt_hit(o, &h, &T[i], &t) && better(t, i, tmin, tb, best)) {
                    tb = t;
                    best = i;
                }
            }
        } else {
            stack[sp++] = nd->left;
            stack[sp++] = nd->right;
        }
    }
    *t_out = best >= 0 ? tb : INFINITY;
    return best;
}

/* ------------------------------------------------------------------------ */
/* Scene.                                                                     */
/* ------------------------------------------------------------------------ */
enum { MAT_DIFFUSE = 0, MAT_MIRROR = 1, MAT_GLASS = 2 };

typedef struct {
    const float *verts;
    const uint32_t *tri_mat;
    int64_t n_tri;
    const int32_t *mat_type;
    const float *mat_rho;
    const float *mat_q;
    const float *mat_Le;
    const float *mat_ior;
    int32_t n_mat;
    float cam_pos[3], cam_look[3], cam_up[3];
    float tan_half_fov;
    int32_t width, height;
} orc_scene_desc;

typedef struct {
    orc_scene_desc d;
    tri_t *T;
    obvh *bvh; /* NULL: brute force */
    float eps; /* secondary-ray offset: 1e-5 * scene diagonal */
    /* emitters */
    int64_t n_emit;
    int32_t *emit_tri;
    double *emit_cdf;
    double power; /* sum of area * Le */
    /* camera basis */
    v3 cf, cr, cu;
} orc_scene;

ORC_EXPORT orc_scene *orc_scene_create(const orc_scene_desc *d, int use_bvh) {
    orc_scene *s = (orc_scene *)calloc(1, sizeof(orc_scene));
    s->d = *d;
    s->T = make_tris(d->verts, d->n_tri);
    float lo[3] = {INFINITY, INFINITY, INFINITY}, hi[3] = {-INFINITY, -INFINITY, -INFINITY};
    for (int64_t i = 0; i < 9 * d->n_tri; ++i) {
        int a = (int)(i % 3);
        if (d->verts[i] < lo[a]) lo[a] = d->verts[i];
        if (d->verts[i] > hi[a]) hi[a] = d->verts[i];
    }
    v3 ext = mk(hi[0] - lo[0], hi[1] - lo[1], hi[2] - lo[2]);
    float diag = sqrtf(dot(ext, ext));
    s->eps = 1e-5f * diag;
    if (use_bvh) s->bvh = obvh_build(d->verts, d->n_tri, (double)diag);
    /* emitter table in triangle order: power_i = area_i * Le_i */
    s->emit_tri = (int32_t *)malloc(sizeof(int32_t) * (size_t)(d->n_tri + 1));
    s->emit_cdf = (double *)malloc(sizeof(double) * (size_t)(d->n_tri + 1));
    double acc = 0.0;
    for (int64_t i = 0; i < d->n_tri; ++i) {
        float Le = d->mat_Le[d->tri_mat[i]];
        if (!(Le > 0.0f)) continue;
        v3 c = cross(s->T[i].e1, s->T[i].e2);
        float area = 0.5f * sqrtf(dot(c, c));
        acc += (double)area * (double)Le;
        s->emit_tri[s->n_emit] = (int32_t)i;
        s->emit_cdf[s->n_emit] = acc;
        s->n_emit++;
    }
    s->power = acc;
    /* pinhole camera basis */
    v3 pos = mk(d->cam_pos[0], d->cam_pos[1], d->cam_pos[2]);
    v3 look = mk(d->cam_look[0], d->cam_look[1], d->cam_look[2]);
    v3 up = mk(d->cam_up[0], d->cam_up[1], d->cam_up[2]);
    s->cf = normalize(sub(look, pos));
    s->cr = normalize(cross(s->cf, up));
    s->cu = cross(s->cr, s->cf);
    return s;
}

ORC_EXPORT void orc_scene_destroy(orc_scene *s) {
    if (!s) return;
    free(s->T);
    obvh_free(s->bvh);
    free(s->emit_tri);
    free(s->emit_cdf);
    free(s);
}

ORC_EXPORT float orc_scene_eps(const orc_scene *s) { return s->eps; }
ORC_EXPORT double orc_scene_power(const orc_scene *s) { return s->power; }

static inline int32_t scene_closest(const orc_scene *s, v3 o, v3 d, float tmin, float tmax, int32_t exclude, float *t) {
    if (s->bvh) return closest_bvh(s->bvh, s->T, o, d, tmin, tmax, exclude, t);
    return closest_bf(s->T, s->d.n_tri, o, d, tmin, tmax, exclude, t);
}

/* ---------------- batched closest hit (trace_rays definition) ------------ */
typedef struct {
    const orc_scene *s;
    const float *rays;
    int32_t *hit;
    float *t;
    int force_bf;
} trace_ctx;

static void trace_range(void *vc, int64_t i0, int64_t i1, int tid) {
    (void)tid;
    trace_ctx *c = (trace_ctx *)vc;
    for (int64_t i = i0; i < i1; ++i) {
        const float *r = c->rays + 8 * i;
        v3 o = mk(r[0], r[1], r[2]), d = mk(r[4], r[5], r[6]);
        float t;
        int32_t h = c->force_bf ? closest_bf(c->s->T, c->s->d.n_tri, o, d, r[3], r[7], -1, &t)
                                : scene_closest(c->s, o, d, r[3], r[7], -1, &t);
        c->hit[i] = h;
        c->t[i] = t;
    }
}

/* rays: n x 8 (o.xyz, tmin, d.xyz, tmax).  Miss: hit=-1, t=+inf. */
ORC_EXPORT void orc_trace(const orc_scene *s, const float *rays, int64_t n, int32_t *hit, float *t,
                          int force_bf, int nthreads) {
    trace_ctx c = {s, rays, hit, t, force_bf};
    par_for(n, nthreads, 16, trace_range, &c);
}

/* Per-ray count of box and triangle tests of the oracle BVH is not exposed;
 * the oracle is about results, not about traversal cost. */

/* ------------------------------------------------------------------------ */
/* Sampling helpers (shared rules: + - * / sqrt only).                        */
/* ------------------------------------------------------------------------ */
/* Orthonormal basis around unit n (Duff et al. 2017, "Building an
 * Orthonormal Basis, Revisited"). */
static inline void onb(v3 n, v3 *b1, v3 *b2) {
    float sign = copysignf(1.0f, n.z);
    float a = -1.0f / (sign + n.z);
    float b = n.x * n.y * a;
    *b1 = mk(1.0f + sign * n.x * n.x * a, sign * b, -sign * n.x);
    *b2 = mk(b, sign + n.y * n.y * a, -n.y);
}

/* Cosine-weighted direction about unit n: uniform point in the unit disk by
 * rejection from the square, lifted to the hemisphere (Malley's method). */
static inline v3 cosine_dir(v3 n, uint32_t s[4]) {
    float a = 0.0f, b = 0.0f, r2 = 0.0f;
    int ok = 0;
    for (int tries = 0; tries < 64; ++tries) {
        a = 2.0f * rng_next(s) - 1.0f;
        b = 2.0f * rng_next(s) - 1.0f;
        r2 = a * a + b * b;
        if (r2 < 1.0f) { ok = 1; break; }
    }
    if (!ok) { a = 0.0f; b = 0.0f; r2 = 0.0f; }
    float z = sqrtf(1.0f - r2);
    v3 t1, t2;
    onb(n, &t1, &t2);
    v3 w = mk((a * t1.x + b * t2.x) + z * n.x, (a * t1.y + b * t2.y) + z * n.y, (a * t1.z + b * t2.z) + z * n.z);
    return normalize(w);
}

static inline v3 reflect(v3 d, v3 n) {
    float c = 2.0f * dot(d, n);
    return mk(d.x - c * n.x, d.y - c * n.y, d.z - c * n.z);
}

/* Smooth dielectric: unpolarised Fresnel reflectance chooses reflection or
 * refraction with one draw (drawn even under total internal reflection). */
/* Unpolarised Fresnel reflectance for cosine ci (> 0) of the incident angle
 * and relative index eta = n_incident / n_transmitted; ct receives the cosine
 * of the transmitted angle (0 under total internal reflection, where F = 1). */
static inline float fresnel(float ci, float eta, float *ct_out) {
    float sin2t = (eta * eta) * (1.0f - ci * ci);
    float k = 1.0f - sin2t;
    float F = 1.0f, ct = 0.0f;
    if (k >= 0.0f) {
        ct = sqrtf(k);
        float rs = (eta * ci - ct) / (eta * ci + ct);
        float rp = (ci - eta * ct) / (ci + eta * ct);
        F = 0.5f * (rs * rs + rp * rp);
    }
    *ct_out = ct;
    return F;
}

static inline v3 glass_dir(v3 d, v3 n, float ior, uint32_t s[4]) {
    float cosi = -dot(d, n);
    float eta, ci;
    v3 nn;
    if (cosi > 0.0f) { eta = 1.0f / ior; nn = n; ci = cosi; }
    else { eta = ior; nn = neg(n); ci = -cosi; }
    float ct;
    float F = fresnel(ci, eta, &ct);
    float u = rng_next(s);
    if (u < F) return reflect(d, n);
    float c = eta * ci - ct;
    return normalize(mk(eta * d.x + c * nn.x, eta * d.y + c * nn.y, eta * d.z + c * nn.z));
}

static inline v3 tri_normal(const tri_t *tr) { return normalize(cross(tr->e1, tr->e2)); }

/* Unit-test hooks for the sampling helpers. */
ORC_EXPORT float orc_fresnel(float ci, float eta) {
    float ct;
    return fresnel(ci, eta, &ct);
}

ORC_EXPORT void orc_onb(const float *n, float *b1, float *b2) {
    v3 a, b;
    onb(mk(n[0], n[1], n[2]), &a, &b);
    b1[0] = a.x; b1[1] = a.y; b1[2] = a.z;
    b2[0] = b.x; b2[1] = b.y; b2[2] = b.z;
}

/* count cosine-distributed directions about n from stream (seed, kind, k, i). */
ORC_EXPORT void orc_cosine_dirs(const float *n, uint64_t seed, int64_t count, float *out) {
    v3 nn = mk(n[0], n[1], n[2]);
    for (int64_t i = 0; i < count; ++i) {
        uint32_t s[4];
        rng_seed(seed, 99u, 0u, (uint64_t)i, s);
        v3 w = cosine_dir(nn, s);
        out[3 * i] = w.x; out[3 * i + 1] = w.y; out[3 * i + 2] = w.z;
    }
}

ORC_EXPORT void orc_glass_dirs(const float *d, const float *n, float ior, uint64_t seed, int64_t count, float *out) {
    v3 dd = mk(d[0], d[1], d[2]), nn = mk(n[0], n[1], n[2]);
    for (int64_t i = 0; i < count; ++i) {
        uint32_t s[4];
        rng_seed(seed, 98u, 0u, (uint64_t)i, s);
        v3 w = glass_dir(dd, nn, ior, s);
        out[3 * i] = w.x; out[3 * i + 1] = w.y; out[3 * i + 2] = w.z;
    }
}

#define INV_PI_F 0.318309886183790671538f
#define PI_D 3.14159265358979323846

/* ------------------------------------------------------------------------ */
/* SPPM iteration pieces (Sec. 2).                                            */
/* ------------------------------------------------------------------------ */
typedef struct {
    uint64_t seed;
    int32_t max_eye_depth;      /* 16 */
    int32_t max_photon_bounces; /* 32 */
    int32_t nthreads;
} orc_run_opts;

/* Hit point of an eye path: first non-specular (diffuse, rho > 0) hit. */
typedef struct {
    uint8_t *valid;
    float *x;  /* [P][3] */
    float *n;  /* [P][3], oriented toward the incoming eye ray */
    float *wk; /* W * rho / pi */
    float *W;  /* path throughput */
    int32_t *mat;
    int32_t *tri;
    double *d_add; /* emission seen directly along the eye path */
} orc_hitpoints;

static void eye_path(const orc_scene *s, const orc_run_opts *op, uint32_t k, int64_t p, orc_hitpoints *hp) {
    const orc_scene_desc *d = &s->d;
    int32_t W = d->width, H = d->height;
    int32_t px = (int32_t)(p % W), py = (int32_t)(p / W);
    uint32_t st[4];
    rng_seed(op->seed, KIND_EYE, k, (uint64_t)p, st);
    float j0 = rng_next(st), j1 = rng_next(st);
    float aspect = (float)W / (float)H;
    float fx = ((float)px + j0) / (float)W;
    float fy = ((float)py + j1) / (float)H;
    float sx = (2.0f * fx - 1.0f) * (d->tan_half_fov * aspect);
    float sy = (1.0f - 2.0f * fy) * d->tan_half_fov;
    v3 dir = normalize(mk((s->cf.x + sx * s->cr.x) + sy * s->cu.x, (s->cf.y + sx * s->cr.y) + sy * s->cu.y,
                          (s->cf.z + sx * s->cr.z) + sy * s->cu.z));
    v3 org = mk(d->cam_pos[0], d->cam_pos[1], d->cam_pos[2]);
    float tmin = 0.0f, thr = 1.0f;
    int32_t excl = -1;
    double dadd = 0.0;
    hp->valid[p] = 0;
    for (int depth = 0; depth < op->max_eye_depth; ++depth) {
        float t;
        int32_t h = scene_closest(s, org, dir, tmin, INFINITY, excl, &t);
        if (h < 0) break;
        v3 x = along(org, t, dir);
        v3 n = tri_normal(&s->T[h]);
        int32_t m = (int32_t)d->tri_mat[h];
        float dn = dot(dir, n);
        int front = dn < 0.0f;
        float Le = d->mat_Le[m];
        if (Le > 0.0f && front) dadd += (double)(thr * Le);
        int type = d->mat_type[m];
        if (type == MAT_DIFFUSE) {
            float rho = d->mat_rho[m];
            if (rho > 0.0f) {
                v3 nh = front ? n : neg(n);
                hp->valid[p] = 1;
                hp->x[3 * p] = x.x; hp->x[3 * p + 1] = x.y; hp->x[3 * p + 2] = x.z;
                hp->n[3 * p] = nh.x; hp->n[3 * p + 1] = nh.y; hp->n[3 * p + 2] = nh.z;
                hp->W[p] = thr;
                hp->wk[p] = (thr * rho) * INV_PI_F;
                hp->mat[p] = m;
                hp->tri[p] = h;
            }
            break;
        } else if (type == MAT_MIRROR) {
            dir = reflect(dir, n);
        } else {
            dir = glass_dir(dir, n, d->mat_ior[m], st);
        }
        org = x;
        tmin = s->eps;
        excl = h;
    }
    hp->d_add[p] = dadd;
}

typedef struct {
    const orc_scene *s;
    const orc_run_opts *op;
    uint32_t k;
    orc_hitpoints *hp;
} eye_ctx;

static void eye_range(void *vc, int64_t i0, int64_t i1, int tid) {
    (void)tid;
    eye_ctx *c = (eye_ctx *)vc;
    for (int64_t p = i0; p < i1; ++p) eye_path(c->s, c->op, c->k, p, c->hp);
}

ORC_EXPORT void orc_eye_pass(const orc_scene *s, const orc_run_opts *op, uint32_t k, orc_hitpoints *hp) {
    eye_ctx c = {s, op, k, hp};
    par_for((int64_t)s->d.width * s->d.height, op->nthreads, 64, eye_range, &c);
}

/* Sampled eye paths: only the listed pixels. */
ORC_EXPORT void orc_eye_pixels(const orc_scene *s, const orc_run_opts *op, uint32_t k, const int64_t *pix, int64_t n,
                               orc_hitpoints *hp) {
    for (int64_t i = 0; i < n; ++i) eye_path(s, op, k, pix[i], hp);
}

/* Photon records in (path, bounce) order. */
typedef struct {
    float *x;       /* [cap][3] */
    float *w;       /* [cap][3] incoming direction */
    float *phi;     /* [cap] */
    uint32_t *path; /* [cap] */
    uint32_t *bounce;
    int32_t *mats;  /* [cap][32] diffuse materials of earlier bounces: filled only when non-NULL */
    int64_t cap;
} orc_photons;

/* Start of a photon path (Sec. 2: photons are traced from the light
 * sources): an emitting triangle chosen with probability proportional to its
 * power area * Le (one draw against the cumulative table), a uniform point on
 * it (two draws, folded into the triangle when u1 + u2 > 1), and a cosine-
 * distributed direction about its normal.  Returns the triangle's index. */
static int32_t photon_emit(const orc_scene *s, uint32_t st[4], v3 *org, v3 *dir) {
    float u0 = rng_next(st);
    double target = (double)u0 * s->power;
    int64_t e = 0;
    while (e < s->n_emit - 1 && !(target < s->emit_cdf[e])) ++e;
    int32_t et = s->emit_tri[e];
    const tri_t *tr = &s->T[et];
    float u1 = rng_next(st), u2 = rng_next(st);
    if (u1 + u2 > 1.0f) { u1 = 1.0f - u1; u2 = 1.0f - u2; }
    *org = mk((tr->v0.x + u1 * tr->e1.x) + u2 * tr->e2.x, (tr->v0.y + u1 * tr->e1.y) + u2 * tr->e2.y,
              (tr->v0.z + u1 * tr->e1.z) + u2 * tr->e2.z);
    *dir = cosine_dir(tri_normal(tr), st);
    return et;
}

/* Emission of photon paths [0, n) of iteration k: origin, direction and the
 * emitting triangle of each (-1 and zeros when the scene has no emitter). */
ORC_EXPORT void orc_photon_emit(const orc_scene *s, uint64_t seed, uint32_t k, int64_t n, float *org, float *dir,
                                int32_t *tri) {
    for (int64_t i = 0; i < n; ++i) {
        v3 o = mk(0.0f, 0.0f, 0.0f), w = mk(0.0f, 0.0f, 0.0f);
        int32_t et = -1;
        if (s->n_emit > 0) {
            uint32_t st[4];
            rng_seed(seed, KIND_PHOTON, k, (uint64_t)i, st);
            et = photon_emit(s, st, &o, &w);
        }
        org[3 * i] = o.x; org[3 * i + 1] = o.y; org[3 * i + 2] = o.z;
        dir[3 * i] = w.x; dir[3 * i + 1] = w.y; dir[3 * i + 2] = w.z;
        tri[i] = et;
    }
}

/* Trace photon path n of iteration k.  Appends up to max_bounces photons to
 * buf (a local buffer), returns the number appended. */
static int photon_path(const orc_scene *s, const orc_run_opts *op, uint32_t k, uint64_t n, float phi0,
                       v3 *bx, v3 *bw, float *bphi, uint32_t *bb, int32_t *bmats) {
    const orc_scene_desc *d = &s->d;
    uint32_t st[4];
    rng_seed(op->seed, KIND_PHOTON, k, n, st);
    if (s->n_emit == 0) return 0;
    v3 org, dir;
    int32_t et = photon_emit(s, st, &org, &dir);
    float phi = phi0;
    int32_t excl = et;
    int stored = 0;
    int32_t hist[64];
    int nhist = 0;
    for (int b = 0; b < op->max_photon_bounces; ++b) {
        float t;
        int32_t h = scene_closest(s, org, dir, s->eps, INFINITY, excl, &t);
        if (h < 0) break;
        v3 x = along(org, t, dir);
        v3 nrm = tri_normal(&s->T[h]);
        int32_t m = (int32_t)d->tri_mat[h];
        int type = d->mat_type[m];
        if (type == MAT_DIFFUSE) {
            float rho = d->mat_rho[m];
            if (!(rho > 0.0f)) break; /* black surface (the emitter) absorbs */
            bx[stored] = x;
            bw[stored] = dir;
            bphi[stored] = phi;
            bb[stored] = (uint32_t)b;
            if (bmats) {
                for (int i = 0; i < 32; ++i) bmats[stored * 32 + i] = i < nhist ? hist[i] : -1;
            }
            stored++;
            float u = rng_next(st);
            if (!(u < d->mat_q[m])) break;
            phi = (phi * rho) / d->mat_q[m];
            if (nhist < 64) hist[nhist++] = m;
            v3 ns = dot(dir, nrm) < 0.0f ? nrm : neg(nrm);
            dir = cosine_dir(ns, st);
        } else if (type == MAT_MIRROR) {
            dir = reflect(dir, nrm);
        } else {
            dir = glass_dir(dir, nrm, d->mat_ior[m], st);
        }
        org = x;
        excl = h;
    }
    return stored;
}

typedef struct {
    const orc_scene *s;
    const orc_run_opts *op;
    uint32_t k;
    float phi0;
    const uint64_t *paths; /* NULL: path id = index */
    /* per-path outputs, fixed stride 64 */
    float *x, *w, *phi;
    uint32_t *bounce;
    int32_t *mats;
    int32_t *cnt;
} photon_ctx;

static void photon_range(void *vc, int64_t i0, int64_t i1, int tid) {
    (void)tid;
    photon_ctx *c = (photon_ctx *)vc;
    v3 bx[64], bw[64];
    float bphi[64];
    uint32_t bb[64];
    for (int64_t i = i0; i < i1; ++i) {
        uint64_t n = c->paths ? c->paths[i] : (uint64_t)i;
        int cnt = photon_path(c->s, c->op, c->k, n, c->phi0, bx, bw, bphi, bb,
                              c->mats ? c->mats + (size_t)i * 64 * 32 : NULL);
        c->cnt[i] = cnt;
        for (int j = 0; j < cnt; ++j) {
            size_t o = (size_t)i * 64 + (size_t)j;
            c->x[3 * o] = bx[j].x; c->x[3 * o + 1] = bx[j].y; c->x[3 * o + 2] = bx[j].z;
            c->w[3 * o] = bw[j].x; c->w[3 * o + 1] = bw[j].y; c->w[3 * o + 2] = bw[j].z;
            c->phi[o] = bphi[j];
            c->bounce[o] = bb[j];
        }
    }
}

/* Initial photon flux: the emitters' total power pi * sum(area * Le) split over
 * the n_photons paths of one iteration. */
ORC_EXPORT float orc_photon_flux(const orc_scene *s, int64_t n_photons) {
    return (float)((PI_D * s->power) / (double)n_photons);
}

/* Trace photon paths (all of [0, n_paths) or the listed ids).  Outputs are
 * dense in (path, bounce) order; returns the number of photons, or -1 if cap
 * is exceeded.  mats (optional, cap x 32) receives the diffuse materials of the
 * bounces before each stored photon (-1 padded). */
ORC_EXPORT int64_t orc_photon_pass(const orc_scene *s, const orc_run_opts *op, uint32_t k, int64_t n_photons_total,
                                   const uint64_t *paths, int64_t n_paths, orc_photons *out) {
    photon_ctx c;
    c.s = s;
    c.op = op;
    c.k = k;
    c.phi0 = orc_photon_flux(s, n_photons_total);
    c.paths = paths;
    int64_t chunk = 4096;
    int64_t total = 0;
    c.x = (float *)malloc(sizeof(float) * 3 * 64 * (size_t)chunk);
    c.w = (float *)malloc(sizeof(float) * 3 * 64 * (size_t)chunk);
    c.phi = (float *)malloc(sizeof(float) * 64 * (size_t)chunk);
    c.bounce = (uint32_t *)malloc(sizeof(uint32_t) * 64 * (size_t)chunk);
    c.cnt = (int32_t *)malloc(sizeof(int32_t) * (size_t)chunk);
    c.mats = out->mats ? (int32_t *)malloc(sizeof(int32_t) * 64 * 32 * (size_t)chunk) : NULL;
    int overflow = 0;
    for (int64_t base = 0; base < n_paths && !overflow; base += chunk) {
        int64_t m = n_paths - base < chunk ? n_paths - base : chunk;
        photon_ctx cc = c;
        cc.paths = paths ? paths + base : NULL;
        /* path ids when paths == NULL: base + i */
        if (!paths) {
            /* shift ids by running with a temporary id list */
            uint64_t *ids = (uint64_t *)malloc(sizeof(uint64_t) * (size_t)m);
            for (int64_t i = 0; i < m; ++i) ids[i] = (uint64_t)(base + i);
            cc.paths = ids;
            par_for(m, op->nthreads, 16, photon_range, &cc);
            free(ids);
        } else {
            par_for(m, op->nthreads, 16, photon_range, &cc);
        }
        for (int64_t i = 0; i < m && !overflow; ++i) {
            for (int j = 0; j < c.cnt[i]; ++j) {
                if (total >= out->cap) { overflow = 1; break; }
                size_t o = (size_t)i * 64 + (size_t)j;
                out->x[3 * total] = c.x[3 * o]; out->x[3 * total + 1] = c.x[3 * o + 1]; out->x[3 * total + 2] = c.x[3 * o + 2];
                out->w[3 * total] = c.w[3 * o]; out->w[3 * total + 1] = c.w[3 * o + 1]; out->w[3 * total + 2] = c.w[3 * o + 2];
                out->phi[total] = c.phi[o];
                out->path[total] = (uint32_t)(paths ? paths[base + i] : (uint64_t)(base + i));
                out->bounce[total] = c.bounce[o];
                if (out->mats) memcpy(out->mats + (size_t)total * 32, c.mats + o * 32, sizeof(int32_t) * 32);
                total++;
            }
        }
    }
    free(c.x); free(c.w); free(c.phi); free(c.bounce); free(c.cnt); free(c.mats);
    return overflow ? -1 : total;
}

/* Fixed-point image of one flux term: round(c * 2^shift) with c = wk * phi
 * formed exactly in double (a product of two floats). */
static inline uint64_t fx_term(float wk, float phi, int shift) {
    double c = ((double)wk * (double)phi) * ldexp(1.0, shift);
    return (uint64_t)rint(c);
}

/* Exact range query: photon j counts for hit point p if its squared distance
 * (float32, fixed order) is below R2[p] and it arrived from the side the eye
 * ray came from. */
static inline int accept(const float *xp, const float *np, const float *xj, const float *wj, double R2) {
    float dx = xj[0] - xp[0], dy = xj[1] - xp[1], dz = xj[2] - xp[2];
    float d2 = (dx * dx + dy * dy) + dz * dz;
    if (!((double)d2 < R2)) return 0;
    float c = (wj[0] * np[0] + wj[1] * np[1]) + wj[2] * np[2];
    return c < 0.0f;
}

typedef struct {
    const orc_hitpoints *hp;
    int64_t n_hp;
    const orc_photons *ph;
    int64_t n_ph;
    const double *R2;
    int shift;
    uint32_t *M;
    uint64_t *Phi;
    double *phid;
    /* grid */
    double lo[3], h;
    int64_t dim[3];
    int64_t *cell_start; /* dim product + 1 */
    int64_t *order;
    /* optional forward-mode derivatives (see orc_sppm_grad) */
    const double *gw;     /* [P] dloss/dL_p / (pi R2_p K) */
    const float *rho;     /* material albedos */
    const int32_t *pmat;  /* [n_par] material of each albedo parameter */
    int n_par;
    double *acc;          /* [nthreads][n_par] */
} gather_ctx;

/* Derivative of one contribution c = W * (rho_h / pi) * phi_j with respect to
 * the albedo of material m: phi_j carries a factor rho_m / q_m for every
 * earlier diffuse bounce on m, and rho_h is the hit point's own albedo, so
 * dc/drho_m = c * (n_m(j) + [mat_h == m]) / rho_m. */
static inline void grad_term(gather_ctx *c, int64_t p, int64_t j, int tid) {
    if (!c->gw) return;
    double cc = (double)c->hp->wk[p] * (double)c->ph->phi[j];
    const int32_t *hist = c->ph->mats + (size_t)j * 32;
    for (int i = 0; i < c->n_par; ++i) {
        int32_t m = c->pmat[i];
        int cnt = (c->hp->mat[p] == m);
        for (int b = 0; b < 32 && hist[b] >= 0; ++b) cnt += (hist[b] == m);
        if (cnt) c->acc[(size_t)tid * c->n_par + i] += c->gw[p] * cc * (double)cnt / (double)c->rho[m];
    }
}

static void gather_bf_range(void *vc, int64_t i0, int64_t i1, int tid) {
    gather_ctx *c = (gather_ctx *)vc;
    for (int64_t p = i0; p < i1; ++p) {
        uint32_t M = 0;
        uint64_t F = 0;
        double fd = 0.0;
        if (c->hp->valid[p]) {
            for (int64_t j = 0; j < c->n_ph; ++j) {
                if (accept(c->hp->x + 3 * p, c->hp->n + 3 * p, c->ph->x + 3 * j, c->ph->w + 3 * j, c->R2[p])) {
                    M++;
                    F += fx_term(c->hp->wk[p], c->ph->phi[j], c->shift);
                    fd += (double)c->hp->wk[p] * (double)c->ph->phi[j];
                    grad_term(c, p, j, tid);
                }
            }
        }
        c->M[p] = M;
        c->Phi[p] = F;
        if (c->phid) c->phid[p] = fd;
    }
}

static inline int64_t cell_of(const gather_ctx *c, const float *x, int64_t ci[3]) {
    for (int a = 0; a < 3; ++a) {
        double f = floor(((double)x[a] - c->lo[a]) / c->h);
        int64_t i = (int64_t)f;
        if (i < 0) i = 0;
        if (i >= c->dim[a]) i = c->dim[a] - 1;
        ci[a] = i;
    }
    return (ci[2] * c->dim[1] + ci[1]) * c->dim[0] + ci[0];
}

static void gather_grid_range(void *vc, int64_t i0, int64_t i1, int tid) {
    gather_ctx *c = (gather_ctx *)vc;
    for (int64_t p = i0; p < i1; ++p) {
        uint32_t M = 0;
        uint64_t F = 0;
        double fd = 0.0;
        if (c->hp->valid[p]) {
            int64_t ci[3];
            cell_of(c, c->hp->x + 3 * p, ci);
            for (int64_t dz = -1; dz <= 1; ++dz)
                for (int64_t dy = -1; dy <= 1; ++dy)
                    for (int64_t dx = -1; dx <= 1; ++dx) {
                        int64_t cx = ci[0] + dx, cy = ci[1] + dy, cz = ci[2] + dz;
                        if (cx < 0 || cy < 0 || cz < 0 || cx >= c->dim[0] || cy >= c->dim[1] || cz >= c->dim[2]) continue;
                        int64_t cell = (cz * c->dim[1] + cy) * c->dim[0] + cx;
                        for (int64_t q = c->cell_start[cell]; q < c->cell_start[cell + 1]; ++q) {
                            int64_t j = c->order[q];
                            if (accept(c->hp->x + 3 * p, c->hp->n + 3 * p, c->ph->x + 3 * j, c->ph->w + 3 * j, c->R2[p])) {
                                M++;
                                F += fx_term(c->hp->wk[p], c->ph->phi[j], c->shift);
                                fd += (double)c->hp->wk[p] * (double)c->ph->phi[j];
                                grad_term(c, p, j, tid);
                            }
                        }
                    }
        }
        c->M[p] = M;
        c->Phi[p] = F;
        if (c->phid) c->phid[p] = fd;
    }
}

/* Range query for every hit point.  method 0: brute force over all photons;
 * method 1: plain uniform grid with cell edge >= the largest radius, visiting
 * the 27 neighbouring cells.  phid (optional) receives the double sums. */
static void gather_run(gather_ctx *cp, int method, int nthreads) {
    gather_ctx c = *cp;
    const orc_hitpoints *hp = c.hp;
    const orc_photons *ph = c.ph;
    const double *R2 = c.R2;
    int64_t n_hp = c.n_hp, n_ph = c.n_ph;
    if (method == 0 || n_ph == 0) {
        par_for(n_hp, nthreads, 16, gather_bf_range, &c);
        return;
    }
    double r2max = 0.0;
    for (int64_t p = 0; p < n_hp; ++p)
        if (hp->valid[p] && R2[p] > r2max) r2max = R2[p];
    double lo[3] = {INFINITY, INFINITY, INFINITY}, hi[3] = {-INFINITY, -INFINITY, -INFINITY};
    for (int64_t j = 0; j < n_ph; ++j)
        for (int a = 0; a < 3; ++a) {
            double x = ph->x[3 * j + a];
            if (x < lo[a]) lo[a] = x;
            if (x > hi[a]) hi[a] = x;
        }
    double ext = 0.0;
    for (int a = 0; a < 3; ++a) ext = fmax(ext, hi[a] - lo[a]);
    double h = 1.01 * sqrt(r2max);
    if (h < ext / 512.0) h = ext / 512.0;
    if (!(h > 0.0)) h = 1.0;
    c.h = h;
    int64_t ncell = 1;
    for (int a = 0; a < 3; ++a) {
        c.lo[a] = lo[a];
        c.dim[a] = (int64_t)floor((hi[a] - lo[a]) / h) + 1;
        ncell *= c.dim[a];
    }
    c.cell_start = (int64_t *)calloc((size_t)ncell + 1, sizeof(int64_t));
    c.order = (int64_t *)malloc(sizeof(int64_t) * (size_t)n_ph);
    int64_t *cid = (int64_t *)malloc(sizeof(int64_t) * (size_t)n_ph);
    for (int64_t j = 0; j < n_ph; ++j) {
        int64_t ci[3];
        cid[j] = cell_of(&c, ph->x + 3 * j, ci);
        c.cell_start[cid[j] + 1]++;
    }
    for (int64_t q = 0; q < ncell; ++q) c.cell_start[q + 1] += c.cell_start[q];
    int64_t *fill = (int64_t *)malloc(sizeof(int64_t) * (size_t)ncell);
    memcpy(fill, c.cell_start, sizeof(int64_t) * (size_t)ncell);
    for (int64_t j = 0; j < n_ph; ++j) c.order[fill[cid[j]]++] = j;
    free(fill);
    free(cid);
    par_for(n_hp, nthreads, 16, gather_grid_range, &c);
    free(c.cell_start);
    free(c.order);
}

ORC_EXPORT void orc_gather(const orc_hitpoints *hp, int64_t n_hp, const orc_photons *ph, int64_t n_ph, const double *R2,
                           int shift, int method, int nthreads, uint32_t *M, uint64_t *Phi, double *phid) {
    gather_ctx c;
    memset(&c, 0, sizeof(c));
    c.hp = hp; c.n_hp = n_hp; c.ph = ph; c.n_ph = n_ph; c.R2 = R2; c.shift = shift;
    c.M = M; c.Phi = Phi; c.phid = phid;
    gather_run(&c, method, nthreads);
}

/* ------------------------------------------------------------------------ */
/* Stochastic spatial hashing (Sec. 3.4): instead of listing every photon of */
/* a hash entry, only one photon per entry survives, and a hit point counts  */
/* that survivor once for every photon the entry received.  The survivor is */
/* decided by a z-buffer test on a random depth drawn independently for     */
/* each photon, so which photon survives does not depend on any property of */
/* its path (nor on the order of the writes).                                */
/*                                                                            */
/* Grid and table (the same for every method that hashes):                   */
/*   lo     per-axis minimum over the scene's vertices                       */
/*   h      2 sqrt(max R^2 over valid hit points) (1 + 2^-10), in double;    */
/*          inv_h = (float)(1/h) (0 when h = 0)                              */
/*   cell   floor((x - lo) * inv_h) per axis, in float32                     */
/*   entry  Teschner et al.'s hash of the cell mod 2^bits, bits the smallest */
/*          value in [12, 24] with 2^bits >= 4 n_photons                     */
/* A hit point's disc lies within the 2x2x2 cells whose lowest corner is    */
/* floor((x - lo) * inv_h - 0.5); each distinct entry of those is visited   */
/* once.  Depth of photon (path, bounce) in iteration k: the float bits of  */
/* the first output of stream (seed, DEPTH, k, path * 32 + bounce); the      */
/* smallest (depth, path * 32 + bounce) survives.                            */
/* ------------------------------------------------------------------------ */
static inline uint32_t teschner(int32_t ix, int32_t iy, int32_t iz, uint32_t mask) {
    uint32_t a = (uint32_t)ix * 73856093u, b = (uint32_t)iy * 19349663u, c = (uint32_t)iz * 83492791u;
    return (a ^ b ^ c) & mask;
}

static inline int32_t grid_coord(float x, float lo, float inv_h, float shift) {
    float f = (x - lo) * inv_h - shift;
    return (int32_t)floorf(f);
}

static uint32_t table_bits_for(int64_t n_photons) {
    uint32_t bits = 12;
    while (bits < 24 && ((int64_t)1 << bits) < 4 * n_photons) bits++;
    return bits;
}

ORC_EXPORT void orc_gather_stochastic(const orc_hitpoints *hp, int64_t n_hp, const orc_photons *ph, int64_t n_ph,
                                      const double *R2, int shift, const float *lo, int64_t n_photons_emitted,
                                      uint64_t seed, uint32_t k, uint32_t *M, uint64_t *Phi, uint32_t *n_entry_out) {
    double r2max = 0.0;
    for (int64_t p = 0; p < n_hp; ++p)
        if (hp->valid[p] && R2[p] > r2max) r2max = R2[p];
    double h = 2.0 * sqrt(r2max) * (1.0 + 1.0 / 1024.0);
    float inv_h = h > 0.0 ? (float)(1.0 / h) : 0.0f;
    uint32_t bits = table_bits_for(n_photons_emitted);
    uint32_t T = 1u << bits, mask = T - 1u;
    uint32_t *count = (uint32_t *)calloc(T, sizeof(uint32_t));
    uint64_t *best = (uint64_t *)malloc(sizeof(uint64_t) * T);
    int64_t *who = (int64_t *)malloc(sizeof(int64_t) * T);
    for (uint32_t e = 0; e < T; ++e) { best[e] = UINT64_MAX; who[e] = -1; }
    for (int64_t j = 0; j < n_ph; ++j) {
        const float *x = ph->x + 3 * j;
        uint32_t e = teschner(grid_coord(x[0], lo[0], inv_h, 0.0f), grid_coord(x[1], lo[1], inv_h, 0.0f),
                              grid_coord(x[2], lo[2], inv_h, 0.0f), mask);
        uint32_t id = ph->path[j] * 32u + ph->bounce[j];
        uint32_t st[4];
        rng_seed(seed, KIND_DEPTH, k, (uint64_t)id, st);
        float depth = rng_next(st);
        uint32_t dbits;
        memcpy(&dbits, &depth, 4);
        uint64_t key = ((uint64_t)dbits << 32) | (uint64_t)id;
        count[e]++;
        if (key < best[e]) { best[e] = key; who[e] = j; }
    }
    for (int64_t p = 0; p < n_hp; ++p) {
        uint32_t m = 0;
        uint64_t f = 0;
        if (hp->valid[p]) {
            const float *x = hp->x + 3 * p;
            int32_t b0 = grid_coord(x[0], lo[0], inv_h, 0.5f), b1 = grid_coord(x[1], lo[1], inv_h, 0.5f),
                    b2 = grid_coord(x[2], lo[2], inv_h, 0.5f);
            uint32_t visited[8];
            int nv = 0;
            for (int dz = 0; dz < 2; ++dz)
                for (int dy = 0; dy < 2; ++dy)
                    for (int dx = 0; dx < 2; ++dx) {
                        uint32_t e = teschner(b0 + dx, b1 + dy, b2 + dz, mask);
                        int seen = 0;
                        for (int v = 0; v < nv; ++v) seen |= (visited[v] == e);
                        if (seen) continue;
                        visited[nv++] = e;
                        if (count[e] == 0) continue;
                        int64_t j = who[e];
                        if (accept(x, hp->n + 3 * p, ph->x + 3 * j, ph->w + 3 * j, R2[p])) {
                            m += count[e];
                            f += (uint64_t)count[e] * fx_term(hp->wk[p], ph->phi[j], shift);
                        }
                    }
        }
        M[p] = m;
        Phi[p] = f;
    }
    if (n_entry_out) memcpy(n_entry_out, count, sizeof(uint32_t) * T);
    free(count);
    free(best);
    free(who);
}

static void scene_lo(const orc_scene *s, float lo[3]) {
    for (int a = 0; a < 3; ++a) lo[a] = INFINITY;
    for (int64_t i = 0; i < 9 * s->d.n_tri; ++i) {
        float v = s->d.verts[i];
        if (v < lo[i % 3]) lo[i % 3] = v;
    }
}

/* Progressive update of one pixel (radius reduction of stochastic
 * progressive photon mapping): with M new photons and fixed-point flux Phi,
 *   N' = N + alpha*M,  R2' = R2 * (N + alpha*M)/(N + M),
 *   tau' = (tau + Phi) * (N + alpha*M)/(N + M).
 * Nothing changes without a hit point or with M = 0. */
ORC_EXPORT void orc_update(int64_t n, const uint8_t *valid, const uint32_t *M, const uint64_t *Phi, double alpha,
                           int shift, double *N, double *R2, double *tau) {
    double scale = ldexp(1.0, -shift);
    for (int64_t p = 0; p < n; ++p) {
        if (!valid[p] || M[p] == 0) continue;
        double m = (double)M[p];
        double nn = N[p] + alpha * m;
        double ratio = nn / (N[p] + m);
        R2[p] = R2[p] * ratio;
        tau[p] = (tau[p] + (double)Phi[p] * scale) * ratio;
        N[p] = nn;
    }
}

/* Radiance estimate after K iterations: density estimate of the accumulated
 * flux over the current disc plus the average directly seen emission. */
ORC_EXPORT void orc_resolve(int64_t n, const double *R2, const double *tau, const double *D, int32_t K, float *img) {
    for (int64_t p = 0; p < n; ++p) {
        double L = tau[p] / ((PI_D * R2[p]) * (double)K) + D[p] / (double)K;
        img[p] = (float)L;
    }
}

/* ------------------------------------------------------------------------ */
/* Whole render: K iterations from the initial state.                          */
/* ------------------------------------------------------------------------ */
typedef struct {
    int64_t n_photons;
    double alpha;
    double r0;
    int32_t shift;
    int32_t gather_method; /* 0 brute force, 1 grid, 2 stochastic spatial hashing */
    int64_t photon_cap;
} orc_sppm_params;

typedef struct {
    double *N, *R2, *tau, *D; /* [P] state, caller-allocated */
    double *R2_hist;          /* optional [K][P]: radius used in iteration k */
    uint32_t *M_hist;         /* optional [K][P] */
    int64_t *n_stored;        /* optional [K] */
} orc_state;

static void hp_alloc(orc_hitpoints *hp, int64_t P) {
    hp->valid = (uint8_t *)calloc((size_t)P, 1);
    hp->x = (float *)malloc(sizeof(float) * 3 * (size_t)P);
    hp->n = (float *)malloc(sizeof(float) * 3 * (size_t)P);
    hp->wk = (float *)malloc(sizeof(float) * (size_t)P);
    hp->W = (float *)malloc(sizeof(float) * (size_t)P);
    hp->mat = (int32_t *)malloc(sizeof(int32_t) * (size_t)P);
    hp->tri = (int32_t *)malloc(sizeof(int32_t) * (size_t)P);
    hp->d_add = (double *)malloc(sizeof(double) * (size_t)P);
}

static void hp_free(orc_hitpoints *hp) {
    free(hp->valid); free(hp->x); free(hp->n); free(hp->wk); free(hp->W); free(hp->mat); free(hp->tri); free(hp->d_add);
}

static int ph_alloc(orc_photons *ph, int64_t cap, int with_mats) {
    ph->cap = cap;
    ph->x = (float *)malloc(sizeof(float) * 3 * (size_t)cap);
    ph->w = (float *)malloc(sizeof(float) * 3 * (size_t)cap);
    ph->phi = (float *)malloc(sizeof(float) * (size_t)cap);
    ph->path = (uint32_t *)malloc(sizeof(uint32_t) * (size_t)cap);
    ph->bounce = (uint32_t *)malloc(sizeof(uint32_t) * (size_t)cap);
    ph->mats = with_mats ? (int32_t *)malloc(sizeof(int32_t) * 32 * (size_t)cap) : NULL;
    return ph->x && ph->w && ph->phi && ph->path && ph->bounce;
}

static void ph_free(orc_photons *ph) {
    free(ph->x); free(ph->w); free(ph->phi); free(ph->path); free(ph->bounce); free(ph->mats);
}

/* Runs iterations k0 .. k0+K-1 on the given state (which the caller
 * initialises: N=0, R2=r0^2, tau=0, D=0).  Returns 0, or -1 on photon-store
 * overflow. */
ORC_EXPORT int orc_sppm_run(const orc_scene *s, const orc_run_opts *op, const orc_sppm_params *pp, int32_t k0, int32_t K,
                            orc_state *st) {
    int64_t P = (int64_t)s->d.width * s->d.height;
    orc_hitpoints hp;
    hp_alloc(&hp, P);
    orc_photons ph;
    ph_alloc(&ph, pp->photon_cap, 0);
    uint32_t *M = (uint32_t *)malloc(sizeof(uint32_t) * (size_t)P);
    uint64_t *Phi = (uint64_t *)malloc(sizeof(uint64_t) * (size_t)P);
    int rc = 0;
    for (int32_t it = 0; it < K; ++it) {
        uint32_t k = (uint32_t)(k0 + it);
        orc_eye_pass(s, op, k, &hp);
        int64_t n = orc_photon_pass(s, op, k, pp->n_photons, NULL, pp->n_photons, &ph);
        if (n < 0) { rc = -1; break; }
        if (st->n_stored) st->n_stored[it] = n;
        if (st->R2_hist) memcpy(st->R2_hist + (size_t)it * P, st->R2, sizeof(double) * (size_t)P);
        if (pp->gather_method == 2) {
            float lo[3];
            scene_lo(s, lo);
            orc_gather_stochastic(&hp, P, &ph, n, st->R2, pp->shift, lo, pp->n_photons, op->seed, k, M, Phi, NULL);
        } else {
            orc_gather(&hp, P, &ph, n, st->R2, pp->shift, pp->gather_method, op->nthreads, M, Phi, NULL);
        }
        if (st->M_hist) memcpy(st->M_hist + (size_t)it * P, M, sizeof(uint32_t) * (size_t)P);
        orc_update(P, hp.valid, M, Phi, pp->alpha, pp->shift, st->N, st->R2, st->tau);
        for (int64_t p = 0; p < P; ++p) st->D[p] += hp.d_add[p];
    }
    free(M);
    free(Phi);
    ph_free(&ph);
    hp_free(&hp);
    return rc;
}

/* ------------------------------------------------------------------------ */
/* Forward-mode gradient of an image loss.                                    */
/*                                                                            */
/* With sampling held fixed (Russian roulette uses the nominal albedo q, so   */
/* every path, hit point and radius is independent of the parameters), the   */
/* accumulated flux telescopes:  L_p = sum_k Phi_{p,k} / (pi R2_{p,k} K)       */
/* + D_p / K, where R2_{p,k} is the radius used in iteration k.  Each term is */
/* linear in the emitted radiance and a monomial in the albedos, so the      */
/* derivative is summed contribution by contribution.                         */
/*                                                                            */
/* g: [P] dloss/dL_p.  pmat: [n_par] material ids of the albedo parameters.   */
/* grad: [n_par + 1] = dloss/drho_m for each parameter, then dloss/dLe of the  */
/* single emitting material (0 if there is none).  img: optional [P] image.   */
/* ------------------------------------------------------------------------ */
ORC_EXPORT int orc_sppm_grad(const orc_scene *s, const orc_run_opts *op, const orc_sppm_params *pp, int32_t K,
                             const double *g, const int32_t *pmat, int32_t n_par, double *grad, float *img) {
    int64_t P = (int64_t)s->d.width * s->d.height;
    double *N = (double *)calloc((size_t)P, sizeof(double));
    double *R2 = (double *)malloc(sizeof(double) * (size_t)P);
    double *tau = (double *)calloc((size_t)P, sizeof(double));
    double *D = (double *)calloc((size_t)P, sizeof(double));
    double *gw = (double *)malloc(sizeof(double) * (size_t)P);
    for (int64_t p = 0; p < P; ++p) R2[p] = pp->r0 * pp->r0;
    orc_hitpoints hp;
    hp_alloc(&hp, P);
    orc_photons ph;
    ph_alloc(&ph, pp->photon_cap, 1);
    uint32_t *M = (uint32_t *)malloc(sizeof(uint32_t) * (size_t)P);
    uint64_t *Phi = (uint64_t *)malloc(sizeof(uint64_t) * (size_t)P);
    int nth = op->nthreads < 1 ? 1 : (op->nthreads > 256 ? 256 : op->nthreads);
    double *acc = (double *)calloc((size_t)nth * (size_t)(n_par > 0 ? n_par : 1), sizeof(double));
    int rc = 0;
    for (int32_t k = 0; k < K; ++k) {
        orc_eye_pass(s, op, (uint32_t)k, &hp);
        int64_t n = orc_photon_pass(s, op, (uint32_t)k, pp->n_photons, NULL, pp->n_photons, &ph);
        if (n < 0) { rc = -1; break; }
        for (int64_t p = 0; p < P; ++p) gw[p] = g[p] / ((PI_D * R2[p]) * (double)K);
        gather_ctx c;
        memset(&c, 0, sizeof(c));
        c.hp = &hp; c.n_hp = P; c.ph = &ph; c.n_ph = n; c.R2 = R2; c.shift = pp->shift;
        c.M = M; c.Phi = Phi;
        c.gw = gw; c.rho = s->d.mat_rho; c.pmat = pmat; c.n_par = n_par; c.acc = acc;
        gather_run(&c, pp->gather_method, nth);
        orc_update(P, hp.valid, M, Phi, pp->alpha, pp->shift, N, R2, tau);
        for (int64_t p = 0; p < P; ++p) D[p] += hp.d_add[p];
    }
    for (int i = 0; i < n_par; ++i) {
        double a = 0.0;
        for (int t = 0; t < nth; ++t) a += acc[(size_t)t * n_par + i];
        grad[i] = a;
    }
    /* emission: every term of L_p is proportional to Le */
    int32_t em = -1, n_em = 0;
    for (int32_t m = 0; m < s->d.n_mat; ++m)
        if (s->d.mat_Le[m] > 0.0f) { em = m; n_em++; }
    double gl = 0.0;
    for (int64_t p = 0; p < P; ++p) {
        double L = tau[p] / ((PI_D * R2[p]) * (double)K) + D[p] / (double)K;
        if (img) img[p] = (float)L;
        gl += g[p] * L;
    }
    grad[n_par] = (n_em == 1) ? gl / (double)s->d.mat_Le[em] : 0.0;
    free(N); free(R2); free(tau); free(D); free(gw); free(M); free(Phi); free(acc);
    ph_free(&ph);
    hp_free(&hp);
    return rc;
}
